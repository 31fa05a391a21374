"""Mutation check of the oracle's pins.

Each case copies oracle/ccc_oracle.c, plants one plausible mistake (a dropped
term, a wrong index or sign, a swapped operand, a wrong normaliser), builds it
on the CPU and runs the pin suites (biallelic and multi-allelic) against it in
a subprocess: at least one pin
must fail for every mutant, and the unmodified copy must pass.  The oracle
sources are not modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ccc_oracle.c")

# (name, text to find, replacement) -- each applied to the first occurrence
MUTANTS = [
    ("rho counts one allele", "return (r1 == a) + (r2 == a);", "return (r1 == a);"),
    ("missing treated as het", "static inline int is_missing(unsigned code) { return code == 2u; }",
     "static inline int is_missing(unsigned code) { return 0; }"),
    ("wrong missing code", "return code == 2u;", "return code == 1u;"),
    ("allele bits swapped in rho", "int r1 = (int)((code >> 1) & 1u), r2 = (int)(code & 1u);",
     "int r1 = (int)((code >> 1) & 1u), r2 = (int)((code >> 1) & 1u);"),
    ("2-way table order b,a", "t[2 * a + b] += (int64_t)rho(ci, a) * rho(cj, b);",
     "t[2 * b + a] += (int64_t)rho(ci, a) * rho(cj, b);"),
    ("f_i normaliser n_f-free 2m", "return m > 0 ? (double)n_a / (2.0 * (double)m) : 0.0;",
     "return m > 0 ? (double)n_a / (1.0 * (double)m) : 0.0;"),
    ("f_ij uses 2 m_ij", "double f_ij = (double)t[2 * a + b] / (4.0 * (double)m_ij);",
     "double f_ij = (double)t[2 * a + b] / (2.0 * (double)m_ij);"),
    ("frequency index swapped", "double fi = freq1(ci[a], ci[2]);", "double fi = freq1(ci[1 - a], ci[2]);"),
    ("dropped (1 - g f_j) factor", "val = f_ij * (1.0 - gamma * fi) * (1.0 - gamma * fj);",
     "val = f_ij * (1.0 - gamma * fi);"),
    ("sign of gamma term", "val = f_ij * (1.0 - gamma * fi) * (1.0 - gamma * fj);",
     "val = f_ij * (1.0 + gamma * fi) * (1.0 - gamma * fj);"),
    ("m_ij from sum/2", "int64_t m_ij = sum / 4;", "int64_t m_ij = sum / 2;"),
    ("3-way drops the k factor", "t[4 * a + 2 * b + c] += (int64_t)rho(ci, a) * rho(cj, b) * rho(ck, c);",
     "t[4 * a + 2 * b + c] += (int64_t)rho(ci, a) * rho(cj, b);"),
    ("3-way k uses j's row", "const uint8_t* rk = v + k * ld;", "const uint8_t* rk = v + j * ld;"),
    ("3-way entry order", "out[4 * a + 2 * b + c] = val;", "out[4 * c + 2 * b + a] = val;"),
    ("3-way m from sum/4", "int64_t m_ijk = sum / 8;", "int64_t m_ijk = sum / 4;"),
    ("pair index off by one", "return i * n - i * (i + 1) / 2 + (j - i - 1);",
     "return i * n - i * (i + 1) / 2 + (j - i);"),
    ("field decode shift", "return (row[q >> 2] >> (2 * (q & 3))) & 3u;",
     "return (row[q >> 2] >> (q & 3)) & 3u;"),
    ("counts miss the n(1) term", "n1 += rho(c, 1);", "n1 += rho(c, 0);"),
    ("checksum prefix excludes w", "pre[a][q - q0] = addmod(pre[a][q - q0], mulmod(w[j], (uint64_t)rho(c, a)));",
     "pre[a][q - q0] = addmod(pre[a][q - q0], mulmod(u[j], (uint64_t)rho(c, a)));"),
    # multi-allelic section
    ("multi state field shift", "return (byte >> (2 * a)) & 3;", "return (byte >> a) & 3;"),
    ("multi one copy counts as present", "return total == 2;", "return total >= 1;"),
    ("multi table order b,a", "t[a * s + b] += (int64_t)mrho(bi, a) * mrho(bj, b);",
     "t[b * s + a] += (int64_t)mrho(bi, a) * mrho(bj, b);"),
    ("multi f_j normaliser index", "double fj = freq1(cj[b], cj[4]);",
     "double fj = freq1(cj[b], cj[3]);"),
    ("multi m_ij from sum/2", "for (int e = 0; e < s * s; ++e) sum += t[e];\n  int64_t m_ij = sum / 4;",
     "for (int e = 0; e < s * s; ++e) sum += t[e];\n  int64_t m_ij = sum / 2;"),
    ("multi counts include missing", "if (!mpresent(b, s)) continue;\n      ++m;", "++m;"),
    ("multi checksum prefix uses u",
     "pre[x][q - q0] = addmod(pre[x][q - q0], mulmod(w[j], (uint64_t)mrho(b, x)));",
     "pre[x][q - q0] = addmod(pre[x][q - q0], mulmod(u[j], (uint64_t)mrho(b, x)));"),
]

PIN_TESTS = [os.path.join(ROOT, "tests", "test_oracle_pins.py"),
             os.path.join(ROOT, "tests", "test_oracle_multi_pins.py")]


def build_variant(tmp_path, name, find, repl):
    text = open(SRC).read()
    if find is not None:
        assert find in text, f"mutation anchor for {name!r} not found"
        text = text.replace(find, repl, 1)
    src = tmp_path / "oracle_variant.c"
    src.write_text(text)
    so = tmp_path / "liboracle_variant.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", str(src), "-o",
                    str(so)], check=True)
    return str(so)


def run_pins(so):
    env = dict(os.environ, CCC_ORACLE_LIB=so, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *PIN_TESTS], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    return r.returncode, r.stdout[-400:]


def test_unmodified_copy_passes(tmp_path):
    rc, out = run_pins(build_variant(tmp_path, "none", None, None))
    assert rc == 0, out


@pytest.mark.parametrize("name,find,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_every_planted_mistake_fails_a_pin(tmp_path, name, find, repl):
    rc, out = run_pins(build_variant(tmp_path, name, find, repl))
    assert rc != 0, f"no pin caught the mutant {name!r}"
