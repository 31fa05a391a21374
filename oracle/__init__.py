"""CPU oracle for the Custom Correlation Coefficient tallies.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke``
and by the CPU-baseline leg of ``bench.py``.  The GPU library
(``paper_1705_08213_amd``) never imports this package and shares no code with
it.

``ccc_oracle.c`` holds the definitions as plain loops (see its header for the
equations, Sec. 2.1-2.2, and the readings taken for missing data);
``brute.py`` holds a literal allele-pair enumerator and the paper's 3-way
decomposition (Table 1 and the mapping identities of Sec. 3.2), used to pin
the C code.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# CCC_ORACLE_LIB points the tests' mutation check at a deliberately broken copy.
_SO = os.environ.get("CCC_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "ccc_oracle.c")

GAMMA = 2.0 / 3.0


def build() -> None:
    """Compile liboracle.so (plain C, -O2, OpenMP, no intrinsics)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11", _SRC, "-o", _SO]
    subprocess.run(cmd, check=True)


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, dbl, ptr, cint = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        lib.oracle_counts1.argtypes = [ptr, i64, i64, i64, ptr]
        lib.oracle_2way_rows.argtypes = [ptr, i64, i64, i64, i64, i64, ptr, dbl, ptr, ptr]
        lib.oracle_3way_rows.argtypes = [ptr, i64, i64, i64, i64, i64, ptr, dbl, ptr, ptr]
        lib.oracle_block_rows.argtypes = [ptr, i64, ptr, i64, i64, i64, i64, i64, ptr, ptr,
                                          dbl, ptr, ptr]
        lib.oracle_2way_list.argtypes = [ptr, i64, ptr, i64, i64, ptr, ptr, i64, ptr, ptr, dbl,
                                         ptr, ptr]
        lib.oracle_3way_list.argtypes = [ptr, i64, i64, ptr, ptr, ptr, i64, ptr, dbl, ptr, ptr]
        lib.oracle_fp2_from_input.argtypes = [ptr, i64, i64, i64, ptr, ptr, ptr]
        lib.oracle_fp2_from_tables.argtypes = [ptr, i64, ptr, ptr, ptr]
        lib.oracle_fpb_from_input.argtypes = [ptr, i64, i64, ptr, i64, i64, i64, ptr, ptr, ptr]
        lib.oracle_fpb_from_tables.argtypes = [ptr, i64, i64, ptr, ptr, ptr]
        lib.oracle_fp3_from_input.argtypes = [ptr, i64, i64, i64, ptr, ptr, ptr, ptr]
        lib.oracle_fp3_from_tables.argtypes = [ptr, i64, i64, i64, ptr, ptr, ptr, ptr]
        lib.oracle_pair_index.argtypes = [i64, i64, i64]
        lib.oracle_pair_index.restype = i64
        lib.oracle_triple_index.argtypes = [i64, i64, i64, i64]
        lib.oracle_triple_index.restype = i64
        lib.oracle_multi_invalid.argtypes = [ptr, i64, i64, i64, cint]
        lib.oracle_multi_invalid.restype = i64
        lib.oracle_multi_counts1.argtypes = [ptr, i64, i64, i64, cint, ptr]
        lib.oracle_multi_2way_rows.argtypes = [ptr, i64, i64, i64, cint, i64, i64, ptr, dbl, ptr,
                                               ptr]
        lib.oracle_multi_2way_list.argtypes = [ptr, i64, i64, cint, ptr, ptr, i64, ptr, dbl, ptr,
                                               ptr]
        lib.oracle_multi_fp2_from_input.argtypes = [ptr, i64, i64, i64, cint, ptr, ptr, ptr]
        lib.oracle_multi_fp2_from_tables.argtypes = [ptr, i64, cint, ptr, ptr, ptr]
        lib.oracle_num_threads.restype = cint
        lib.oracle_set_num_threads.argtypes = [cint]
        _lib_handle = lib
    return _lib_handle


def _c(a: np.ndarray, dtype) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def num_threads() -> int:
    return _lib().oracle_num_threads()


def set_num_threads(n: int) -> None:
    _lib().oracle_set_num_threads(n)


def pair_index(n, i, j) -> int:
    return _lib().oracle_pair_index(n, i, j)


def triple_index(n, i, j, k) -> int:
    return _lib().oracle_triple_index(n, i, j, k)


def n_pairs(n: int) -> int:
    return n * (n - 1) // 2 if n >= 2 else 0


def n_triples(n: int) -> int:
    return n * (n - 1) * (n - 2) // 6 if n >= 3 else 0


def counts1(v: np.ndarray, n_f: int) -> np.ndarray:
    """int64 [n_v, 3]: n_i(0), n_i(1), m_i."""
    v = _c(v, np.uint8)
    out = np.zeros((v.shape[0], 3), dtype=np.int64)
    if v.shape[0]:
        _lib().oracle_counts1(v.ctypes.data, v.shape[0], n_f, v.shape[1], out.ctypes.data)
    return out


def two_way(v, n_f, i0=0, i1=None, gamma=GAMMA, with_ccc=True):
    """Tables int64 [P, 4] and CCC double [P, 4] for the pairs whose first index
    lies in [i0, i1) (all pairs by default), in lexicographic order."""
    v = _c(v, np.uint8)
    n_v, ld = v.shape
    i1 = n_v if i1 is None else min(i1, n_v)
    i1 = min(i1, max(n_v - 1, 0))
    if i0 >= i1:
        return np.zeros((0, 4), np.int64), np.zeros((0, 4), np.float64)
    npair = pair_index(n_v, i1 - 1, n_v - 1) + 1 - pair_index(n_v, i0, i0 + 1)
    tables = np.zeros((npair, 4), dtype=np.int64)
    ccc = np.zeros((npair, 4), dtype=np.float64) if with_ccc else None
    cnt = counts1(v, n_f)
    _lib().oracle_2way_rows(v.ctypes.data, n_v, n_f, ld, i0, i1, cnt.ctypes.data, gamma,
                            tables.ctypes.data, ccc.ctypes.data if with_ccc else None)
    return tables, ccc


def three_way(v, n_f, i0=0, i1=None, gamma=GAMMA, with_ccc=True):
    """Tables int64 [T, 8] and CCC double [T, 8] for the triples whose first
    index lies in [i0, i1), in lexicographic order."""
    v = _c(v, np.uint8)
    n_v, ld = v.shape
    i1 = n_v if i1 is None else min(i1, n_v)
    i1 = min(i1, max(n_v - 2, 0))
    if i0 >= i1:
        return np.zeros((0, 8), np.int64), np.zeros((0, 8), np.float64)
    ntri = triple_index(n_v, i1 - 1, n_v - 2, n_v - 1) + 1 - triple_index(n_v, i0, i0 + 1,
                                                                             i0 + 2)
    tables = np.zeros((ntri, 8), dtype=np.int64)
    ccc = np.zeros((ntri, 8), dtype=np.float64) if with_ccc else None
    cnt = counts1(v, n_f)
    _lib().oracle_3way_rows(v.ctypes.data, n_v, n_f, ld, i0, i1, cnt.ctypes.data, gamma,
                            tables.ctypes.data, ccc.ctypes.data if with_ccc else None)
    return tables, ccc


def block(va, vb, n_f, a0=0, a1=None, gamma=GAMMA, with_ccc=True):
    """Tables int64 [a1-a0, n_b, 4] and CCC for rows [a0, a1) of A against all
    of B.  ``va``/``vb`` are 2-D uint8 arrays, or (array, n_f_total) views of
    the same fields."""
    va = _c(va, np.uint8)
    vb = _c(vb, np.uint8)
    n_a, lda = va.shape
    n_b, ldb = vb.shape
    a1 = n_a if a1 is None else min(a1, n_a)
    rows = max(a1 - a0, 0)
    tables = np.zeros((rows, n_b, 4), dtype=np.int64)
    ccc = np.zeros((rows, n_b, 4), dtype=np.float64) if with_ccc else None
    if rows and n_b:
        ca = counts1(va, n_f)
        cb = counts1(vb, n_f)
        _lib().oracle_block_rows(va.ctypes.data, lda, vb.ctypes.data, n_b, ldb, n_f, a0, a1,
                                 ca.ctypes.data, cb.ctypes.data, gamma, tables.ctypes.data,
                                 ccc.ctypes.data if with_ccc else None)
    return tables, ccc


def pairs_list(va, vb, n_f, ia, jb, gamma=GAMMA, counts_a=None, counts_b=None):
    """Tables int64 [np, 4] and CCC [np, 4] for explicit pairs (ia[p] of A,
    jb[p] of B); pass the same array as A and B for pairs of one set."""
    va = _c(va, np.uint8)
    vb = _c(vb, np.uint8)
    ia = _c(ia, np.int64)
    jb = _c(jb, np.int64)
    ca = counts1(va, n_f) if counts_a is None else _c(counts_a, np.int64)
    cb = (ca if vb is va else counts1(vb, n_f)) if counts_b is None else _c(counts_b, np.int64)
    tables = np.zeros((len(ia), 4), dtype=np.int64)
    ccc = np.zeros((len(ia), 4), dtype=np.float64)
    if len(ia):
        _lib().oracle_2way_list(va.ctypes.data, va.shape[1], vb.ctypes.data, vb.shape[1], n_f,
                                ia.ctypes.data, jb.ctypes.data, len(ia), ca.ctypes.data,
                                cb.ctypes.data, gamma, tables.ctypes.data, ccc.ctypes.data)
    return tables, ccc


def triples_list(v, n_f, ii, jj, kk, gamma=GAMMA, counts=None):
    """Tables int64 [np, 8] and CCC [np, 8] for explicit triples."""
    v = _c(v, np.uint8)
    ii, jj, kk = (_c(x, np.int64) for x in (ii, jj, kk))
    cnt = counts1(v, n_f) if counts is None else _c(counts, np.int64)
    tables = np.zeros((len(ii), 8), dtype=np.int64)
    ccc = np.zeros((len(ii), 8), dtype=np.float64)
    if len(ii):
        _lib().oracle_3way_list(v.ctypes.data, v.shape[1], n_f, ii.ctypes.data, jj.ctypes.data,
                                kk.ctypes.data, len(ii), cnt.ctypes.data, gamma,
                                tables.ctypes.data, ccc.ctypes.data)
    return tables, ccc


def fp2_from_input(v, n_f, w, u) -> np.ndarray:
    v = _c(v, np.uint8)
    out = np.zeros(4, dtype=np.uint64)
    _lib().oracle_fp2_from_input(v.ctypes.data, v.shape[0], n_f, v.shape[1],
                                 _c(w, np.uint64).ctypes.data, _c(u, np.uint64).ctypes.data,
                                 out.ctypes.data)
    return out


def fp2_from_tables(tables_i32, n_v, w, u) -> np.ndarray:
    t = _c(tables_i32, np.int32)
    assert t.size == 4 * n_pairs(n_v)
    out = np.zeros(4, dtype=np.uint64)
    _lib().oracle_fp2_from_tables(t.ctypes.data, n_v, _c(w, np.uint64).ctypes.data,
                                  _c(u, np.uint64).ctypes.data, out.ctypes.data)
    return out


def fpb_from_input(va, vb, n_f, w, u) -> np.ndarray:
    va = _c(va, np.uint8)
    vb = _c(vb, np.uint8)
    out = np.zeros(4, dtype=np.uint64)
    _lib().oracle_fpb_from_input(va.ctypes.data, va.shape[0], va.shape[1], vb.ctypes.data,
                                 vb.shape[0], vb.shape[1], n_f, _c(w, np.uint64).ctypes.data,
                                 _c(u, np.uint64).ctypes.data, out.ctypes.data)
    return out


def fpb_from_tables(tables_i32, n_a, n_b, w, u) -> np.ndarray:
    t = _c(tables_i32, np.int32)
    assert t.size == 4 * n_a * n_b
    out = np.zeros(4, dtype=np.uint64)
    _lib().oracle_fpb_from_tables(t.ctypes.data, n_a, n_b, _c(w, np.uint64).ctypes.data,
                                  _c(u, np.uint64).ctypes.data, out.ctypes.data)
    return out


def fp3_from_input(v, n_f, w, u, z) -> np.ndarray:
    v = _c(v, np.uint8)
    out = np.zeros(8, dtype=np.uint64)
    _lib().oracle_fp3_from_input(v.ctypes.data, v.shape[0], n_f, v.shape[1],
                                 _c(w, np.uint64).ctypes.data, _c(u, np.uint64).ctypes.data,
                                 _c(z, np.uint64).ctypes.data, out.ctypes.data)
    return out


def fp3_from_tables(tables_i32, n_v, w, u, z, t_begin=0) -> np.ndarray:
    """Checksum contribution of a slice of triple tables starting at
    lexicographic index ``t_begin``; slices add up mod 2^61-1."""
    t = _c(tables_i32, np.int32)
    n_t = t.size // 8
    out = np.zeros(8, dtype=np.uint64)
    _lib().oracle_fp3_from_tables(t.ctypes.data, n_v, t_begin, n_t,
                                  _c(w, np.uint64).ctypes.data, _c(u, np.uint64).ctypes.data,
                                  _c(z, np.uint64).ctypes.data, out.ctypes.data)
    return out


P61 = (1 << 61) - 1


def fp_add(a, b) -> np.ndarray:
    """Element-wise (a + b) mod 2^61-1 for checksum vectors."""
    return np.array([(int(x) + int(y)) % P61 for x, y in zip(a, b)], dtype=np.uint64)


# ---------------------------------------------------------------------------
# Multi-allelic 2-way CCC (s states per marker, one byte per field; see the
# multi-allelic section of ccc_oracle.c).
# ---------------------------------------------------------------------------

def multi_invalid(v, n_f, s) -> int:
    """Number of entries that are neither a genotype over the first s states
    nor the missing byte 0."""
    v = _c(v, np.uint8)
    return int(_lib().oracle_multi_invalid(v.ctypes.data, v.shape[0], n_f, v.shape[1], s))


def multi_counts1(v, n_f, s) -> np.ndarray:
    """int64 [n_v, 5]: n_i(0..3) (0 for states >= s) and m_i."""
    v = _c(v, np.uint8)
    out = np.zeros((v.shape[0], 5), dtype=np.int64)
    if v.shape[0]:
        _lib().oracle_multi_counts1(v.ctypes.data, v.shape[0], n_f, v.shape[1], s,
                                    out.ctypes.data)
    return out


def multi_two_way(v, n_f, s, i0=0, i1=None, gamma=GAMMA, with_ccc=True):
    """Tables int64 [P, s*s] and CCC double [P, s*s] (entry a*s + b) for the
    pairs whose first index lies in [i0, i1), in lexicographic order."""
    v = _c(v, np.uint8)
    n_v, ld = v.shape
    ss = s * s
    i1 = n_v if i1 is None else min(i1, n_v)
    i1 = min(i1, max(n_v - 1, 0))
    if i0 >= i1:
        return np.zeros((0, ss), np.int64), np.zeros((0, ss), np.float64)
    npair = pair_index(n_v, i1 - 1, n_v - 1) + 1 - pair_index(n_v, i0, i0 + 1)
    tables = np.zeros((npair, ss), dtype=np.int64)
    ccc = np.zeros((npair, ss), dtype=np.float64) if with_ccc else None
    cnt = multi_counts1(v, n_f, s)
    _lib().oracle_multi_2way_rows(v.ctypes.data, n_v, n_f, ld, s, i0, i1, cnt.ctypes.data, gamma,
                                  tables.ctypes.data, ccc.ctypes.data if with_ccc else None)
    return tables, ccc


def multi_pairs_list(v, n_f, s, ia, jb, gamma=GAMMA):
    """Tables int64 [np, s*s] and CCC double [np, s*s] of the pairs (ia[p], jb[p])."""
    v = _c(v, np.uint8)
    ia = _c(ia, np.int64)
    jb = _c(jb, np.int64)
    ss = s * s
    tables = np.zeros((len(ia), ss), dtype=np.int64)
    ccc = np.zeros((len(ia), ss), dtype=np.float64)
    cnt = multi_counts1(v, n_f, s)
    if len(ia):
        _lib().oracle_multi_2way_list(v.ctypes.data, v.shape[1], n_f, s, ia.ctypes.data,
                                      jb.ctypes.data, len(ia), cnt.ctypes.data, gamma,
                                      tables.ctypes.data, ccc.ctypes.data)
    return tables, ccc


def multi_fp2_from_input(v, n_f, s, w, u) -> np.ndarray:
    v = _c(v, np.uint8)
    out = np.zeros(s * s, dtype=np.uint64)
    _lib().oracle_multi_fp2_from_input(v.ctypes.data, v.shape[0], n_f, v.shape[1], s,
                                       _c(w, np.uint64).ctypes.data, _c(u, np.uint64).ctypes.data,
                                       out.ctypes.data)
    return out


def multi_fp2_from_tables(tables, n_v, s, w, u) -> np.ndarray:
    t = _c(tables, np.int32)
    out = np.zeros(s * s, dtype=np.uint64)
    _lib().oracle_multi_fp2_from_tables(t.ctypes.data, n_v, s, _c(w, np.uint64).ctypes.data,
                                        _c(u, np.uint64).ctypes.data, out.ctypes.data)
    return out
