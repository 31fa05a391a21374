"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: each test reaches the expected
result by another route -- the literal allele enumeration of the worked
examples (Sec. 2.1/2.2), the paper's own 3-way construction (Table 1 and the
mapping identities of Sec. 3.2), a float64 BLAS product (exact for these
integers), closed forms, or invariants the paper states.
"""
import itertools
import math
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G = 2.0 / 3.0


def codes_to_packed(codes, pad_value=-1):
    return synth.pack_codes(np.asarray(codes, dtype=np.uint8), pad_value=pad_value)


# ---------------------------------------------------------------------------
# Table 1 (Sec. 3.2) as printed.
# ---------------------------------------------------------------------------

def _pair(s):
    a, b = s.split(",")
    return (int(a), int(b))


def test_table1_x_matrix_rule_matches_printed_table():
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "table1_xjxi.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 9
    for row in rows:
        v, vj, x1, x2, x3 = map(_pair, row)
        for xi, want in zip((1, 2, 3), (x1, x2, x3)):
            assert brute.x_entry(v, vj, xi, missing_aware=False) == want, (row, xi)


# ---------------------------------------------------------------------------
# Exhaustive tiny inputs vs the literal enumeration of Figs. 1-2.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n_v,n_f", [(2, 1), (2, 2), (2, 3), (3, 2)])
def test_2way_exhaustive_vs_literal_enumeration(n_v, n_f):
    for flat in itertools.product(range(4), repeat=n_v * n_f):
        codes = np.array(flat, dtype=np.uint8).reshape(n_v, n_f)
        v = codes_to_packed(codes)
        got, _ = oracle.two_way(v, n_f, with_ccc=False)
        want = brute.all_pairs(codes)
        assert np.array_equal(got, want), codes


@pytest.mark.parametrize("n_v,n_f", [(3, 1), (3, 2), (4, 1)])
def test_3way_exhaustive_vs_literal_enumeration(n_v, n_f):
    for flat in itertools.product(range(4), repeat=n_v * n_f):
        codes = np.array(flat, dtype=np.uint8).reshape(n_v, n_f)
        v = codes_to_packed(codes)
        got, _ = oracle.three_way(v, n_f, with_ccc=False)
        want = brute.all_triples(codes)
        assert np.array_equal(got, want), codes


def test_1way_exhaustive_single_entries():
    # rho(a) per code: 00 -> (2,0), 01 -> (1,1), 11 -> (0,2), 10 -> missing.
    want = {0: (2, 0, 1), 1: (1, 1, 1), 3: (0, 2, 1), 2: (0, 0, 0)}
    codes = np.array([[0], [1], [2], [3]], dtype=np.uint8)
    c = oracle.counts1(codes_to_packed(codes), 1)
    for row, code in zip(c, (0, 1, 2, 3)):
        assert tuple(row) == want[code]


# ---------------------------------------------------------------------------
# The paper's 3-way construction (Table 1 + mapping identities).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("missing", [0.0, 0.2])
def test_3way_matches_paper_x_decomposition(missing):
    n_v, n_f = 6, 23
    v = synth.uniform(n_v, n_f, seed=11, missing=missing)
    codes = brute.unpack_codes(v, n_f)
    got, _ = oracle.three_way(v, n_f, with_ccc=False)
    want = brute.tally3_via_x(codes, missing_aware=True)
    assert np.array_equal(got, want)


def test_3way_x_decomposition_without_missing_folds_10_into_01():
    # With no missing data the paper treats (1,0) like (0,1); the oracle's
    # missing reading differs only where code 10 occurs, so use codes {0,1,3}.
    rng = np.random.default_rng(5)
    codes = rng.choice(np.array([0, 1, 3], dtype=np.uint8), size=(5, 17))
    v = codes_to_packed(codes)
    got, _ = oracle.three_way(v, 17, with_ccc=False)
    assert np.array_equal(got, brute.tally3_via_x(codes, missing_aware=False))


# ---------------------------------------------------------------------------
# Float64 BLAS reduction: C(a,b) = R_a R_b^T (exact: integers < 2^53).
# ---------------------------------------------------------------------------

def rho_matrices(v, n_f):
    """R_a [n_v, n_f] built from the literal allele pairs of brute.py."""
    codes = brute.unpack_codes(v, n_f)
    tab = np.zeros((2, 4))
    for code in range(4):
        e = brute.allele_pair(code)
        if e == brute.MISSING:
            continue
        for a in range(2):
            tab[a, code] = sum(1 for x in e if x == a)
    return tab[0][codes], tab[1][codes]


@pytest.mark.parametrize("gen", ["uniform", "beta_hw"])
def test_2way_vs_float64_gemm(gen):
    n_v, n_f = 150, 3001
    f = synth.uniform if gen == "uniform" else synth.beta_hw
    v = f(n_v, n_f, seed=3, missing=0.05)
    R = rho_matrices(v, n_f)
    got, _ = oracle.two_way(v, n_f, with_ccc=False)
    iu = np.triu_indices(n_v, 1)
    for a in range(2):
        for b in range(2):
            full = R[a] @ R[b].T
            assert np.array_equal(got[:, 2 * a + b], full[iu].astype(np.int64))


def test_3way_vs_float64_gemm_per_j():
    n_v, n_f = 24, 777
    v = synth.beta_hw(n_v, n_f, seed=4, missing=0.05)
    R = rho_matrices(v, n_f)
    got, _ = oracle.three_way(v, n_f, with_ccc=False)
    for i, j, k in [(0, 1, 2), (0, 5, 23), (3, 11, 12), (21, 22, 23), (7, 8, 20)]:
        p = oracle.triple_index(n_v, i, j, k)
        for a in range(2):
            for b in range(2):
                for c in range(2):
                    m = R[a] @ (R[b][j][None, :] * R[c]).T
                    assert got[p, 4 * a + 2 * b + c] == int(m[i, k])


def test_block_vs_float64_gemm():
    va = synth.beta_hw(37, 999, seed=5, missing=0.02)
    vb = synth.beta_hw(41, 999, seed=6, missing=0.02)
    Ra, Rb = rho_matrices(va, 999), rho_matrices(vb, 999)
    got, _ = oracle.block(va, vb, 999, with_ccc=False)
    for a in range(2):
        for b in range(2):
            assert np.array_equal(got[:, :, 2 * a + b], (Ra[a] @ Rb[b].T).astype(np.int64))


# ---------------------------------------------------------------------------
# Invariants stated by the paper (Sec. 2.1-2.2).
# ---------------------------------------------------------------------------

def test_invariants_2way_with_missing():
    n_v, n_f = 40, 1013
    v = synth.beta_hw(n_v, n_f, seed=7, missing=0.1)
    codes = brute.unpack_codes(v, n_f)
    pres = (codes != 2).astype(np.int64)
    t, ccc = oracle.two_way(v, n_f)
    cnt = oracle.counts1(v, n_f)
    # f_i(0) + f_i(1) = 1 whenever something is present
    assert np.all(cnt[:, 0] + cnt[:, 1] == 2 * cnt[:, 2])
    assert np.array_equal(cnt[:, 2], pres.sum(1))
    p = 0
    for i in range(n_v):
        for j in range(i + 1, n_v):
            m_ij = int((pres[i] * pres[j]).sum())
            assert t[p].sum() == 4 * m_ij  # the joint frequencies sum to 1
            # marginal over b: 2 * sum over fields where j is present of rho_i(a)
            r0i = np.where(codes[i] == 0, 2, np.where(codes[i] == 1, 1, 0)) * pres[j]
            assert t[p, 0] + t[p, 1] == 2 * int(r0i.sum())
            assert np.all(ccc[p] >= 0.0)
            p += 1


def test_transpose_symmetry_via_block():
    va = synth.beta_hw(13, 517, seed=8, missing=0.05)
    vb = synth.beta_hw(9, 517, seed=9, missing=0.05)
    tab, cab = oracle.block(va, vb, 517)
    tba, cba = oracle.block(vb, va, 517)
    # C_ij(a,b) = C_ji(b,a)
    swapped = tba.transpose(1, 0, 2)[:, :, [0, 2, 1, 3]]
    assert np.array_equal(tab, swapped)
    assert np.allclose(cab, cba.transpose(1, 0, 2)[:, :, [0, 2, 1, 3]], rtol=1e-15, atol=0)


def test_block_of_a_set_with_itself_is_the_triangle():
    v = synth.beta_hw(30, 700, seed=10, missing=0.03)
    t2, c2 = oracle.two_way(v, 700)
    tb, cb = oracle.block(v, v, 700)
    iu = np.triu_indices(30, 1)
    assert np.array_equal(t2, tb[iu])
    assert np.array_equal(c2, cb[iu])


def test_3way_permutation_symmetry():
    n_v, n_f = 7, 301
    v = synth.beta_hw(n_v, n_f, seed=12, missing=0.05)
    t, _ = oracle.three_way(v, n_f, with_ccc=False)
    tt = t.reshape(-1, 2, 2, 2)
    for perm in itertools.permutations(range(3)):
        order = np.array([2, 0, 6, 4, 1, 3, 5])  # arbitrary relabelling of vectors
        vp = v[order]
        tp, _ = oracle.three_way(vp, n_f, with_ccc=False)
        # triple (i,j,k) of the relabelled set is triple sorted(order[i,j,k]) of the original
        p = 0
        for i in range(n_v):
            for j in range(i + 1, n_v):
                for k in range(j + 1, n_v):
                    idx = [order[i], order[j], order[k]]
                    srt = np.argsort(idx)
                    oi, oj, ok = (idx[s] for s in srt)
                    q = oracle.triple_index(n_v, oi, oj, ok)
                    want = np.transpose(tt[q], np.argsort(srt))
                    assert np.array_equal(tp[p].reshape(2, 2, 2), want)
                    p += 1
        break  # one relabelling covers every axis permutation across the triples


def test_3way_margin_is_2way_restricted_to_present_k():
    n_v, n_f = 6, 411
    v = synth.beta_hw(n_v, n_f, seed=13, missing=0.1)
    codes = brute.unpack_codes(v, n_f)
    t3, _ = oracle.three_way(v, n_f, with_ccc=False)
    for (i, j, k) in [(0, 1, 2), (1, 3, 5), (0, 4, 5)]:
        keep = codes[k] != 2
        vv = synth.pack_codes(np.where(keep[None, :], codes[[i, j]], 2))
        t2, _ = oracle.two_way(vv, n_f, with_ccc=False)
        p = oracle.triple_index(n_v, i, j, k)
        s = t3[p].reshape(2, 2, 2).sum(axis=2)
        assert np.array_equal(s.reshape(4), 2 * t2[0])


# ---------------------------------------------------------------------------
# Closed forms for the CCC values (Eqs. (1)-(5)).
# ---------------------------------------------------------------------------

def close(x, y):
    return abs(x - y) <= 1e-15 * max(abs(x), abs(y), 1e-300)


def test_closed_form_het_het_and_homozygous():
    n_f = 333
    # codes: 0 = 00, 1 = 01 (het), 3 = 11
    v = synth.constant([1, 1, 0, 0, 3], n_f)
    t, c = oracle.two_way(v, n_f)
    P = lambda i, j: oracle.pair_index(5, i, j)
    # het x het: every entry n_f, CCC = (1/4)(2/3)(2/3) = 1/9
    assert list(t[P(0, 1)]) == [n_f] * 4
    assert all(close(x, 1 / 9) for x in c[P(0, 1)])
    # 00 x 00: C(0,0) = 4 n_f; f = 1, (1 - 2/3)^2 -> 1/9
    assert list(t[P(2, 3)]) == [4 * n_f, 0, 0, 0]
    assert close(c[P(2, 3)][0], 1 / 9) and list(c[P(2, 3)][1:]) == [0, 0, 0]
    # 00 x 11: only C(0,1); f_i(0) = f_j(1) = 1 -> 1/9.  Swapping the roles of
    # a and b in the frequencies would give 1 here.
    assert list(t[P(2, 4)]) == [0, 4 * n_f, 0, 0]
    assert close(c[P(2, 4)][1], 1 / 9)
    # het x 00: C(0,0) = C(1,0) = 2 n_f; f_ij = 1/2; (1-1/3)(1-2/3) -> 1/9
    assert list(t[P(0, 2)]) == [2 * n_f, 0, 2 * n_f, 0]
    assert close(c[P(0, 2)][0], 1 / 9) and close(c[P(0, 2)][2], 1 / 9)


def test_closed_form_mixed_frequencies():
    # i: 00 on 3/4 of the fields, 11 on 1/4; j: het everywhere.
    n_f = 400
    codes = np.zeros((2, n_f), dtype=np.uint8)
    codes[0, ::4] = 3
    codes[1, :] = 1
    v = codes_to_packed(codes)
    t, c = oracle.two_way(v, n_f)
    assert list(t[0]) == [3 * n_f // 2, 3 * n_f // 2, n_f // 2, n_f // 2]
    # f_i(0) = 3/4, f_i(1) = 1/4, f_j = 1/2
    # CCC(0,b) = 3/8 * (1 - 1/2) * (2/3) = 1/8;  CCC(1,b) = 1/8 * (5/6) * (2/3) = 5/72
    assert close(c[0][0], 1 / 8) and close(c[0][1], 1 / 8)
    assert close(c[0][2], 5 / 72) and close(c[0][3], 5 / 72)


def test_closed_form_with_missing_uses_present_counts():
    # i het on even fields, missing on odd; j het everywhere.  Under the
    # present-field reading m_i = m_ij = n_f/2 and every CCC is still 1/9.
    n_f = 200
    codes = np.ones((2, n_f), dtype=np.uint8)
    codes[0, 1::2] = 2
    v = codes_to_packed(codes)
    t, c = oracle.two_way(v, n_f)
    assert list(t[0]) == [n_f // 2] * 4
    assert all(close(x, 1 / 9) for x in c[0])


def test_closed_form_3way_het_cube_and_all_missing():
    n_f = 129
    v = synth.constant([1, 1, 1, 2], n_f)
    t, c = oracle.three_way(v, n_f)
    p = oracle.triple_index(4, 0, 1, 2)
    assert list(t[p]) == [n_f] * 8
    assert all(close(x, 1 / 27) for x in c[p])  # (1/8)(2/3)^3
    for (i, j, k) in [(0, 1, 3), (0, 2, 3), (1, 2, 3)]:
        q = oracle.triple_index(4, i, j, k)
        assert list(t[q]) == [0] * 8 and list(c[q]) == [0.0] * 8


def test_gamma_zero_gives_joint_frequencies_summing_to_one():
    v = synth.beta_hw(12, 555, seed=14, missing=0.05)
    _, c = oracle.two_way(v, 555, gamma=0.0)
    assert np.allclose(c.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    _, c3 = oracle.three_way(v, 555, gamma=0.0)
    assert np.allclose(c3.sum(axis=1), 1.0, rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# Analytic placement inputs (Sec. 5: synthetic inputs checkable analytically).
# ---------------------------------------------------------------------------

def test_placement_inputs_closed_form():
    s = np.array([1, 2, 3, 4, 6, 7, 12, 5])
    n_f = 1001
    v = synth.placement(s, n_f)
    t, _ = oracle.two_way(v, n_f, with_ccc=False)
    t3, _ = oracle.three_way(v, n_f, with_ccc=False)
    cnt = lambda m: (n_f + m - 1) // m  # fields q in [0, n_f) with q % m == 0
    lcm = lambda *xs: math.lcm(*[int(x) for x in xs])
    p = 0
    for i in range(len(s)):
        for j in range(i + 1, len(s)):
            ci, cj, cij = cnt(s[i]), cnt(s[j]), cnt(lcm(s[i], s[j]))
            # C(0,1): i is 00 where j is 11; C(1,0): i is 11 where j is 00
            want = [4 * (n_f - ci - cj + cij), 4 * (cj - cij), 4 * (ci - cij), 4 * cij]
            assert list(t[p]) == want
            p += 1
    q = 0
    n = len(s)
    for i in range(n):
        for j in range(i + 1, n):
            for k in range(j + 1, n):
                # fields where each vector is 11 (1) or 00 (0): count of each
                # pattern by inclusion-exclusion over the three residues
                def n_pattern(pat):
                    tot = 0
                    for sub in itertools.product([0, 1], repeat=3):
                        if any(sub[x] == 0 and pat[x] == 1 for x in range(3)):
                            continue
                        members = [s[[i, j, k][x]] for x in range(3) if sub[x] or pat[x]]
                        sign = (-1) ** sum(sub[x] and not pat[x] for x in range(3))
                        tot += sign * (cnt(lcm(*members)) if members else n_f)
                    return tot
                want = [8 * n_pattern((a, b, c)) for a in range(2) for b in range(2)
                        for c in range(2)]
                assert list(t3[q]) == want
                q += 1


# ---------------------------------------------------------------------------
# Indexing and row slicing.
# ---------------------------------------------------------------------------

def test_pair_and_triple_index_enumeration():
    n = 9
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    assert [oracle.pair_index(n, i, j) for i, j in pairs] == list(range(len(pairs)))
    tri = [(i, j, k) for i in range(n) for j in range(i + 1, n) for k in range(j + 1, n)]
    assert [oracle.triple_index(n, *x) for x in tri] == list(range(len(tri)))


def test_row_slices_concatenate_to_the_whole():
    v = synth.beta_hw(25, 300, seed=15, missing=0.02)
    t, c = oracle.two_way(v, 300)
    parts = [oracle.two_way(v, 300, a, b) for a, b in [(0, 3), (3, 17), (17, 25)]]
    assert np.array_equal(np.concatenate([x[0] for x in parts]), t)
    t3, _ = oracle.three_way(v, 300, with_ccc=False)
    parts3 = [oracle.three_way(v, 300, a, b, with_ccc=False)[0] for a, b in [(0, 4), (4, 25)]]
    assert np.array_equal(np.concatenate(parts3), t3)


def test_padding_bits_are_ignored():
    codes = np.random.default_rng(1).integers(0, 4, size=(8, 37), dtype=np.uint8)
    a = synth.pack_codes(codes, pad_value=0)
    b = synth.pack_codes(codes, pad_value=-1)
    c = synth.pack_codes(codes, ld=64, pad_value=3)
    ta, _ = oracle.two_way(a, 37)
    assert np.array_equal(ta, oracle.two_way(b, 37)[0])
    assert np.array_equal(ta, oracle.two_way(c, 37)[0])


# ---------------------------------------------------------------------------
# Whole-output checksums.
# ---------------------------------------------------------------------------

def test_fingerprints_match_direct_sums_and_detect_one_change():
    n_v, n_f = 35, 1200
    v = synth.beta_hw(n_v, n_f, seed=16, missing=0.03)
    w, u, z = (synth.weights(n_v, seed=1, tag=k) for k in range(3))
    t, _ = oracle.two_way(v, n_f, with_ccc=False)
    f_in = oracle.fp2_from_input(v, n_f, w, u)
    assert np.array_equal(f_in, oracle.fp2_from_tables(t.astype(np.int32), n_v, w, u))
    bad = t.astype(np.int32).copy()
    bad[123, 2] += 1
    assert not np.array_equal(f_in, oracle.fp2_from_tables(bad, n_v, w, u))

    t3, _ = oracle.three_way(v[:20], n_f, with_ccc=False)
    f3 = oracle.fp3_from_input(v[:20], n_f, w[:20], u[:20], z[:20])
    t3i = t3.astype(np.int32)
    assert np.array_equal(f3, oracle.fp3_from_tables(t3i, 20, w, u, z))
    half = len(t3i) // 2
    s = oracle.fp_add(oracle.fp3_from_tables(t3i[:half], 20, w, u, z, 0),
                      oracle.fp3_from_tables(t3i[half:], 20, w, u, z, half))
    assert np.array_equal(f3, s)

    vb = synth.beta_hw(17, n_f, seed=17, missing=0.03)
    tb, _ = oracle.block(v, vb, n_f, with_ccc=False)
    fb = oracle.fpb_from_input(v, vb, n_f, w, u[:17])
    assert np.array_equal(fb, oracle.fpb_from_tables(tb.astype(np.int32), n_v, 17, w, u[:17]))


def test_list_forms_match_the_row_forms():
    n_v, n_f = 30, 901
    v = synth.beta_hw(n_v, n_f, seed=18, missing=0.05)
    t, c = oracle.two_way(v, n_f)
    rng = np.random.default_rng(3)
    ii = rng.integers(0, n_v - 1, 50)
    jj = np.array([rng.integers(i + 1, n_v) for i in ii])
    lt, lc = oracle.pairs_list(v, v, n_f, ii, jj)
    idx = [oracle.pair_index(n_v, i, j) for i, j in zip(ii, jj)]
    assert np.array_equal(lt, t[idx]) and np.array_equal(lc, c[idx])
    t3, c3 = oracle.three_way(v, n_f)
    tri = [tuple(sorted(rng.choice(n_v, 3, replace=False))) for _ in range(40)]
    a, b, cc = (np.array(x) for x in zip(*tri))
    lt3, lc3 = oracle.triples_list(v, n_f, a, b, cc)
    idx3 = [oracle.triple_index(n_v, *x) for x in tri]
    assert np.array_equal(lt3, t3[idx3]) and np.array_equal(lc3, c3[idx3])
    vb = synth.beta_hw(11, n_f, seed=19, missing=0.05)
    tb, cb = oracle.block(v, vb, n_f)
    jb = rng.integers(0, 11, 50)
    lbt, lbc = oracle.pairs_list(v, vb, n_f, ii, jb)
    assert np.array_equal(lbt, tb[ii, jb]) and np.array_equal(lbc, cb[ii, jb])


def test_closed_form_3way_asymmetric_entry_order():
    # i = 00, j = het, k = 11 on every field: only (a,b,c) = (0,b,1) is nonzero,
    # rho_i(0) rho_j(b) rho_k(1) = 2*1*2 per field -> C = 4 n_f, f = 1/2 and
    # CCC = 1/2 (1 - 2/3)(1 - 1/3)(1 - 2/3) = 1/27 at entries 4a+2b+c = 1 and 3.
    n_f = 211
    v = synth.constant([0, 1, 3], n_f)
    t, c = oracle.three_way(v, n_f)
    assert list(t[0]) == [0, 4 * n_f, 0, 4 * n_f, 0, 0, 0, 0]
    assert close(c[0][1], 1 / 27) and close(c[0][3], 1 / 27)
    assert all(c[0][e] == 0.0 for e in (0, 2, 4, 5, 6, 7))
    # k = 00 instead: a=0, c=0 -> entries 0 and 2
    v2 = synth.constant([0, 1, 0], n_f)
    t2, c2 = oracle.three_way(v2, n_f)
    assert list(t2[0]) == [4 * n_f, 0, 4 * n_f, 0, 0, 0, 0, 0]
    assert close(c2[0][0], 1 / 27) and close(c2[0][2], 1 / 27)
