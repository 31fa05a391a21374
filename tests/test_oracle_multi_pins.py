"""Pins of the multi-allelic oracle (markers with s = 2..4 states, the
extension of Sec. 7 item 2: an s x s table per pair) against facts that do
not come from the oracle itself: the literal allele-pair enumerator, the
biallelic oracle for s = 2, float64 matrix products, closed forms and
invariants."""
import numpy as np
import pytest

import oracle
import oracle.brute as brute
import synth

GAMMA = 2.0 / 3.0


def random_alleles(rng, n_v, n_f, s, missing):
    a1 = rng.integers(0, s, size=(n_v, n_f))
    a2 = rng.integers(0, s, size=(n_v, n_f))
    miss = rng.random((n_v, n_f)) < missing
    a1[miss] = -1
    a2[miss] = -1
    return a1, a2


def rho_matrix(a1, a2, a):
    return ((a1 == a).astype(np.float64) + (a2 == a).astype(np.float64)) * (a1 >= 0)


@pytest.mark.parametrize("s", [2, 3, 4])
@pytest.mark.parametrize("n_v,n_f,missing", [(2, 1, 0.0), (5, 7, 0.2), (9, 33, 0.1), (12, 50, 0.0)])
def test_multi_tables_match_allele_enumerator(s, n_v, n_f, missing):
    rng = np.random.default_rng(100 * s + n_v)
    a1, a2 = random_alleles(rng, n_v, n_f, s, missing)
    v = synth.pack_alleles(a1, a2)
    assert oracle.multi_invalid(v, n_f, s) == 0
    t, _ = oracle.multi_two_way(v, n_f, s)
    assert np.array_equal(t, brute.multi_all_pairs(a1, a2, s))


@pytest.mark.parametrize("missing", [0.0, 0.05, 0.4])
def test_multi_s2_equals_biallelic_oracle(missing):
    """With s = 2 the multi-allelic definitions are the paper's 2-way ones:
    the biallelic code 00/01/11 is the allele pair (0,0)/(0,1)/(1,1) and 10
    the missing marker."""
    v2 = synth.beta_hw(40, 301, seed=11, missing=missing)
    codes = brute.unpack_codes(v2, 301)
    a1 = np.where(codes == 2, -1, (codes >> 1) & 1)
    a2 = np.where(codes == 2, -1, codes & 1)
    vm = synth.pack_alleles(a1, a2)
    tm, cm = oracle.multi_two_way(vm, 301, 2)
    tb, cb = oracle.two_way(v2, 301)
    assert np.array_equal(tm, tb)
    assert np.array_equal(cm.view(np.uint64), cb.view(np.uint64))
    cnt = oracle.multi_counts1(vm, 301, 2)
    assert np.array_equal(cnt[:, [0, 1, 4]], oracle.counts1(v2, 301))
    assert np.all(cnt[:, 2:4] == 0)


@pytest.mark.parametrize("s", [3, 4])
def test_multi_tables_equal_float64_matrix_products(s):
    """C(a,b) = R_a R_b^T with R_a[i][q] = copies of state a (0 when missing):
    exact in float64 since every partial sum is an integer below 2^53."""
    rng = np.random.default_rng(7 + s)
    a1, a2 = random_alleles(rng, 30, 400, s, 0.03)
    v = synth.pack_alleles(a1, a2)
    t, _ = oracle.multi_two_way(v, 400, s)
    R = [rho_matrix(a1, a2, a) for a in range(s)]
    iu, ju = np.triu_indices(30, k=1)
    for a in range(s):
        for b in range(s):
            G = R[a] @ R[b].T
            assert np.array_equal(t[:, a * s + b], G[iu, ju].astype(np.int64))


@pytest.mark.parametrize("s", [3, 4])
def test_multi_invariants_and_ccc_formula(s):
    rng = np.random.default_rng(21 + s)
    a1, a2 = random_alleles(rng, 14, 120, s, 0.1)
    v = synth.pack_alleles(a1, a2)
    t, c = oracle.multi_two_way(v, 120, s)
    cnt = oracle.multi_counts1(v, 120, s)
    present = (a1 >= 0)
    # counts: copies of each state and present fields
    for a in range(s):
        assert np.array_equal(cnt[:, a], rho_matrix(a1, a2, a).sum(axis=1).astype(np.int64))
    assert np.array_equal(cnt[:, 4], present.sum(axis=1))
    assert np.array_equal(cnt[:, :s].sum(axis=1), 2 * cnt[:, 4])
    p = 0
    for i in range(14):
        for j in range(i + 1, 14):
            both = present[i] & present[j]
            m_ij = int(both.sum())
            tab = t[p].reshape(s, s)
            assert tab.sum() == 4 * m_ij
            # marginal over b: twice the copies of a in i on fields where j is present
            for a in range(s):
                assert tab[a].sum() == 2 * int(rho_matrix(a1, a2, a)[i][present[j]].sum())
            # the CCC formula entry by entry (Eqs. (1)-(3) over s states)
            for a in range(s):
                for b in range(s):
                    fi = cnt[i, a] / (2 * cnt[i, 4]) if cnt[i, 4] else 0.0
                    fj = cnt[j, b] / (2 * cnt[j, 4]) if cnt[j, 4] else 0.0
                    want = (tab[a, b] / (4 * m_ij)) * (1 - GAMMA * fi) * (1 - GAMMA * fj) \
                        if m_ij else 0.0
                    assert abs(c[p, a * s + b] - want) <= 1e-15 * max(1.0, abs(want))
            p += 1
    # transpose symmetry: swapping the two vectors transposes the table
    va = synth.pack_alleles(a1[[1, 0]], a2[[1, 0]])
    tt, _ = oracle.multi_two_way(va, 120, s)
    assert np.array_equal(tt[0].reshape(s, s), t[0].reshape(s, s).T)


def test_multi_closed_forms():
    n_f = 333
    # vector 0: all (0,0); vector 1: all (3,3); vector 2: all (1,2); vector 3: all (0,3)
    a1 = np.array([[0] * n_f, [3] * n_f, [1] * n_f, [0] * n_f])
    a2 = np.array([[0] * n_f, [3] * n_f, [2] * n_f, [3] * n_f])
    v = synth.pack_alleles(a1, a2)
    t, c = oracle.multi_two_way(v, n_f, 4)
    P = lambda i, j: oracle.pair_index(4, i, j)
    want = np.zeros(16, dtype=np.int64)
    want[0 * 4 + 3] = 4 * n_f
    assert np.array_equal(t[P(0, 1)], want)
    assert abs(c[P(0, 1), 3] - 1 / 9) <= 1e-15        # (1/1)(1-2/3)(1-2/3)
    # two hets with four distinct states: four entries of n_f, CCC 1/4 (2/3)^2
    want = np.zeros(16, dtype=np.int64)
    for a in (1, 2):
        for b in (0, 3):
            want[a * 4 + b] = n_f
    assert np.array_equal(t[P(2, 3)], want)
    assert np.all(np.abs(c[P(2, 3)][want > 0] - 1 / 9) <= 1e-15)
    assert np.all(c[P(2, 3)][want == 0] == 0.0)


def test_multi_missing_everywhere_and_invalid_bytes():
    v = np.zeros((4, 32), dtype=np.uint8)
    t, c = oracle.multi_two_way(v, 20, 3)
    assert np.all(t == 0) and np.all(c == 0.0)
    assert np.all(oracle.multi_counts1(v, 20, 3) == 0)
    v[0, 3] = 1                    # one copy of state 0 only
    v[1, 5] = 0b11                 # three copies
    v[2, 7] = 1 << 6               # a state beyond s = 3
    v[3, 25] = 1                   # past n_f: ignored
    assert oracle.multi_invalid(v, 20, 3) == 3
    assert oracle.multi_invalid(synth.multi_hw(20, 500, 3, seed=2, missing=0.1), 500, 3) == 0


@pytest.mark.parametrize("s", [2, 4])
def test_multi_list_and_checksum_agree_with_rows(s):
    v = synth.multi_hw(60, 700, s, seed=3, missing=0.02)
    t, c = oracle.multi_two_way(v, 700, s)
    rng = np.random.default_rng(5)
    ij = rng.integers(0, 60, size=(200, 2))
    ij = ij[ij[:, 0] != ij[:, 1]]
    ia, jb = ij.min(axis=1), ij.max(axis=1)
    tl, cl = oracle.multi_pairs_list(v, 700, s, ia, jb)
    p = ia * 60 - ia * (ia + 1) // 2 + (jb - ia - 1)
    assert np.array_equal(tl, t[p]) and np.array_equal(cl, c[p])
    w, u = synth.weights(60, seed=1, tag=0), synth.weights(60, seed=1, tag=1)
    assert np.array_equal(oracle.multi_fp2_from_tables(t.astype(np.int32), 60, s, w, u),
                          oracle.multi_fp2_from_input(v, 700, s, w, u))
    # rows split into two ranges concatenate to the whole triangle
    t1, _ = oracle.multi_two_way(v, 700, s, 0, 17)
    t2, _ = oracle.multi_two_way(v, 700, s, 17, 60)
    assert np.array_equal(np.concatenate([t1, t2]), t)
