"""Multi-allelic 2-way CCC (s = 2..4 states per marker, an s x s table per
pair) on the GPU against the CPU oracle: tables bit-exact, CCC within 1e-12
(and bit-identical), counts in full."""
import numpy as np
import pytest

import oracle
import oracle.brute
import paper_1705_08213_amd as ccc
import synth
from gpu_util import (MFMA_FORMS, assert_ccc_close, assert_ccc_identical, assert_tables_equal,
                      dev, form_kw, host, say)

pytestmark = pytest.mark.gpu

# (n_v, n_f, missing, extra ld units): tiny, ragged in both dimensions, several
# tiles and K steps, every tail length class
SHAPES = [(2, 1, 0.0, 0), (3, 5, 0.3, 0), (17, 100, 0.05, 1), (64, 64, 0.0, 0),
          (65, 257, 0.02, 0), (130, 1000, 0.01, 2), (200, 1537, 0.1, 0), (97, 16, 0.0, 0)]


def run_multi(v, n_f, s, **kw):
    import torch
    t, c, cnt = ccc.ccc_2way_multi(dev(v), n_f, s, **kw)
    torch.cuda.synchronize()
    return (None if t is None else host(t)), (None if c is None else host(c)), host(cnt)


def check_counts(cnt, v, n_f, s):
    oc = oracle.multi_counts1(v, n_f, s)
    assert np.array_equal(cnt[:, :4], oc[:, :4])
    assert np.array_equal(cnt[:, 4], oc[:, 4])
    assert np.all(cnt[:, 5:] == 0)


@pytest.mark.parametrize("form", MFMA_FORMS)
@pytest.mark.parametrize("s", [2, 3, 4])
@pytest.mark.parametrize("n_v,n_f,missing,extra", SHAPES)
def test_multi_parity(s, n_v, n_f, missing, extra, form):
    say("multi", s, n_v, n_f, missing, extra, form)
    v = synth.multi_hw(n_v, n_f, s, seed=n_v * 3 + n_f + s, missing=missing,
                       ld=synth.ld_multi(n_f, extra))
    t, c, cnt = run_multi(v, n_f, s, **form_kw(form))
    ot, oc = oracle.multi_two_way(v, n_f, s)
    assert_tables_equal(t, ot)
    assert_ccc_close(c, oc)
    assert_ccc_identical(c, oc)
    check_counts(cnt, v, n_f, s)


def test_multi_s2_equals_biallelic_path():
    """With s = 2 the multi-allelic call on re-encoded input gives exactly the
    biallelic call's tables and CCC."""
    say("multi s=2 vs 2-way")
    v2 = synth.beta_hw(300, 2001, seed=31, missing=0.02)
    codes = oracle.brute.unpack_codes(v2, 2001)
    a1 = np.where(codes == 2, -1, (codes >> 1) & 1)
    a2 = np.where(codes == 2, -1, codes & 1)
    vm = synth.pack_alleles(a1, a2)
    tm, cm, _ = run_multi(vm, 2001, 2)
    import torch
    tb, cb, _ = ccc.ccc_2way(dev(v2), 2001, path="mfma")
    torch.cuda.synchronize()
    assert np.array_equal(tm, host(tb))
    assert np.array_equal(cm.view(np.uint64), host(cb).view(np.uint64))


def test_multi_closed_forms_and_optional_outputs():
    say("multi closed")
    n_f = 777
    a1 = np.array([[0] * n_f, [3] * n_f, [1] * n_f, [0] * n_f])
    a2 = np.array([[0] * n_f, [3] * n_f, [2] * n_f, [3] * n_f])
    v = synth.pack_alleles(a1, a2)
    t, c, _ = run_multi(v, n_f, 4)
    P = lambda i, j: oracle.pair_index(4, i, j)
    assert t[P(0, 1)][3] == 4 * n_f and t[P(0, 1)].sum() == 4 * n_f
    assert abs(c[P(0, 1)][3] - 1 / 9) <= 1e-15
    for a in (1, 2):
        for b in (0, 3):
            assert t[P(2, 3)][a * 4 + b] == n_f
    t_only, c_none, _ = run_multi(v, n_f, 4, want_ccc=False)
    assert c_none is None and np.array_equal(t_only, t)
    t_none, c_only, _ = run_multi(v, n_f, 4, want_tables=False, gamma=0.25)
    assert t_none is None
    _, oc = oracle.multi_two_way(v, n_f, 4, gamma=0.25)
    assert_ccc_close(c_only, oc)


def test_multi_all_missing_and_zero_fields():
    say("multi edge")
    v = np.zeros((40, 48), dtype=np.uint8)
    t, c, cnt = run_multi(v, 40, 3)
    assert np.all(t == 0) and np.all(c == 0.0) and np.all(cnt == 0)
    v0 = synth.multi_hw(70, 0, 4, seed=1)
    t0, c0, cnt0 = run_multi(v0, 0, 4)
    assert np.all(t0 == 0) and np.all(c0 == 0.0) and np.all(cnt0 == 0)


def test_multi_full_size():
    """The multi-allelic bench shape (n_v = 16384, n_f = 32768, s = 4, 1%
    missing) in the launch configuration bench.py times: sampled pairs
    against the oracle one by one, every table through the checksum."""
    import torch
    n_v, n_f, s = 16384, 32768, 4
    say("multi full size: generate")
    v = synth.multi_hw(n_v, n_f, s, seed=0, missing=0.01)
    dv = dev(v)
    say("multi full size: ccc_2way_multi")
    t, c, cnt = ccc.ccc_2way_multi(dv, n_f, s)
    torch.cuda.synchronize()
    check_counts(host(cnt), v, n_f, s)
    rng = np.random.default_rng(17)
    idx = sorted({0, 1, 63, 64, 65, 127, 128, n_v // 2, n_v - 2, n_v - 1})
    ia = [a for a in idx for b in idx if a < b]
    jb = [b for a in idx for b in idx if a < b]
    r = rng.integers(0, n_v, size=(1500, 2))
    r = r[r[:, 0] != r[:, 1]]
    ia = np.array(ia + list(r.min(1)), dtype=np.int64)
    jb = np.array(jb + list(r.max(1)), dtype=np.int64)
    say("multi full size: sampled pairs", len(ia))
    ot, oc = oracle.multi_pairs_list(v, n_f, s, ia, jb)
    p = ia * n_v - ia * (ia + 1) // 2 + (jb - ia - 1)
    pt = torch.from_numpy(p).cuda()
    assert_tables_equal(host(t[pt]), ot)
    assert_ccc_close(host(c[pt]), oc)
    del c
    say("multi full size: checksum")
    w, u = synth.weights(n_v, seed=10, tag=0), synth.weights(n_v, seed=10, tag=1)
    assert np.array_equal(oracle.multi_fp2_from_tables(host(t), n_v, s, w, u),
                          oracle.multi_fp2_from_input(v, n_f, s, w, u))
