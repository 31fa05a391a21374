"""Staged output (row ranges) and threshold-filtered output on the GPU,
against the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_1705_08213_amd as ccc
import synth
from gpu_util import FORMS, assert_ccc_close, assert_tables_equal, dev, form_kw, host, say

pytestmark = pytest.mark.gpu

PATHS = FORMS


def sync():
    import torch
    torch.cuda.synchronize()


# missing 0: every row complete, so the MFMA forms take the complete-data
# kernel (256 x 128 workgroup tiles) instead of the general one
MISSING = [0.02, 0.0]


@pytest.mark.parametrize("missing", MISSING)
@pytest.mark.parametrize("path", PATHS)
def test_2way_rows_concatenate_to_the_triangle(path, missing):
    import torch
    n, n_f = 300, 1537
    say("2way rows", path, missing)
    v = synth.beta_hw(n, n_f, seed=901, missing=missing)
    dv = dev(v)
    t_full, c_full, _ = ccc.ccc_2way(dv, n_f, **form_kw(path))
    parts = []
    for i0, i1 in [(0, 1), (1, 57), (57, 128), (128, 129), (129, 299), (299, 300), (10, 10)]:
        t, c, _ = ccc.ccc_2way_rows(dv, n_f, i0, i1, **form_kw(path))
        sync()
        ot, oc = oracle.two_way(v, n_f, i0, i1)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)
        if i1 > i0:
            parts.append((t, c))
    assert torch.equal(torch.cat([p[0] for p in parts]), t_full)
    assert torch.equal(torch.cat([p[1] for p in parts]), c_full)


@pytest.mark.parametrize("missing", MISSING)
@pytest.mark.parametrize("path", PATHS)
def test_2way_rows_across_square_strips(path, missing):
    # 1500 rows are 12 square rows of 128 (6 of 256 for complete data): the
    # MFMA launch walks them in strips of 8 (one whole, one partial); ranges
    # start and end inside strips and squares
    import torch
    n, n_f = 1500, 300
    say("2way rows across strips", path, missing)
    v = synth.beta_hw(n, n_f, seed=907, missing=missing)
    dv = dev(v)
    t_full, c_full, _ = ccc.ccc_2way(dv, n_f, **form_kw(path))
    sync()
    ot, oc = oracle.two_way(v, n_f)
    assert_tables_equal(host(t_full), ot)
    assert_ccc_close(host(c_full), oc)
    parts = []
    for i0, i1 in [(0, 700), (700, 1030), (1030, 1100), (1100, 1500)]:
        t, c, _ = ccc.ccc_2way_rows(dv, n_f, i0, i1, **form_kw(path))
        sync()
        ot, oc = oracle.two_way(v, n_f, i0, i1)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)
        if i1 > i0:
            parts.append((t, c))
    assert torch.equal(torch.cat([p[0] for p in parts]), t_full)
    assert torch.equal(torch.cat([p[1] for p in parts]), c_full)


@pytest.mark.parametrize("path", PATHS)
def test_3way_rows_concatenate_to_the_tetrahedron(path):
    import torch
    n, n_f = 90, 700
    say("3way rows", path)
    v = synth.beta_hw(n, n_f, seed=902, missing=0.02)
    dv = dev(v)
    t_full, c_full, _ = ccc.ccc_3way(dv, n_f, **form_kw(path))
    parts = []
    for i0, i1 in [(0, 5), (5, 64), (64, 65), (65, 88), (88, 90)]:
        t, c, _ = ccc.ccc_3way_rows(dv, n_f, i0, i1, **form_kw(path))
        sync()
        ot, oc = oracle.three_way(v, n_f, i0, i1)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)
        if len(ot):
            parts.append((t, c))
    assert torch.equal(torch.cat([p[0] for p in parts]), t_full)
    assert torch.equal(torch.cat([p[1] for p in parts]), c_full)


def threshold_between(values, keep_fraction):
    """A threshold strictly between two distinct values of `values`, keeping
    about keep_fraction of them."""
    u = np.unique(values)
    k = max(1, int(len(u) * (1 - keep_fraction)))
    return 0.5 * (u[k - 1] + u[k])


@pytest.mark.parametrize("missing", MISSING)
@pytest.mark.parametrize("path", PATHS)
def test_2way_select_matches_filtered_oracle(path, missing):
    n, n_f = 257, 2001
    say("2way select", path, missing)
    v = synth.beta_hw(n, n_f, seed=903, missing=missing)
    ot, oc = oracle.two_way(v, n_f)
    thr = threshold_between(oc.max(axis=1), 0.01)
    want = np.flatnonzero(oc.max(axis=1) >= thr)
    found, idx, cc, tt = ccc.ccc_2way_select(dev(v), n_f, thr, cap=len(want) + 100,
                                             **form_kw(path))
    assert found == len(want)
    idx, cc, tt = host(idx), host(cc), host(tt)
    order = np.argsort(idx)
    assert np.array_equal(idx[order], want)
    assert_tables_equal(tt[order], ot[want])
    assert_ccc_close(cc[order], oc[want])
    # a cap below the number found: the count is exact, the records a subset
    found2, idx2, cc2, _ = ccc.ccc_2way_select(dev(v), n_f, thr, cap=7, **form_kw(path))
    assert found2 == len(want) and len(host(idx2)) == 7
    assert set(host(idx2).tolist()) <= set(want.tolist())
    # threshold above every value: nothing kept
    found3, _, _, _ = ccc.ccc_2way_select(dev(v), n_f, 2.0, cap=4, **form_kw(path))
    assert found3 == 0


@pytest.mark.parametrize("path", PATHS)
def test_3way_select_matches_filtered_oracle(path):
    n, n_f = 70, 999
    say("3way select", path)
    v = synth.beta_hw(n, n_f, seed=904, missing=0.02)
    ot, oc = oracle.three_way(v, n_f)
    thr = threshold_between(oc.max(axis=1), 0.005)
    want = np.flatnonzero(oc.max(axis=1) >= thr)
    found, idx, cc, tt = ccc.ccc_3way_select(dev(v), n_f, thr, cap=len(want), **form_kw(path))
    assert found == len(want)
    idx, cc, tt = host(idx), host(cc), host(tt)
    order = np.argsort(idx)
    assert np.array_equal(idx[order], want)
    assert_tables_equal(tt[order], ot[want])
    assert_ccc_close(cc[order], oc[want])


def test_select_at_full_size_2way():
    """Selection at the large 2-way shape, in the same launch configuration as
    the dense call: the kept set equals the dense output filtered on the GPU,
    and sampled kept pairs match the oracle."""
    import torch
    n_v, n_f = 32768, 65536
    say("2way select full size: generate")
    v = synth.beta_hw(n_v, n_f, seed=0, missing=0.01)
    dv = dev(v)
    say("2way select full size: dense + select")
    t, c, _ = ccc.ccc_2way(dv, n_f)
    mx = c.max(dim=1).values
    # threshold at a high quantile of a random sample: keeps ~1e-5 of the pairs
    g = torch.Generator(device="cuda").manual_seed(3)
    sample = mx[torch.randint(0, mx.numel(), (1 << 20,), device="cuda", generator=g)]
    thr = float(torch.sort(sample).values[-10])
    want = torch.nonzero(mx >= thr).flatten()
    assert 100 < want.numel() < (1 << 22)
    found, idx, cc, tt = ccc.ccc_2way_select(dv, n_f, thr, cap=int(want.numel()) + 1000)
    assert found == want.numel()
    order = torch.argsort(idx)
    assert torch.equal(idx[order], want)
    assert torch.equal(cc[order], c[want]) and torch.equal(tt[order], t[want])
    del t, c
    # a few kept pairs against the oracle, one by one
    pick_t = order[:: max(1, found // 50)]
    pick = host(idx[pick_t])
    rows = np.arange(n_v, dtype=np.int64)
    starts = rows * n_v - rows * (rows + 1) // 2
    ii = np.searchsorted(starts, pick, side="right") - 1
    jj = pick - starts[ii] + ii + 1
    ot, oc = oracle.pairs_list(v, v, n_f, ii, jj)
    assert_tables_equal(host(tt[pick_t]), ot)
    assert_ccc_close(host(cc[pick_t]), oc)
