"""3-way and block (field-chunked) parity on the GPU against the CPU oracle."""
import numpy as np
import pytest

import oracle
import oracle.brute
import paper_1705_08213_amd as ccc
import synth
from gpu_util import (FORMS, MFMA_FORMS, assert_ccc_close, assert_ccc_identical,
                      assert_tables_equal, dev, form_kw, host, say)

pytestmark = pytest.mark.gpu

PATHS = FORMS

SHAPES3 = [(3, 1, 0.0), (4, 7, 0.2), (9, 100, 0.05), (33, 257, 0.01), (66, 300, 0.01),
           (70, 1000, 0.005), (130, 129, 0.02), (150, 2050, 0.005)]


def sync():
    import torch
    torch.cuda.synchronize()


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_v,n_f,missing", SHAPES3)
def test_3way_parity(path, n_v, n_f, missing):
    say("3way", path, n_v, n_f, missing)
    v = synth.beta_hw(n_v, n_f, seed=n_v + 13 * n_f, missing=missing)
    t, c, cnt = ccc.ccc_3way(dev(v), n_f, **form_kw(path))
    sync()
    ot, oc = oracle.three_way(v, n_f)
    assert_tables_equal(host(t), ot)
    assert_ccc_close(host(c), oc)
    assert np.array_equal(host(cnt)[:, :3], oracle.counts1(v, n_f))


@pytest.mark.parametrize("path", PATHS)
def test_3way_closed_form_and_zero_fields(path):
    say("3way closed", path)
    v = synth.constant([1, 1, 1, 2, 0], 515)
    t, c, _ = ccc.ccc_3way(dev(v), 515, **form_kw(path))
    sync()
    t, c = host(t), host(c)
    p = oracle.triple_index(5, 0, 1, 2)
    assert list(t[p]) == [515] * 8
    assert np.all(np.abs(c[p] - 1 / 27) <= 1e-15)
    v0 = synth.uniform(20, 0)
    t0, c0, _ = ccc.ccc_3way(dev(v0), 0, **form_kw(path))
    sync()
    assert np.all(host(t0) == 0) and np.all(host(c0) == 0.0)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_v,n_f", [(70, 1000), (130, 3001), (66, 100), (140, 257), (5, 9)])
def test_3way_complete_data_and_single_missing_entry(path, n_v, n_f):
    """Complete inputs take the one-plane MFMA form in every 64 x 64 unit
    (four waves over quarters of the fields, tail included); one missing entry
    sends only the units that hold its row (as i, j or k) to the general form."""
    say("3way complete", path, n_v, n_f)
    v = synth.beta_hw(n_v, n_f, seed=300 + n_v, missing=0.0)
    t, c, _ = ccc.ccc_3way(dev(v), n_f, **form_kw(path))
    sync()
    ot, oc = oracle.three_way(v, n_f)
    assert_tables_equal(host(t), ot)
    assert_ccc_close(host(c), oc)
    codes = oracle.brute.unpack_codes(v, n_f)
    codes[n_v // 2, n_f // 3] = 2  # one missing entry
    v2 = synth.pack_codes(codes, pad_value=-1)
    t2, c2, _ = ccc.ccc_3way(dev(v2), n_f, **form_kw(path))
    sync()
    ot2, oc2 = oracle.three_way(v2, n_f)
    assert_tables_equal(host(t2), ot2)
    assert_ccc_close(host(c2), oc2)


@pytest.mark.parametrize("form", MFMA_FORMS)
def test_3way_complete_data_rows_and_select(form):
    """Row ranges whose first row is not on a 64-row unit boundary (the pair
    sums then start at the unit boundary below it) and threshold selection,
    on complete data."""
    import torch
    n, n_f = 150, 777
    say("3way complete rows/select", form)
    v = synth.beta_hw(n, n_f, seed=905, missing=0.0)
    dv = dev(v)
    t_full, c_full, _ = ccc.ccc_3way(dv, n_f, **form_kw(form))
    parts = []
    for i0, i1 in [(0, 5), (5, 64), (64, 70), (70, 129), (129, 150)]:
        t, c, _ = ccc.ccc_3way_rows(dv, n_f, i0, i1, **form_kw(form))
        sync()
        ot, oc = oracle.three_way(v, n_f, i0, i1)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)
        if len(ot):
            parts.append((t, c))
    assert torch.equal(torch.cat([p[0] for p in parts]), t_full)
    assert torch.equal(torch.cat([p[1] for p in parts]), c_full)
    ot, oc = oracle.three_way(v, n_f)
    mx = oc.max(axis=1)
    u = np.unique(mx)
    thr = 0.5 * (u[-51] + u[-50])
    want = np.flatnonzero(mx >= thr)
    found, idx, cc, tt = ccc.ccc_3way_select(dv, n_f, thr, cap=len(want), **form_kw(form))
    assert found == len(want)
    idx, cc, tt = host(idx), host(cc), host(tt)
    order = np.argsort(idx)
    assert np.array_equal(idx[order], want)
    assert_tables_equal(tt[order], ot[want])
    assert_ccc_close(cc[order], oc[want])


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("missing", [0.0, 0.01, 0.3])
def test_3way_ccc_bit_identical_to_oracle(path, missing):
    """Beyond the 1e-12 contract: every CCC double equals the oracle's."""
    say("3way bit-identical", path, missing)
    v = synth.beta_hw(100, 1500, seed=42, missing=missing)
    _, c, _ = ccc.ccc_3way(dev(v), 1500, **form_kw(path))
    sync()
    _, oc = oracle.three_way(v, 1500)
    assert_ccc_identical(host(c), oc)


def test_3way_paths_agree():
    say("3way cross-path")
    v = synth.beta_hw(200, 3000, seed=21, missing=0.005)
    tm, cm, _ = ccc.ccc_3way(dev(v), 3000, **form_kw("fp4"))
    tp, cp, _ = ccc.ccc_3way(dev(v), 3000, path="popcount")
    ti, ci, _ = ccc.ccc_3way(dev(v), 3000, **form_kw("int8"))
    sync()
    assert np.array_equal(host(tm), host(tp)) and np.array_equal(host(tm), host(ti))
    assert np.array_equal(host(cm), host(cp)) and np.array_equal(host(cm), host(ci))
    ot, oc = oracle.three_way(v, 3000, 100, 102)
    lo = oracle.triple_index(200, 100, 101, 102)
    assert_tables_equal(host(tm)[lo:lo + len(ot)], ot)


BLOCK_SHAPES = [(1, 1, 5, 0.0), (5, 3, 100, 0.1), (64, 64, 256, 0.02), (100, 37, 999, 0.02),
                (129, 200, 1025, 0.02), (300, 77, 64, 0.3)]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_a,n_b,n_f,missing", BLOCK_SHAPES)
def test_block_one_shot(path, n_a, n_b, n_f, missing):
    import torch
    say("block", path, n_a, n_b, n_f, missing)
    va = synth.beta_hw(n_a, n_f, seed=n_a, missing=missing)
    vb = synth.beta_hw(n_b, n_f, seed=1000 + n_b, missing=missing)
    tables = torch.empty((n_a, n_b, 4), dtype=torch.int32, device="cuda")
    ca = torch.empty((n_a, 4), dtype=torch.int32, device="cuda")
    cb = torch.empty((n_b, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((n_a, n_b, 4), dtype=torch.float64, device="cuda")
    ccc.ccc_2way_block(dev(va), dev(vb), n_f, tables, ca, cb, cc, **form_kw(path))
    sync()
    ot, oc = oracle.block(va, vb, n_f)
    assert_tables_equal(host(tables), ot)
    assert_ccc_close(host(cc), oc)


@pytest.mark.parametrize("n_a,n_b", [(200, 150), (600, 300)])
@pytest.mark.parametrize("path", PATHS)
def test_block_complete_data_and_one_missing_entry(path, n_a, n_b):
    """Complete A and B take the complete-data kernel (MFMA) in a one-shot
    block call; with one missing entry in B the general kernel runs, and
    its workgroups whose rows are all complete take the cooperative
    one-plane form."""
    import torch
    n_f = 3001
    say("block complete", path, n_a, n_b)
    va = synth.beta_hw(n_a, n_f, seed=61, missing=0.0)
    vb = synth.beta_hw(n_b, n_f, seed=62, missing=0.0)
    codes = oracle.brute.unpack_codes(vb, n_f)
    codes[n_b // 2, 1234] = 2
    vb2 = synth.pack_codes(codes, pad_value=-1)
    for b in (vb, vb2):
        tables = torch.empty((n_a, n_b, 4), dtype=torch.int32, device="cuda")
        ca = torch.empty((n_a, 4), dtype=torch.int32, device="cuda")
        cb = torch.empty((n_b, 4), dtype=torch.int32, device="cuda")
        cc = torch.empty((n_a, n_b, 4), dtype=torch.float64, device="cuda")
        ccc.ccc_2way_block(dev(va), dev(b), n_f, tables, ca, cb, cc, **form_kw(path))
        sync()
        ot, oc = oracle.block(va, b, n_f)
        assert_tables_equal(host(tables), ot)
        assert_ccc_close(host(cc), oc)


@pytest.mark.parametrize("path", PATHS)
def test_block_chunked_equals_one_shot(path):
    import torch
    # 5 chunks of 1024 fields plus a ragged last chunk of 333, garbage padding
    n_a, n_b, chunk, nchunks, last = 150, 90, 1024, 5, 333
    n_f = chunk * nchunks + last
    say("block chunked", path, n_a, n_b, n_f)
    va = synth.beta_hw(n_a, n_f, seed=31, missing=0.02)
    vb = synth.beta_hw(n_b, n_f, seed=32, missing=0.02)
    da, db = dev(va), dev(vb)
    tables = torch.full((n_a, n_b, 4), -7, dtype=torch.int32, device="cuda")
    ca = torch.full((n_a, 4), -7, dtype=torch.int32, device="cuda")
    cb = torch.full((n_b, 4), -7, dtype=torch.int32, device="cuda")
    cc = torch.zeros((n_a, n_b, 4), dtype=torch.float64, device="cuda")
    for k in range(nchunks + 1):
        nf_k = chunk if k < nchunks else last
        ccc.ccc_2way_block(da, db, nf_k, tables, ca, cb, cc, accumulate=k > 0,
                           finalize=k == nchunks, field_offset=k * chunk // 4, **form_kw(path))
    sync()
    ot, oc = oracle.block(va, vb, n_f)
    assert_tables_equal(host(tables), ot)
    assert_ccc_close(host(cc), oc)
    assert np.array_equal(host(ca)[:, :3], oracle.counts1(va, n_f))
    assert np.array_equal(host(cb)[:, :3], oracle.counts1(vb, n_f))


def test_block_decomposition_equals_triangle():
    """The 2-way triangle equals the paper's block decomposition (diagonal
    blocks as triangles, off-diagonal blocks as rectangles) run on one GPU."""
    import torch
    n, n_f, nb = 300, 1500, 3
    say("block decomposition", n, n_f)
    v = synth.beta_hw(n, n_f, seed=41, missing=0.01)
    t_full, c_full, _ = ccc.ccc_2way(dev(v), n_f)
    sync()
    t_full, c_full = host(t_full), host(c_full)
    edges = [0, 100, 200, 300]
    for bi in range(nb):
        for bj in range(bi + 1, nb):
            a0, a1, b0, b1 = edges[bi], edges[bi + 1], edges[bj], edges[bj + 1]
            tables = torch.empty((a1 - a0, b1 - b0, 4), dtype=torch.int32, device="cuda")
            ca = torch.empty((a1 - a0, 4), dtype=torch.int32, device="cuda")
            cb = torch.empty((b1 - b0, 4), dtype=torch.int32, device="cuda")
            cc = torch.empty((a1 - a0, b1 - b0, 4), dtype=torch.float64, device="cuda")
            ccc.ccc_2way_block(dev(v[a0:a1]), dev(v[b0:b1]), n_f, tables, ca, cb, cc)
            sync()
            tb, cbk = host(tables), host(cc)
            for i in range(a0, a1, 37):
                p0 = oracle.pair_index(n, i, b0)
                assert np.array_equal(t_full[p0:p0 + (b1 - b0)], tb[i - a0])
                assert np.array_equal(c_full[p0:p0 + (b1 - b0)], cbk[i - a0])
