"""3-way and block (field-chunked) parity on the GPU against the CPU oracle."""
import numpy as np
import pytest

import oracle
import paper_1705_08213_amd as ccc
import synth
from gpu_util import assert_ccc_close, assert_tables_equal, dev, host, say

pytestmark = pytest.mark.gpu

PATHS = ["popcount", "mfma"]

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
    t, c, cnt = ccc.ccc_3way(dev(v), n_f, path=path)
    sync()
    ot, oc = oracle.three_way(v, n_f)
    assert_tables_equal(host(t), ot)
    assert_ccc_close(host(c), oc)
    assert np.array_equal(host(cnt)[:, :3], oracle.counts1(v, n_f))


@pytest.mark.parametrize("path", PATHS)
def test_3way_closed_form_and_zero_fields(path):
    say("3way closed", path)
    v = synth.constant([1, 1, 1, 2, 0], 515)
    t, c, _ = ccc.ccc_3way(dev(v), 515, path=path)
    sync()
    t, c = host(t), host(c)
    p = oracle.triple_index(5, 0, 1, 2)
    assert list(t[p]) == [515] * 8
    assert np.all(np.abs(c[p] - 1 / 27) <= 1e-15)
    v0 = synth.uniform(20, 0)
    t0, c0, _ = ccc.ccc_3way(dev(v0), 0, path=path)
    sync()
    assert np.all(host(t0) == 0) and np.all(host(c0) == 0.0)


def test_3way_paths_agree():
    say("3way cross-path")
    v = synth.beta_hw(200, 3000, seed=21, missing=0.005)
    tm, cm, _ = ccc.ccc_3way(dev(v), 3000, path="mfma")
    tp, cp, _ = ccc.ccc_3way(dev(v), 3000, path="popcount")
    sync()
    assert np.array_equal(host(tm), host(tp))
    assert np.array_equal(host(cm), host(cp))
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
    ccc.ccc_2way_block(dev(va), dev(vb), n_f, tables, ca, cb, cc, path=path)
    sync()
    ot, oc = oracle.block(va, vb, n_f)
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
                           finalize=k == nchunks, path=path, field_offset=k * chunk // 4)
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
