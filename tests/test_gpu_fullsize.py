"""Parity at the workloads' full sizes, in the launch configuration bench.py
times: every table through a whole-output checksum (weighted sums mod 2^61-1
that the oracle evaluates from the input in O(n_v n_f)), sampled pairs and
triples against the oracle one by one (tables bit-exact, CCC within 1e-12),
the 1-way counts in full, and the HIP forms against each other: popcount,
and the MFMA path with fp4 and with int8 operands (forced; fp4 is what the
default picks at these sizes)."""
import numpy as np
import pytest

import oracle
import paper_1705_08213_amd as ccc
import synth
from gpu_util import assert_ccc_close, assert_tables_equal, dev, say

pytestmark = pytest.mark.gpu


def sync():
    import torch
    torch.cuda.synchronize()


def boundary_indices(n, tile=64, extra=()):
    xs = {0, 1, n - 2, n - 1, *extra}
    for b in range(tile, n, tile * 7):
        xs.update({b - 1, b, b + 1})
    return sorted(x for x in xs if 0 <= x < n)


def sample_pairs(n, rng, count=2000):
    idx = boundary_indices(n)
    ia, jb = [], []
    for i in idx:
        for j in idx:
            if i < j:
                ia.append(i)
                jb.append(j)
    r = rng.integers(0, n, size=(count, 2))
    r = r[r[:, 0] != r[:, 1]]
    ia += list(r.min(1))
    jb += list(r.max(1))
    return np.array(ia, dtype=np.int64), np.array(jb, dtype=np.int64)


def gather_rows(t, idx):
    import torch
    return t[torch.from_numpy(np.asarray(idx, dtype=np.int64)).cuda()].cpu().numpy()


def pair_index_np(n, i, j):
    return i * n - i * (i + 1) // 2 + (j - i - 1)


def test_c2_2way_large_full_size():
    import torch
    n_v, n_f = 32768, 65536
    say("c2 full size: generate")
    v = synth.beta_hw(n_v, n_f, seed=0, missing=0.01)
    dv = dev(v)
    say("c2 full size: mfma ccc_2way")
    t, c, cnt = ccc.ccc_2way(dv, n_f, path="mfma")
    sync()
    assert np.array_equal(cnt.cpu().numpy()[:, :3], oracle.counts1(v, n_f))
    rng = np.random.default_rng(2)
    ia, jb = sample_pairs(n_v, rng)
    say("c2 full size: sampled pairs", len(ia))
    ot, oc = oracle.pairs_list(v, v, n_f, ia, jb)
    p = pair_index_np(n_v, ia, jb)
    assert_tables_equal(gather_rows(t, p), ot)
    assert_ccc_close(gather_rows(c, p), oc)
    say("c2 full size: int8 ccc_2way")
    ti, ci, _ = ccc.ccc_2way(dv, n_f, path="mfma", operands="int8")
    sync()
    assert_tables_equal(gather_rows(ti, p), ot)
    assert_ccc_close(gather_rows(ci, p), oc)
    assert torch.equal(t, ti) and torch.equal(c, ci)
    del c, ti, ci
    say("c2 full size: popcount ccc_2way")
    tp, _, _ = ccc.ccc_2way(dv, n_f, path="popcount", want_ccc=False)
    sync()
    assert torch.equal(t, tp)
    del tp
    say("c2 full size: checksum")
    w, u = synth.weights(n_v, seed=5, tag=0), synth.weights(n_v, seed=5, tag=1)
    th = t.cpu().numpy()
    assert np.array_equal(oracle.fp2_from_tables(th, n_v, w, u),
                          oracle.fp2_from_input(v, n_f, w, u))


def test_c3_3way_full_size():
    import torch
    n_v, n_f = 2048, 16384
    say("c3 full size: generate")
    v = synth.beta_hw(n_v, n_f, seed=0, missing=0.005)
    dv = dev(v)
    say("c3 full size: mfma ccc_3way")
    t, c, cnt = ccc.ccc_3way(dv, n_f, path="mfma")
    sync()
    assert np.array_equal(cnt.cpu().numpy()[:, :3], oracle.counts1(v, n_f))
    rng = np.random.default_rng(3)
    idx = boundary_indices(n_v, tile=32)
    tri = set()
    for a in range(len(idx)):
        for b in range(a + 1, len(idx), 3):
            for cc in range(b + 1, len(idx), 5):
                tri.add((idx[a], idx[b], idx[cc]))
    for _ in range(1500):
        x = np.sort(rng.choice(n_v, 3, replace=False))
        tri.add(tuple(int(y) for y in x))
    for j in (1, 63, 64, 1000, 2046):  # neighbours of the middle index
        tri.update({(j - 1, j, j + 1)} if 0 < j < n_v - 1 else set())
    ii, jj, kk = (np.array(z, dtype=np.int64) for z in zip(*sorted(tri)))
    say("c3 full size: sampled triples", len(ii))
    ot, oc = oracle.triples_list(v, n_f, ii, jj, kk)
    p = [oracle.triple_index(n_v, int(a), int(b), int(d)) for a, b, d in zip(ii, jj, kk)]
    assert_tables_equal(gather_rows(t, p), ot)
    assert_ccc_close(gather_rows(c, p), oc)
    # int8 operands: every table (45.7 GB beside the fp4 output), and the CCC
    # values of two staged row runs
    say("c3 full size: int8 ccc_3way tables")
    ti, _, _ = ccc.ccc_3way(dv, n_f, path="mfma", operands="int8", want_ccc=False)
    sync()
    assert_tables_equal(gather_rows(ti, p), ot)
    assert torch.equal(t, ti)
    del ti
    for i0, i1 in [(0, 3), (1000, 1066)]:
        say("c3 full size: int8 ccc_3way_rows", i0, i1)
        tr, cr, _ = ccc.ccc_3way_rows(dv, n_f, i0, i1, path="mfma", operands="int8")
        sync()
        lo = oracle.triple_index(n_v, i0, i0 + 1, i0 + 2)
        assert torch.equal(tr, t[lo:lo + tr.shape[0]])
        assert torch.equal(cr, c[lo:lo + cr.shape[0]])
        del tr, cr
    del c
    say("c3 full size: checksum over slices")
    w, u, z = (synth.weights(n_v, seed=6, tag=k) for k in range(3))
    total = np.zeros(8, dtype=np.uint64)
    T = t.shape[0]
    step = 1 << 27
    for s in range(0, T, step):
        e = min(T, s + step)
        total = oracle.fp_add(total, oracle.fp3_from_tables(t[s:e].cpu().numpy(), n_v, w, u, z,
                                                            t_begin=s))
    assert np.array_equal(total, oracle.fp3_from_input(v, n_f, w, u, z))


def test_c3_shape_complete_data_full_size():
    """The 3-way shape with no missing entries: every unit takes the one-plane
    complete-data form.  Sampled triples against the oracle one by one, every
    table through the whole-output checksum."""
    import torch
    n_v, n_f = 2048, 16384
    say("c3 complete: generate")
    v = synth.beta_hw(n_v, n_f, seed=0, missing=0.0)
    dv = dev(v)
    say("c3 complete: mfma ccc_3way")
    t, c, cnt = ccc.ccc_3way(dv, n_f, path="mfma")
    sync()
    assert int(cnt[:, 2].min()) == n_f
    rng = np.random.default_rng(13)
    tri = set()
    for _ in range(1500):
        x = np.sort(rng.choice(n_v, 3, replace=False))
        tri.add(tuple(int(y) for y in x))
    for j in (1, 63, 64, 65, 127, 128, 1000, 2046):
        tri.add((j - 1, j, j + 1))
        tri.add((0, j, n_v - 1))
    ii, jj, kk = (np.array(z, dtype=np.int64) for z in zip(*sorted(tri)))
    say("c3 complete: sampled triples", len(ii))
    ot, oc = oracle.triples_list(v, n_f, ii, jj, kk)
    p = [oracle.triple_index(n_v, int(a), int(b), int(d)) for a, b, d in zip(ii, jj, kk)]
    assert_tables_equal(gather_rows(t, p), ot)
    assert_ccc_close(gather_rows(c, p), oc)
    del c
    say("c3 complete: int8 ccc_3way tables")
    ti, _, _ = ccc.ccc_3way(dv, n_f, path="mfma", operands="int8", want_ccc=False)
    sync()
    assert_tables_equal(gather_rows(ti, p), ot)
    assert torch.equal(t, ti)
    del ti
    say("c3 complete: checksum over slices")
    w, u, z = (synth.weights(n_v, seed=14, tag=k) for k in range(3))
    total = np.zeros(8, dtype=np.uint64)
    T = t.shape[0]
    step = 1 << 27
    for s in range(0, T, step):
        e = min(T, s + step)
        total = oracle.fp_add(total, oracle.fp3_from_tables(t[s:e].cpu().numpy(), n_v, w, u, z,
                                                            t_begin=s))
    assert np.array_equal(total, oracle.fp3_from_input(v, n_f, w, u, z))


def test_c5_block_full_size_chunked():
    import torch
    n, n_f, chunk = 16384, 131072, 16384
    say("c5 full size: generate")
    va = synth.beta_hw(n, n_f, seed=0, missing=0.02)
    vb = synth.beta_hw(n, n_f, seed=1, missing=0.02)
    da, db = dev(va), dev(vb)
    tables = torch.empty((n, n, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((n, n, 4), dtype=torch.float64, device="cuda")
    ca = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    cb = torch.empty((n, 4), dtype=torch.int32, device="cuda")
    say("c5 full size: 8 chunk calls")
    for k in range(n_f // chunk):
        ccc.ccc_2way_block(da, db, chunk, tables, ca, cb, cc, accumulate=k > 0,
                           finalize=k == n_f // chunk - 1, field_offset=k * chunk // 4)
    sync()
    say("c5 full size: 8 chunk calls, int8 operands")
    ti, ci = torch.empty_like(tables), torch.empty_like(cc)
    cai, cbi = torch.empty_like(ca), torch.empty_like(cb)
    for k in range(n_f // chunk):
        ccc.ccc_2way_block(da, db, chunk, ti, cai, cbi, ci, accumulate=k > 0,
                           finalize=k == n_f // chunk - 1, field_offset=k * chunk // 4,
                           path="mfma", operands="int8")
    sync()
    assert torch.equal(ti, tables) and torch.equal(ci, cc)
    assert torch.equal(cai, ca) and torch.equal(cbi, cb)
    del ti, ci
    assert np.array_equal(ca.cpu().numpy()[:, :3], oracle.counts1(va, n_f))
    assert np.array_equal(cb.cpu().numpy()[:, :3], oracle.counts1(vb, n_f))
    rng = np.random.default_rng(4)
    bi = boundary_indices(n)
    ia = np.array([a for a in bi for _ in bi] + list(rng.integers(0, n, 1500)), dtype=np.int64)
    jb = np.array([b for _ in bi for b in bi] + list(rng.integers(0, n, 1500)), dtype=np.int64)
    say("c5 full size: sampled pairs", len(ia))
    ot, oc = oracle.pairs_list(va, vb, n_f, ia, jb)
    flat = ia * n + jb
    assert_tables_equal(gather_rows(tables.view(-1, 4), flat), ot)
    assert_ccc_close(gather_rows(cc.view(-1, 4), flat), oc)
    del cc
    say("c5 full size: checksum")
    w, u = synth.weights(n, seed=7, tag=0), synth.weights(n, seed=7, tag=1)
    assert np.array_equal(oracle.fpb_from_tables(tables.cpu().numpy(), n, n, w, u),
                          oracle.fpb_from_input(va, vb, n_f, w, u))


def test_c4_batched_full_size():
    import torch
    nv, nf = synth.batch_sizes(64, seed=0)
    say("c4 full size: generate", int(nv.sum()))
    hosts, probs = [], []
    for k in range(64):
        v = synth.beta_hw(int(nv[k]), int(nf[k]), seed=100 + k, missing=0.01)
        hosts.append(v)
        probs.append(dict(v=dev(v), n_f=int(nf[k])))
    say("c4 full size: ccc_2way_many")
    outs = ccc.ccc_2way_many(probs)
    sync()
    rng = np.random.default_rng(5)
    for k in range(64):
        n_v, n_f = int(nv[k]), int(nf[k])
        t, c, cnt = outs[k]
        v = hosts[k]
        assert np.array_equal(cnt.cpu().numpy()[:, :3], oracle.counts1(v, n_f)), k
        ia, jb = sample_pairs(n_v, rng, count=100)
        ot, oc = oracle.pairs_list(v, v, n_f, ia, jb)
        p = pair_index_np(n_v, ia, jb)
        assert_tables_equal(gather_rows(t, p), ot)
        assert_ccc_close(gather_rows(c, p), oc)
        w, u = synth.weights(n_v, seed=8, tag=0), synth.weights(n_v, seed=8, tag=1)
        assert np.array_equal(oracle.fp2_from_tables(t.cpu().numpy(), n_v, w, u),
                              oracle.fp2_from_input(v, n_f, w, u)), k
    say("c4 full size: ccc_2way_many, int8 operands")
    outs_i = ccc.ccc_2way_many([dict(v=p["v"], n_f=p["n_f"]) for p in probs], path="mfma",
                               operands="int8")
    sync()
    for k in range(64):
        assert all(torch.equal(x, y) for x, y in zip(outs[k], outs_i[k])), k
    del outs_i
    # the batch equals independent calls
    say("c4 full size: against single calls")
    for k in (0, 17, 63):
        t1, c1, _ = ccc.ccc_2way(probs[k]["v"], probs[k]["n_f"])
        sync()
        assert torch.equal(t1, outs[k][0]) and torch.equal(c1, outs[k][1])


def test_c2_shape_complete_data_full_size():
    """The large 2-way shape with no missing entries (the paper's main-text
    setting): every tile takes the one-plane MFMA path."""
    import torch
    n_v, n_f = 32768, 65536
    say("c2 complete: generate")
    v = synth.beta_hw(n_v, n_f, seed=0, missing=0.0)
    dv = dev(v)
    say("c2 complete: mfma")
    t, c, cnt = ccc.ccc_2way(dv, n_f, path="mfma")
    sync()
    assert int(cnt[:, 2].min()) == n_f
    rng = np.random.default_rng(12)
    ia, jb = sample_pairs(n_v, rng, count=1000)
    ot, oc = oracle.pairs_list(v, v, n_f, ia, jb)
    p = pair_index_np(n_v, ia, jb)
    assert_tables_equal(gather_rows(t, p), ot)
    assert_ccc_close(gather_rows(c, p), oc)
    say("c2 complete: int8 operands")
    ti, ci, _ = ccc.ccc_2way(dv, n_f, path="mfma", operands="int8")
    sync()
    assert torch.equal(t, ti) and torch.equal(c, ci)
    del c, ti, ci
    say("c2 complete: checksum")
    w, u = synth.weights(n_v, seed=9, tag=0), synth.weights(n_v, seed=9, tag=1)
    assert np.array_equal(oracle.fp2_from_tables(t.cpu().numpy(), n_v, w, u),
                          oracle.fp2_from_input(v, n_f, w, u))


@pytest.mark.parametrize("missing", [0.0, 1e-6])
def test_huge_field_count_exact_in_int32(missing):
    """n_f = 2^27 + 3 fields (a ragged tail) for a handful of vectors: 2-way
    entries reach 4 n_f ~ 2^29 and 3-way entries 8 n_f ~ 2^30, near the int32
    limits the API enforces; the complete-data forms rebuild entries through
    sums that wrap modulo 2^32 on the way.  Both paths, every table and CCC
    value against the oracle."""
    n_v, n_f = 5, (1 << 27) + 3
    say("huge n_f", missing)
    v = synth.beta_hw(n_v, n_f, seed=21, missing=missing)
    dv = dev(v)
    ot2, oc2 = oracle.two_way(v, n_f)
    ot3, oc3 = oracle.three_way(v, n_f)
    for path in ("mfma", "popcount"):
        say("huge n_f", missing, path)
        t, c, _ = ccc.ccc_2way(dv, n_f, path=path)
        t3, c3, _ = ccc.ccc_3way(dv, n_f, path=path)
        sync()
        assert_tables_equal(t.cpu().numpy(), ot2)
        assert_ccc_close(c.cpu().numpy(), oc2)
        assert_tables_equal(t3.cpu().numpy(), ot3)
        assert_ccc_close(c3.cpu().numpy(), oc3)
    assert int(ot3.max()) > (1 << 29)  # the wide entries were exercised


def test_huge_field_count_multi_allelic():
    n_v, n_f, s = 4, (1 << 26) + 5, 4
    say("huge n_f multi")
    v = synth.multi_hw(n_v, n_f, s, seed=22, missing=0.0)
    t, c, _ = ccc.ccc_2way_multi(dev(v), n_f, s)
    sync()
    ot, oc = oracle.multi_two_way(v, n_f, s)
    assert_tables_equal(t.cpu().numpy(), ot)
    assert_ccc_close(c.cpu().numpy(), oc)
