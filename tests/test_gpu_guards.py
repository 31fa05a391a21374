"""Guard regions around every output the library writes at computed offsets:
each output is an interior slice of a larger buffer whose head and tail hold a
known pattern, and after the call the guards must be untouched while the
interior matches the oracle.  Covers the dense triangle and tetrahedron,
row-range (staged) calls, threshold selection (records, tables and counter),
field-chunked block calls and batched problems, on the popcount path and on
the MFMA path with each operand format."""
import numpy as np
import pytest

import oracle
import paper_1705_08213_amd as ccc
import synth
from gpu_util import FORMS, assert_ccc_close, assert_tables_equal, dev, form_kw, host, say

pytestmark = pytest.mark.gpu

G = 64  # guard rows on each side (a multiple of 16 bytes for every element width)
I32_GUARD = 0x5A5A5A5A
F64_GUARD_BITS = 0x7FF4DEADBEEF0001  # a NaN no computation produces


def sync():
    import torch
    torch.cuda.synchronize()


class Guarded:
    """A [rows, width] output as the interior of a [G + rows + G, width] buffer."""

    def __init__(self, rows, width, dtype):
        import torch
        self.rows = rows
        self.buf = torch.empty((G + rows + G, width), dtype=dtype, device="cuda")
        if dtype == torch.float64:
            self.buf.view(torch.int64).fill_(F64_GUARD_BITS)
        else:
            self.buf.view(torch.int32).fill_(I32_GUARD)
        self.ref = self.buf[:G].clone(), self.buf[G + rows:].clone()

    @property
    def inner(self):
        return self.buf[G:G + self.rows]

    def check(self, what):
        import torch
        head, tail = self.ref
        assert torch.equal(self.buf[:G].view(torch.uint8), head.view(torch.uint8)), f"{what}: head"
        assert torch.equal(self.buf[G + self.rows:].view(torch.uint8), tail.view(torch.uint8)), \
            f"{what}: tail"


def guarded_2way(n_v, rows, width=4):
    import torch
    return (Guarded(rows, width, torch.int32), Guarded(rows, width, torch.float64),
            Guarded(n_v, 4, torch.int32))


# missing 0: the complete-data kernel of the MFMA forms writes the output
@pytest.mark.parametrize("missing", [0.02, 0.0])
@pytest.mark.parametrize("form", FORMS)
def test_guards_2way_triangle_and_rows(form, missing):
    n, n_f = 300, 1537
    say("guards 2way", form, missing)
    v = synth.beta_hw(n, n_f, seed=71, missing=missing)
    dv = dev(v)
    t, c, cnt = guarded_2way(n, ccc.n_pairs(n))
    ccc.ccc_2way(dv, n_f, t.inner, c.inner, cnt.inner, **form_kw(form))
    sync()
    for g, name in ((t, "tables"), (c, "ccc"), (cnt, "counts")):
        g.check(name)
    ot, oc = oracle.two_way(v, n_f)
    assert_tables_equal(host(t.inner), ot)
    assert_ccc_close(host(c.inner), oc)
    for i0, i1 in [(0, 1), (5, 130), (129, 257), (298, 300)]:
        P = ccc.pair_run_length(n, i0, i1)
        t, c, cnt = guarded_2way(n, P)
        ccc.ccc_2way_rows(dv, n_f, i0, i1, t.inner, c.inner, cnt.inner, **form_kw(form))
        sync()
        for g, name in ((t, "tables"), (c, "ccc"), (cnt, "counts")):
            g.check(f"rows [{i0},{i1}) {name}")
        ot, oc = oracle.two_way(v, n_f, i0, i1)
        assert_tables_equal(host(t.inner), ot)
        assert_ccc_close(host(c.inner), oc)


@pytest.mark.parametrize("form", FORMS)
def test_guards_3way_tetrahedron_and_rows(form):
    n, n_f = 90, 777
    say("guards 3way", form)
    v = synth.beta_hw(n, n_f, seed=72, missing=0.02)
    dv = dev(v)
    t, c, cnt = guarded_2way(n, ccc.n_triples(n), width=8)
    ccc.ccc_3way(dv, n_f, t.inner, c.inner, cnt.inner, **form_kw(form))
    sync()
    for g, name in ((t, "tables"), (c, "ccc"), (cnt, "counts")):
        g.check(name)
    ot, oc = oracle.three_way(v, n_f)
    assert_tables_equal(host(t.inner), ot)
    assert_ccc_close(host(c.inner), oc)
    for i0, i1 in [(0, 2), (3, 65), (64, 88)]:
        T = ccc.triple_run_length(n, i0, i1)
        t, c, cnt = guarded_2way(n, T, width=8)
        ccc.ccc_3way_rows(dv, n_f, i0, i1, t.inner, c.inner, cnt.inner, **form_kw(form))
        sync()
        for g, name in ((t, "tables"), (c, "ccc"), (cnt, "counts")):
            g.check(f"rows [{i0},{i1}) {name}")
        ot, oc = oracle.three_way(v, n_f, i0, i1)
        assert_tables_equal(host(t.inner), ot)
        assert_ccc_close(host(c.inner), oc)


@pytest.mark.parametrize("form", FORMS)
@pytest.mark.parametrize("way", [2, 3])
def test_guards_selection_records_and_counter(form, way):
    """A cap below the number of kept entries: the records stop at the cap,
    nothing is written past it, and the counter (two int64, the second
    untouched) holds the exact count."""
    import torch
    n, n_f = (257, 2001) if way == 2 else (70, 999)
    say("guards select", way, form)
    v = synth.beta_hw(n, n_f, seed=73 + way, missing=0.02)
    ot, oc = (oracle.two_way if way == 2 else oracle.three_way)(v, n_f)
    width = 4 if way == 2 else 8
    mx = oc.max(axis=1)
    u = np.unique(mx)
    thr = 0.5 * (u[-41] + u[-40])
    want = np.flatnonzero(mx >= thr)
    for cap in (len(want) + 5, 16):
        index = Guarded(cap, 1, torch.int64)
        cc = Guarded(cap, width, torch.float64)
        tt = Guarded(cap, width, torch.int32)
        count = Guarded(2, 1, torch.int64)
        count.buf[G + 1] = -12345
        count.ref = count.buf[:G].clone(), count.buf[G + 2:].clone()
        sel = ccc.ccc_selection(index.inner.data_ptr(), cc.inner.data_ptr(), tt.inner.data_ptr(),
                                cap, count.inner.data_ptr())
        fn = ccc.lib().ccc_2way_select if way == 2 else ccc.lib().ccc_3way_select
        o = ccc.make_opts(**form_kw(form))
        import ctypes
        dv = dev(v)
        st = fn(ctypes.c_void_p(dv.data_ptr()), n, n_f, v.shape[1], float(thr), ctypes.byref(sel),
                None, ctypes.byref(o), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == 0
        sync()
        for g, name in ((index, "index"), (cc, "ccc"), (tt, "tables"), (count, "count")):
            g.check(f"cap {cap} {name}")
        assert int(count.inner[0]) == len(want) and int(count.inner[1]) == -12345
        k = min(cap, len(want))
        idx = host(index.inner[:k, 0])
        assert len(set(idx.tolist())) == k and set(idx.tolist()) <= set(want.tolist())
        order = np.argsort(idx)
        assert_tables_equal(host(tt.inner[:k])[order], ot[np.sort(idx)])
        assert_ccc_close(host(cc.inner[:k])[order], oc[np.sort(idx)])


@pytest.mark.parametrize("form", FORMS)
def test_guards_block_chunked(form):
    import torch
    n_a, n_b, chunk, nchunks = 150, 90, 1024, 3
    n_f = chunk * nchunks
    say("guards block", form)
    va = synth.beta_hw(n_a, n_f, seed=74, missing=0.02)
    vb = synth.beta_hw(n_b, n_f, seed=75, missing=0.02)
    da, db = dev(va), dev(vb)
    t = Guarded(n_a * n_b, 4, torch.int32)
    c = Guarded(n_a * n_b, 4, torch.float64)
    ca = Guarded(n_a, 4, torch.int32)
    cb = Guarded(n_b, 4, torch.int32)
    for k in range(nchunks):
        ccc.ccc_2way_block(da, db, chunk, t.inner.view(n_a, n_b, 4), ca.inner, cb.inner,
                           c.inner.view(n_a, n_b, 4), accumulate=k > 0, finalize=k == nchunks - 1,
                           field_offset=k * chunk // 4, **form_kw(form))
    sync()
    for g, name in ((t, "tables"), (c, "ccc"), (ca, "counts_a"), (cb, "counts_b")):
        g.check(name)
    ot, oc = oracle.block(va, vb, n_f)
    assert_tables_equal(host(t.inner).reshape(n_a, n_b, 4), ot)
    assert_ccc_close(host(c.inner).reshape(n_a, n_b, 4), oc)


@pytest.mark.parametrize("form", FORMS)
def test_guards_batched_problems(form):
    import torch
    sizes = [(300, 1000), (2, 5), (129, 4097), (700, 333), (1, 77), (64, 256)]
    say("guards many", form)
    hosts, probs, guards = [], [], []
    for k, (n_v, n_f) in enumerate(sizes):
        v = synth.beta_hw(n_v, n_f, seed=760 + k, missing=0.02)
        hosts.append(v)
        P = ccc.n_pairs(n_v)
        t = Guarded(P, 4, torch.int32)
        c = Guarded(P, 4, torch.float64)
        cnt = Guarded(n_v, 4, torch.int32)
        guards.append((t, c, cnt))
        probs.append(dict(v=dev(v), n_f=n_f, tables=t.inner, ccc=c.inner, counts=cnt.inner))
    ccc.ccc_2way_many(probs, **form_kw(form))
    sync()
    for (n_v, n_f), v, (t, c, cnt) in zip(sizes, hosts, guards):
        for g, name in ((t, "tables"), (c, "ccc"), (cnt, "counts")):
            g.check(f"problem {n_v}x{n_f} {name}")
        ot, oc = oracle.two_way(v, n_f)
        assert_tables_equal(host(t.inner), ot)
        assert_ccc_close(host(c.inner), oc)


@pytest.mark.parametrize("form", ["fp4", "int8"])
def test_guards_multi_allelic(form):
    import torch
    n, n_f, s = 150, 1001, 3
    say("guards multi", form)
    v = synth.multi_hw(n, n_f, s, seed=77, missing=0.02)
    P = ccc.n_pairs(n)
    t = Guarded(P, s * s, torch.int32)
    c = Guarded(P, s * s, torch.float64)
    cnt = Guarded(n, 8, torch.int32)
    ccc.ccc_2way_multi(dev(v), n_f, s, t.inner, c.inner, cnt.inner, **form_kw(form))
    sync()
    for g, name in ((t, "tables"), (c, "ccc"), (cnt, "counts")):
        g.check(name)
    ot, oc = oracle.multi_two_way(v, n_f, s)
    assert_tables_equal(host(t.inner), ot)
    assert_ccc_close(host(c.inner), oc)
