"""Batched 2-way problems (one persistent launch per tile variant, captured in
a HIP graph and replayed): every problem equals the oracle and the one-shot
entry point, on every replay."""
import ctypes
import os

import numpy as np
import pytest

import oracle
import paper_1705_08213_amd as ccc
import synth
from gpu_util import FORMS, MFMA_FORMS, assert_ccc_close, assert_tables_equal, dev, form_kw, host, say

pytestmark = pytest.mark.gpu


def sync():
    import torch
    torch.cuda.synchronize()


def make_batch(sizes, seed, missing=0.02):
    hosts, probs = [], []
    for k, (n_v, n_f) in enumerate(sizes):
        v = synth.beta_hw(n_v, n_f, seed=seed + k, missing=missing)
        hosts.append(v)
        probs.append(dict(v=dev(v), n_f=n_f))
    return hosts, probs


SIZES = [(300, 1000), (2, 5), (1, 77), (129, 4097), (64, 256), (700, 333), (5, 0), (257, 1500),
         (1000, 2000), (3, 64)]


# every tile variant of the persistent kernels (forced), one with a forced
# workgroups-per-CU figure, and the tuned choice
@pytest.fixture(params=["0", "1", "2", "3", "1/wg1", "tuned"])
def variant(request, monkeypatch):
    monkeypatch.delenv("CCC_MANY_VARIANT", raising=False)
    monkeypatch.delenv("CCC_MANY_WG", raising=False)
    if request.param != "tuned":
        var, _, wg = request.param.partition("/wg")
        monkeypatch.setenv("CCC_MANY_VARIANT", var)
        if wg:
            monkeypatch.setenv("CCC_MANY_WG", wg)
    yield request.param


@pytest.mark.parametrize("path", FORMS)
def test_many_matches_oracle(variant, path):
    say("many", variant, path)
    hosts, probs = make_batch(SIZES, seed=500)
    outs = ccc.ccc_2way_many(probs, **form_kw(path))
    sync()
    for (n_v, n_f), v, (t, c, cnt) in zip(SIZES, hosts, outs):
        ot, oc = oracle.two_way(v, n_f)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)
        assert np.array_equal(host(cnt)[:, :3], oracle.counts1(v, n_f))


@pytest.mark.parametrize("path", FORMS)
def test_many_complete_data_problems(variant, path):
    """A batch with no missing entries: the persistent kernels take the
    per-wave (MFMA) or per-workgroup (popcount) complete-data form."""
    say("many complete", variant, path)
    hosts, probs = make_batch(SIZES, seed=700, missing=0.0)
    outs = ccc.ccc_2way_many(probs, **form_kw(path))
    sync()
    for (n_v, n_f), v, (t, c, _) in zip(SIZES, hosts, outs):
        ot, oc = oracle.two_way(v, n_f)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)


@pytest.mark.parametrize("form", MFMA_FORMS)
def test_many_graph_replays_with_eager_work_between(variant, form):
    import torch
    say("many replays", variant, form)
    hosts, probs = make_batch(SIZES[:6] + [(2000, 3000)], seed=600)
    outs = ccc.ccc_2way_many(probs, **form_kw(form))
    sync()
    ref = [(t.clone(), c.clone(), cnt.clone()) for t, c, cnt in outs]
    for p, (t, c, cnt) in zip(probs, outs):
        p.update(tables=t, ccc=c, counts=cnt)
    for rep in range(4):
        for t, c, cnt in outs:  # scribble over the outputs between replays
            t.fill_(-1)
            c.fill_(-1.0)
            cnt.fill_(-1)
        x = torch.randn(1 << 20, device="cuda")
        (x * 2).sum().item()  # unrelated eager work and a sync
        ccc.ccc_2way_many(probs, **form_kw(form))
        sync()
        for (t, c, cnt), (rt, rc, rcnt) in zip(outs, ref):
            assert torch.equal(t, rt) and torch.equal(c, rc) and torch.equal(cnt, rcnt), rep


def test_many_equals_single_calls_and_graph_off(monkeypatch):
    import torch
    say("many vs single")
    sizes = [(1500, 5000), (333, 12345), (4000, 1000), (90, 50000)]
    hosts, probs = make_batch(sizes, seed=700)
    outs = ccc.ccc_2way_many(probs)
    monkeypatch.setenv("CCC_MANY_GRAPH", "0")
    outs_direct = ccc.ccc_2way_many([dict(v=p["v"], n_f=p["n_f"]) for p in probs])
    sync()
    for p, (t, c, _), (t2, c2, _) in zip(probs, outs, outs_direct):
        t1, c1, _ = ccc.ccc_2way(p["v"], p["n_f"])
        sync()
        assert torch.equal(t, t1) and torch.equal(c, c1)
        assert torch.equal(t2, t1) and torch.equal(c2, c1)


def test_many_counts_null_through_the_c_abi():
    import torch
    say("many counts NULL")
    hosts, probs = make_batch([(100, 700), (37, 64)], seed=800)
    arr = (ccc.ccc_problem * 2)()
    keep = []
    for k, p in enumerate(probs):
        n_v, ld = p["v"].shape
        t = torch.empty((ccc.n_pairs(n_v), 4), dtype=torch.int32, device="cuda")
        c = torch.empty((ccc.n_pairs(n_v), 4), dtype=torch.float64, device="cuda")
        keep += [t, c]
        arr[k] = ccc.ccc_problem(p["v"].data_ptr(), n_v, p["n_f"], ld, t.data_ptr(),
                                 c.data_ptr(), None)
    st = ccc.lib().ccc_2way_many(arr, 2, None, ctypes.c_void_p(torch.cuda.current_stream()
                                                                 .cuda_stream))
    assert st == 0
    sync()
    for k, v in enumerate(hosts):
        ot, oc = oracle.two_way(v, probs[k]["n_f"])
        assert_tables_equal(host(keep[2 * k]), ot)
        assert_ccc_close(host(keep[2 * k + 1]), oc)
