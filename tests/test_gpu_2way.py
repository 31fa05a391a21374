"""2-way parity on the GPU: the popcount path and the MFMA path with fp4 and
with int8 operands, against the CPU oracle, element by element: bit-exact
tables and CCC within 1e-12."""
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

# (n_v, n_f, missing, extra ld units): tiny, ragged in both dimensions, several
# tiles and super-steps, tails of every length class
SHAPES = [
    (2, 1, 0.0, 0), (3, 5, 0.3, 0), (17, 100, 0.05, 1), (64, 256, 0.0, 0), (65, 257, 0.02, 0),
    (127, 511, 0.01, 2), (128, 1000, 0.01, 0), (130, 1024, 0.1, 0), (200, 1537, 0.01, 1),
    (257, 3001, 0.01, 0), (300, 64, 0.5, 0), (129, 16, 0.0, 0),
]


def run2(v, n_f, path, **kw):
    t, c, cnt = ccc.ccc_2way(dev(v), n_f, **form_kw(path), **kw)
    import torch
    torch.cuda.synchronize()
    return (None if t is None else host(t)), (None if c is None else host(c)), host(cnt)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_v,n_f,missing,extra", SHAPES)
def test_2way_parity_small(path, n_v, n_f, missing, extra):
    say("2way", path, n_v, n_f, missing, extra)
    v = synth.beta_hw(n_v, n_f, seed=n_v * 7 + n_f, missing=missing,
                      ld=synth.ld_for(n_f, extra))
    t, c, cnt = run2(v, n_f, path)
    ot, oc = oracle.two_way(v, n_f)
    assert_tables_equal(t, ot)
    assert_ccc_close(c, oc)
    ocnt = oracle.counts1(v, n_f)
    assert np.array_equal(cnt[:, :3], ocnt) and np.all(cnt[:, 3] == 0)


@pytest.mark.parametrize("path", PATHS)
def test_2way_config1_full(path):
    # 512 vectors x 1000 fields, genotypes uniform over {00,01,11}, no missing, seed 0
    say("2way config1", path)
    v = synth.uniform(512, 1000, seed=0, missing=0.0)
    t, c, _ = run2(v, 1000, path)
    ot, oc = oracle.two_way(v, 1000)
    assert_tables_equal(t, ot)
    assert_ccc_close(c, oc)


@pytest.mark.parametrize("path", PATHS)
def test_2way_zero_fields_and_all_missing(path):
    say("2way edge", path)
    v = synth.uniform(70, 0, seed=1)
    t, c, cnt = run2(v, 0, path)
    assert np.all(t == 0) and np.all(c == 0.0) and np.all(cnt == 0)
    codes = np.full((40, 333), 2, dtype=np.uint8)  # every entry missing
    codes[5] = 1
    v = synth.pack_codes(codes, pad_value=-1)
    t, c, _ = run2(v, 333, path)
    ot, oc = oracle.two_way(v, 333)
    assert_tables_equal(t, ot)
    assert_ccc_close(c, oc)
    assert np.all(t == 0) and np.all(c == 0.0)


@pytest.mark.parametrize("path", PATHS)
def test_2way_closed_forms(path):
    say("2way closed", path)
    v = synth.constant([1, 1, 0, 0, 3], 777)
    t, c, _ = run2(v, 777, path)
    P = lambda i, j: oracle.pair_index(5, i, j)
    assert list(t[P(0, 1)]) == [777] * 4
    assert np.all(np.abs(c[P(0, 1)] - 1 / 9) <= 1e-15)
    assert list(t[P(2, 4)]) == [0, 4 * 777, 0, 0]


@pytest.mark.parametrize("path", PATHS)
def test_2way_outputs_optional_and_gamma(path):
    say("2way optional", path)
    v = synth.beta_hw(90, 700, seed=5, missing=0.02)
    t_only, c_none, _ = run2(v, 700, path, want_ccc=False)
    assert c_none is None
    t_none, c_only, _ = run2(v, 700, path, want_tables=False, gamma=0.25)
    assert t_none is None
    ot, oc = oracle.two_way(v, 700, gamma=0.25)
    assert_tables_equal(t_only, ot)
    assert_ccc_close(c_only, oc)


def test_2way_paths_agree_and_are_deterministic():
    say("2way cross-path")
    v = synth.beta_hw(1000, 5003, seed=9, missing=0.01)
    tm, cm, _ = run2(v, 5003, "fp4")
    tp, cp, _ = run2(v, 5003, "popcount")
    ti, ci, _ = run2(v, 5003, "int8")
    tm2, cm2, _ = run2(v, 5003, "fp4")
    assert np.array_equal(tm, tp) and np.array_equal(tm, tm2) and np.array_equal(tm, ti)
    assert np.array_equal(cm, cm2)
    assert_ccc_close(cm, cp, rtol=0.0)
    assert_ccc_close(cm, ci, rtol=0.0)
    # sampled rows against the oracle
    for i0, i1 in [(0, 2), (511, 513), (997, 999)]:
        ot, oc = oracle.two_way(v, 5003, i0, i1)
        lo = oracle.pair_index(1000, i0, i0 + 1)
        assert_tables_equal(tm[lo:lo + len(ot)], ot)
        assert_ccc_close(cm[lo:lo + len(ot)], oc)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("n_v,n_f", [(200, 3001), (300, 512), (70, 9)])
def test_2way_complete_data_and_single_missing_entry(path, n_v, n_f):
    """Complete inputs take the complete-data kernel on the MFMA side; with
    one missing entry in one row the general kernel runs, and only its
    tiles holding that row use the four-plane form.  Both must match the
    oracle."""
    say("2way complete", path, n_v, n_f)
    v = synth.beta_hw(n_v, n_f, seed=77 + n_v, missing=0.0)
    t, c, _ = run2(v, n_f, path)
    ot, oc = oracle.two_way(v, n_f)
    assert_tables_equal(t, ot)
    assert_ccc_close(c, oc)
    codes = oracle.brute.unpack_codes(v, n_f)
    codes[n_v // 2, n_f // 3] = 2  # one missing entry
    v2 = synth.pack_codes(codes, pad_value=-1)
    t2, c2, _ = run2(v2, n_f, path)
    ot2, oc2 = oracle.two_way(v2, n_f)
    assert_tables_equal(t2, ot2)
    assert_ccc_close(c2, oc2)


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("missing", [0.0, 0.01, 0.3])
def test_2way_ccc_bit_identical_to_oracle(path, missing):
    """Beyond the 1e-12 contract: the shared-reciprocal quotient is the
    correctly rounded t/den, so every CCC double equals the oracle's."""
    say("2way bit-identical", path, missing)
    v = synth.beta_hw(300, 2500, seed=41, missing=missing)
    _, c, _ = run2(v, 2500, path)
    _, oc = oracle.two_way(v, 2500)
    assert_ccc_identical(c, oc)


@pytest.mark.parametrize("variant", ["0", "1", "2"])
@pytest.mark.parametrize("form", MFMA_FORMS)
def test_2way_oneshot_tile_variants(variant, form, monkeypatch):
    """Every workgroup-tile shape of the one-shot general kernel, forced (the
    kernel-shape table picks among them by size): ragged triangles, a row
    range, a block, and complete data with one missing entry (complete tiles
    inside a call that is not complete)."""
    import torch
    monkeypatch.setenv("CCC_ONESHOT_VARIANT", variant)
    for n_v, n_f in [(300, 1537), (97, 300)]:
        say("2way variant", variant, form, n_v, n_f)
        v = synth.beta_hw(n_v, n_f, seed=1300 + n_v, missing=0.02)
        t, c, _ = run2(v, n_f, form)
        ot, oc = oracle.two_way(v, n_f)
        assert_tables_equal(t, ot)
        assert_ccc_close(c, oc)
        t, c, _ = ccc.ccc_2way_rows(dev(v), n_f, 37, 70, **form_kw(form))
        torch.cuda.synchronize()
        ot, oc = oracle.two_way(v, n_f, 37, 70)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)
    say("2way variant block", variant, form)
    n_a, n_b, n_f = 150, 70, 999
    va = synth.beta_hw(n_a, n_f, seed=1401, missing=0.02)
    vb = synth.beta_hw(n_b, n_f, seed=1402, missing=0.02)
    tables = torch.empty((n_a, n_b, 4), dtype=torch.int32, device="cuda")
    ca = torch.empty((n_a, 4), dtype=torch.int32, device="cuda")
    cb = torch.empty((n_b, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((n_a, n_b, 4), dtype=torch.float64, device="cuda")
    ccc.ccc_2way_block(dev(va), dev(vb), n_f, tables, ca, cb, cc, **form_kw(form))
    torch.cuda.synchronize()
    ot, oc = oracle.block(va, vb, n_f)
    assert_tables_equal(host(tables), ot)
    assert_ccc_close(host(cc), oc)
    say("2way variant mixed complete", variant, form)
    n_v, n_f = 260, 700
    codes = oracle.brute.unpack_codes(synth.beta_hw(n_v, n_f, seed=1403, missing=0.0), n_f)
    codes[200, 345] = 2  # one missing entry: the call is not complete
    v = synth.pack_codes(codes, pad_value=-1)
    t, c, _ = run2(v, n_f, form)
    ot, oc = oracle.two_way(v, n_f)
    assert_tables_equal(t, ot)
    assert_ccc_close(c, oc)
