"""The 2-way MFMA kernels take fp4 (e2m1) operands while n_f <= 2^22, where
every sum of quarter-multiples they accumulate stays exact in fp32, and int8
operands beyond.  Both sides of that bound at the extreme values (rows with
every field 11, so C11 = 4 n_f reaches 2^24 at the bound; rows all 00, all 01,
all missing; random rows with and without missing entries) on the triangle,
the block call and batched calls, tables bit-exact and CCC against the
oracle."""
import numpy as np
import pytest

import oracle
import paper_1705_08213_amd as ccc
import synth
from gpu_util import assert_ccc_close, assert_tables_equal, dev, host, say

pytestmark = pytest.mark.gpu

LIMIT = 1 << 22


def sync():
    import torch
    torch.cuda.synchronize()


def extreme_rows(n_f, seed):
    const = synth.constant([3, 3, 0, 1, 2], n_f, seed=seed)  # 11, 11, 00, 01, missing
    rand = synth.beta_hw(2, n_f, seed=seed, missing=0.0)
    miss = synth.beta_hw(2, n_f, seed=seed + 1, missing=0.02)
    return np.ascontiguousarray(np.concatenate([const, rand, miss]))


@pytest.mark.parametrize("n_f", [LIMIT - 1, LIMIT, LIMIT + 1, LIMIT + 256])
def test_triangle_on_both_sides_of_the_fp4_bound(n_f):
    say("fp4 bound triangle", n_f)
    v = extreme_rows(n_f, seed=n_f % 97)
    t, c, _ = ccc.ccc_2way(dev(v), n_f, path="mfma")
    sync()
    ot, oc = oracle.two_way(v, n_f)
    assert_tables_equal(host(t), ot)
    assert_ccc_close(host(c), oc)
    assert int(ot.max()) == 4 * n_f  # the two all-11 rows


@pytest.mark.parametrize("n_f", [LIMIT, LIMIT + 1])
def test_block_on_both_sides_of_the_fp4_bound(n_f):
    import torch
    say("fp4 bound block", n_f)
    v = extreme_rows(n_f, seed=3)
    va, vb = np.ascontiguousarray(v[:6]), np.ascontiguousarray(v[2:])
    n_a, n_b = va.shape[0], vb.shape[0]
    tables = torch.empty((n_a, n_b, 4), dtype=torch.int32, device="cuda")
    ca = torch.empty((n_a, 4), dtype=torch.int32, device="cuda")
    cb = torch.empty((n_b, 4), dtype=torch.int32, device="cuda")
    cc = torch.empty((n_a, n_b, 4), dtype=torch.float64, device="cuda")
    ccc.ccc_2way_block(dev(va), dev(vb), n_f, tables, ca, cb, cc, path="mfma")
    sync()
    ot, oc = oracle.block(va, vb, n_f)
    assert_tables_equal(host(tables), ot)
    assert_ccc_close(host(cc), oc)


@pytest.mark.parametrize("big", [LIMIT, LIMIT + 1])
def test_batch_mixing_sizes_across_the_fp4_bound(big):
    """One problem decides the operand format of the whole batch."""
    say("fp4 bound many", big)
    hosts = [extreme_rows(big, seed=5), synth.beta_hw(300, 1000, seed=6, missing=0.02),
             synth.beta_hw(129, 4097, seed=7, missing=0.0)]
    sizes = [big, 1000, 4097]
    outs = ccc.ccc_2way_many([dict(v=dev(v), n_f=f) for v, f in zip(hosts, sizes)], path="mfma")
    sync()
    for v, n_f, (t, c, _) in zip(hosts, sizes, outs):
        ot, oc = oracle.two_way(v, n_f)
        assert_tables_equal(host(t), ot)
        assert_ccc_close(host(c), oc)


@pytest.mark.parametrize("complete", [False, True])
@pytest.mark.parametrize("n_f", [LIMIT, LIMIT + 1])
def test_3way_on_both_sides_of_the_fp4_bound(n_f, complete):
    """Three all-11 rows put C(1,1,1) at 8 n_f; with no missing entry every
    unit takes the one-plane complete-data form (its Gram pair sums too)."""
    say("fp4 bound 3-way", n_f, complete)
    if complete:
        v = np.ascontiguousarray(np.concatenate([
            synth.constant([3, 3, 3, 0, 1], n_f, seed=4),
            synth.beta_hw(3, n_f, seed=5, missing=0.0)]))
    else:
        v = np.ascontiguousarray(np.concatenate([synth.constant([3], n_f, seed=4),
                                                 extreme_rows(n_f, seed=6)]))
    t, c, _ = ccc.ccc_3way(dev(v), n_f, path="mfma")
    sync()
    ot, oc = oracle.three_way(v, n_f)
    assert_tables_equal(host(t), ot)
    assert_ccc_close(host(c), oc)
    assert int(ot.max()) == 8 * n_f


@pytest.mark.parametrize("n_f", [LIMIT, LIMIT + 1])
def test_multi_allelic_on_both_sides_of_the_fp4_bound(n_f):
    """s = 4: two rows homozygous for state 3 (byte 0x80: rho(3) = 2) put
    C(3,3) at 4 n_f; a row homozygous for state 0 (0x02), random rows with
    and without missing entries."""
    s = 4
    say("fp4 bound multi", n_f)
    rand = synth.multi_hw(4, n_f, s, seed=8, missing=0.01)
    ld = rand.shape[1]
    const = np.zeros((3, ld), dtype=np.uint8)
    const[0, :n_f] = 0x80
    const[1, :n_f] = 0x80
    const[2, :n_f] = 0x02
    v = np.ascontiguousarray(np.concatenate([const, rand]))
    t, c, _ = ccc.ccc_2way_multi(dev(v), n_f, s)
    sync()
    ot, oc = oracle.multi_two_way(v, n_f, s)
    assert_tables_equal(host(t), ot)
    assert_ccc_close(host(c), oc)
    assert int(ot.max()) == 4 * n_f
