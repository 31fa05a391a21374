"""The no-allocation 3-way entry point (ccc_3way_noalloc, scratch in the
library's fixed per-device array) against ccc_3way (workspace scratch) and
the CPU oracle: two calls in a row, the second on a smaller input, so that
the scratch keeps the first call's contents when the second one starts."""
import ctypes

import numpy as np
import pytest

import oracle
import oracle.brute
import paper_1705_08213_amd as ccc
import synth
from gpu_util import assert_ccc_close, assert_ccc_identical, assert_tables_equal, dev, host, say

pytestmark = pytest.mark.gpu


def _input(n_v, n_f, seed, missing_rows):
    """Beta/Hardy-Weinberg rows with no missing entry except in
    `missing_rows`, so that both the complete-data units (which read the Gram
    matrix in the scratch) and the general ones run."""
    v = synth.beta_hw(n_v, n_f, seed=seed, missing=0.0)
    codes = oracle.brute.unpack_codes(v, n_f)
    rng = np.random.default_rng(seed)
    for r in missing_rows:
        codes[r, rng.integers(0, n_f, size=3)] = 2
    return synth.pack_codes(codes, pad_value=-1)


def _call(fn_name, dv, n_f, operands, path="mfma"):
    """One call through the C ABI with caller-owned outputs and no counts
    buffer (the counts then live in the call's scratch too)."""
    import torch
    n_v, ld = dv.shape
    T = ccc.n_triples(n_v)
    tables = torch.full((T, 8), -7, dtype=torch.int32, device=dv.device)
    cc = torch.full((T, 8), -7.0, dtype=torch.float64, device=dv.device)
    o = ccc.make_opts(path, operands=operands)
    st = getattr(ccc.lib(), fn_name)(ctypes.c_void_p(dv.data_ptr()), n_v, n_f, ld,
                                     ctypes.c_void_p(tables.data_ptr()),
                                     ctypes.c_void_p(cc.data_ptr()), None, ctypes.byref(o),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == ccc.CCC_OK, ccc.status_string(st)
    torch.cuda.synchronize()
    return host(tables), host(cc)


# (n_v, n_f, rows with missing entries, operand format, path): the second
# input of each sequence is smaller than the first
SEQUENCES = [
    [(200, 3001, (5, 77, 150), "fp4", "mfma"), (90, 700, (3,), "fp4", "mfma")],
    [(160, 2050, (64, 100), "int8", "mfma"), (70, 257, (), "int8", "mfma")],
    [(130, 1000, (1, 129), "auto", "popcount"), (40, 300, (7,), "auto", "popcount")],
]


@pytest.mark.parametrize("seq", SEQUENCES, ids=["fp4", "int8", "popcount"])
def test_noalloc_3way_matches_3way_twice(seq):
    import torch
    for k, (n_v, n_f, miss, operands, path) in enumerate(seq):
        say("3way noalloc", k, n_v, n_f, operands, path)
        v = _input(n_v, n_f, seed=900 + 7 * k + n_v, missing_rows=miss)
        dv = dev(v)
        nt, nc = _call("ccc_3way_noalloc", dv, n_f, operands, path)
        wt, wc = _call("ccc_3way", dv, n_f, operands, path)
        assert_tables_equal(nt, wt)
        assert_ccc_identical(nc, wc)
        if n_v <= 200:  # the oracle in seconds
            ot, oc = oracle.three_way(v, n_f)
            assert_tables_equal(nt, ot)
            assert_ccc_close(nc, oc)
        torch.cuda.synchronize()
