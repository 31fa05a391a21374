"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np


def dev(v: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(v)).cuda()


def host(t):
    return t.cpu().numpy()


def say(*args):
    """Name the case before each GPU step (flushed, so a lost box still shows it)."""
    print("[gpu-case]", *args, flush=True)
    sys.stdout.flush()


def assert_ccc_close(got: np.ndarray, want: np.ndarray, rtol=1e-12):
    """|g - o| <= rtol * max(|g|, |o|) elementwise; exact zeros must match."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    diff = np.abs(got - want)
    scale = np.maximum(np.abs(got), np.abs(want))
    bad = diff > rtol * scale
    bad |= (want == 0) != (got == 0)
    if bad.any():
        idx = np.argwhere(bad)[:5]
        raise AssertionError(f"{int(bad.sum())} CCC values off, first at {idx.tolist()}: "
                             f"got {got[bad][:5]} want {want[bad][:5]}")


def assert_ccc_identical(got: np.ndarray, want: np.ndarray):
    """The same doubles bit for bit (the epilogue rounds every quotient and
    product as the oracle's plain formula does)."""
    got = np.ascontiguousarray(got, dtype=np.float64)
    want = np.ascontiguousarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    diff = got.view(np.uint64) != want.view(np.uint64)
    if diff.any():
        idx = np.argwhere(diff)[:5]
        raise AssertionError(f"{int(diff.sum())} CCC values not bit-identical, first at "
                             f"{idx.tolist()}: got {got[diff][:5]!r} want {want[diff][:5]!r}")


def assert_tables_equal(got: np.ndarray, want: np.ndarray):
    got = np.asarray(got).astype(np.int64)
    want = np.asarray(want).astype(np.int64)
    assert got.shape == want.shape, (got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)[:5]
        raise AssertionError(f"{int((got != want).sum())} table entries differ, first at "
                             f"{bad.tolist()}: got {got[tuple(bad.T)]} want {want[tuple(bad.T)]}")


# The computation forms the parity tests run: the popcount path and the MFMA
# path with each operand format forced (fp4 and int8 both run on multi-tile
# problems, whatever size would pick by default).
FORMS = ["popcount", "fp4", "int8"]
MFMA_FORMS = ["fp4", "int8"]


def form_kw(form: str) -> dict:
    """Keyword arguments of a binding call for one of FORMS."""
    if form == "popcount":
        return dict(path="popcount")
    return dict(path="mfma", operands=form)
