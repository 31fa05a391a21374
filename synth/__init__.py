"""Seeded synthetic genotype inputs in the packed 2-bit row layout.

This package draws and packs inputs only; it holds no part of the correlation
method.  The CPU oracle (``oracle/``) and the GPU library
(``paper_1705_08213_amd``) both consume its output and neither imports the
other.

Packed layout: ``uint8 v[n_v][ld]``, ``ld % 16 == 0``, ``ld >= ceil(n_f/4)``;
field ``q`` of vector ``i`` is at bits ``2*(q%4)`` (low) and ``2*(q%4)+1``
(high) of byte ``i*ld + q//4``.  The code is the allele pair, high bit first:
``0b00`` = (0,0), ``0b01`` = (0,1), ``0b11`` = (1,1), ``0b10`` = missing.
Bits past ``n_f`` are padding; by default they are filled with random garbage
so that every consumer is tested for ignoring them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")

CODE_00, CODE_01, CODE_MISSING, CODE_11 = 0, 1, 2, 3
PAD_ZERO, PAD_GARBAGE = 0, 1

# The five synthetic workloads (shapes, value distributions, missing rates).
CONFIGS = {
    "c1_2way_small": dict(kind="2way", gen="uniform", n_v=512, n_f=1000, missing=0.0, seed=0),
    "c2_2way_large": dict(kind="2way", gen="beta_hw", n_v=32768, n_f=65536, missing=0.01, seed=0),
    "c3_3way": dict(kind="3way", gen="beta_hw", n_v=2048, n_f=16384, missing=0.005, seed=0),
    "c4_batched": dict(kind="many", gen="beta_hw", n_probs=64, v_lo=256, v_hi=8192,
                       f_lo=1000, f_hi=50000, missing=0.01, seed=0),
    "c5_block": dict(kind="block", gen="beta_hw", n_a=16384, n_b=16384, n_f=131072,
                     chunk=16384, missing=0.02, seed=0),
}


def build() -> None:
    """Compile libsynth.so with gcc (host code only)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", _SRC, "-o", _SO, "-lm"]
    subprocess.run(cmd, check=True)


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i64, u64, dbl, ptr, cint = (ctypes.c_int64, ctypes.c_uint64, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_int)
        lib.synth_uniform.argtypes = [ptr, i64, i64, i64, u64, dbl, cint]
        lib.synth_beta_hw.argtypes = [ptr, i64, i64, i64, u64, dbl, cint]
        lib.synth_placement.argtypes = [ptr, i64, i64, i64, ptr, u64, cint]
        lib.synth_constant.argtypes = [ptr, i64, i64, i64, ptr, u64, cint]
        lib.synth_batch_sizes.argtypes = [i64, u64, i64, i64, i64, i64, ptr, ptr]
        lib.synth_weights.argtypes = [ptr, i64, u64, u64]
        lib.synth_beta_half.argtypes = [u64, i64]
        lib.synth_beta_half.restype = dbl
        lib.synth_multi_hw.argtypes = [ptr, i64, i64, i64, cint, u64, dbl, cint]
        for f in (lib.synth_uniform, lib.synth_beta_hw, lib.synth_placement, lib.synth_constant,
                  lib.synth_batch_sizes, lib.synth_weights, lib.synth_multi_hw):
            f.restype = None
        _lib_handle = lib
    return _lib_handle


def ld_for(n_f: int, extra: int = 0) -> int:
    """Smallest legal row stride (a multiple of 16 bytes, at least 16), plus
    ``extra`` further 16-byte units."""
    nb = (n_f + 3) // 4
    return max(16, (nb + 15) // 16 * 16) + 16 * extra


def _alloc(n_v: int, ld: int) -> np.ndarray:
    return np.zeros((n_v, ld), dtype=np.uint8)


def _pad(pad) -> int:
    return {"zero": PAD_ZERO, "garbage": PAD_GARBAGE, 0: 0, 1: 1}[pad]


def uniform(n_v, n_f, seed=0, missing=0.0, ld=None, pad="garbage") -> np.ndarray:
    """Genotypes uniform over {00,01,11}; each entry missing with prob. ``missing``."""
    ld = ld_for(n_f) if ld is None else ld
    v = _alloc(n_v, ld)
    if n_v:
        _lib().synth_uniform(v.ctypes.data, n_v, n_f, ld, seed, float(missing), _pad(pad))
    return v


def beta_hw(n_v, n_f, seed=0, missing=0.0, ld=None, pad="garbage", out=None) -> np.ndarray:
    """Per-vector p ~ Beta(1/2,1/2); Hardy-Weinberg genotypes; then missing."""
    ld = ld_for(n_f) if ld is None else ld
    v = _alloc(n_v, ld) if out is None else out
    assert v.shape == (n_v, ld) and v.dtype == np.uint8 and v.flags.c_contiguous
    if n_v:
        _lib().synth_beta_hw(v.ctypes.data, n_v, n_f, ld, seed, float(missing), _pad(pad))
    return v


def beta_half(seed: int, i: int) -> float:
    """The allele-0 frequency drawn for vector ``i``."""
    return _lib().synth_beta_half(seed, i)


def placement(s, n_f, seed=0, ld=None, pad="garbage") -> np.ndarray:
    """Vector i holds 11 where q % s[i] == 0, else 00."""
    s = np.ascontiguousarray(s, dtype=np.int64)
    assert (s >= 1).all()
    ld = ld_for(n_f) if ld is None else ld
    v = _alloc(len(s), ld)
    if len(s):
        _lib().synth_placement(v.ctypes.data, len(s), n_f, ld, s.ctypes.data, seed, _pad(pad))
    return v


def constant(codes, n_f, seed=0, ld=None, pad="garbage") -> np.ndarray:
    """Vector i holds the code ``codes[i]`` in every field."""
    codes = np.ascontiguousarray(codes, dtype=np.uint8)
    ld = ld_for(n_f) if ld is None else ld
    v = _alloc(len(codes), ld)
    if len(codes):
        _lib().synth_constant(v.ctypes.data, len(codes), n_f, ld, codes.ctypes.data, seed,
                              _pad(pad))
    return v


def pack_codes(codes: np.ndarray, ld=None, pad_value=0) -> np.ndarray:
    """Pack an explicit ``[n_v, n_f]`` matrix of 2-bit codes (values 0..3).
    Padding fields get ``pad_value`` (a code, or -1 for random garbage)."""
    codes = np.asarray(codes, dtype=np.uint8)
    n_v, n_f = codes.shape
    ld = ld_for(n_f) if ld is None else ld
    full = np.zeros((n_v, ld * 4), dtype=np.uint8)
    if pad_value == -1:
        rng = np.random.default_rng(12345)
        full[:] = rng.integers(0, 4, size=full.shape, dtype=np.uint8)
    else:
        full[:] = pad_value & 3
    full[:, :n_f] = codes & 3
    q = full.reshape(n_v, ld, 4).astype(np.uint32)
    packed = q[:, :, 0] | (q[:, :, 1] << 2) | (q[:, :, 2] << 4) | (q[:, :, 3] << 6)
    return packed.astype(np.uint8)


def ld_multi(n_f: int, extra: int = 0) -> int:
    """Smallest legal row stride of the one-byte multi-allelic layout (a
    multiple of 16 bytes, at least 16), plus ``extra`` 16-byte units."""
    return (max(1, (n_f + 15) // 16) + extra) * 16


def multi_hw(n_v, n_f, s, seed=0, missing=0.0, ld=None, pad="garbage") -> np.ndarray:
    """Multi-allelic genotypes with ``s`` (2..4) states per marker in the
    one-byte count layout (bits 2a..2a+1 = copies of state a; 0 = missing):
    per-vector frequencies from normalised sin^2 weights, Hardy-Weinberg
    pairs, then missing with probability ``missing``."""
    if not 2 <= s <= 4:
        raise ValueError("s must be 2, 3 or 4")
    ld = ld_multi(n_f) if ld is None else ld
    v = _alloc(n_v, ld)
    if n_v:
        _lib().synth_multi_hw(v.ctypes.data, n_v, n_f, ld, s, seed, missing, _pad(pad))
    return v


def pack_alleles(a1: np.ndarray, a2: np.ndarray, ld=None, pad="garbage") -> np.ndarray:
    """One-byte count layout from explicit ``[n_v, n_f]`` allele indices (the
    two alleles of each entry, values 0..3; -1 in either marks a missing
    entry)."""
    a1 = np.asarray(a1, dtype=np.int64)
    a2 = np.asarray(a2, dtype=np.int64)
    n_v, n_f = a1.shape
    ld = ld_multi(n_f) if ld is None else ld
    out = np.zeros((n_v, ld), dtype=np.uint8)
    if pad == "garbage":
        out[:] = np.random.default_rng(4321).integers(0, 256, size=out.shape, dtype=np.uint8)
    else:
        out[:] = 0
    miss = (a1 < 0) | (a2 < 0)
    byte = (np.left_shift(1, 2 * np.clip(a1, 0, 3)) + np.left_shift(1, 2 * np.clip(a2, 0, 3)))
    out[:, :n_f] = np.where(miss, 0, byte).astype(np.uint8)
    return out


def batch_sizes(n_probs, seed=0, v_lo=256, v_hi=8192, f_lo=1000, f_hi=50000):
    """(n_v, n_f) per problem: n_v log-uniform in [v_lo, v_hi], n_f uniform in
    [f_lo, f_hi]."""
    nv = np.zeros(n_probs, dtype=np.int64)
    nf = np.zeros(n_probs, dtype=np.int64)
    _lib().synth_batch_sizes(n_probs, seed, v_lo, v_hi, f_lo, f_hi, nv.ctypes.data,
                             nf.ctypes.data)
    return nv, nf


def weights(n, seed=0, tag=0) -> np.ndarray:
    """Random uint64 weights in [0, 2^61-1) for whole-output checksums."""
    w = np.zeros(n, dtype=np.uint64)
    if n:
        _lib().synth_weights(w.ctypes.data, n, seed, tag)
    return w


def make_config_input(name: str, **overrides):
    """Packed input(s) for one of the named synthetic workloads."""
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    gen = uniform if cfg["gen"] == "uniform" else beta_hw
    if cfg["kind"] in ("2way", "3way"):
        return gen(cfg["n_v"], cfg["n_f"], seed=cfg["seed"], missing=cfg["missing"])
    raise ValueError("use the kind-specific helpers for " + name)
