"""MI355X (gfx950) Custom Correlation Coefficient tallies: Python binding.

Thin ctypes layer over ``libccc.so`` (C ABI in ``include/ccc.h``): it checks
tensor dtypes/devices, allocates output tensors through PyTorch when the
caller passes none, passes raw device pointers and the current HIP stream, and
turns negative status codes into :class:`CccError`.  Every step of the
computation runs in the library's HIP kernels; there is no fallback.

Functions carry the C names: :func:`ccc_2way`, :func:`ccc_3way`,
:func:`ccc_2way_block`, :func:`ccc_2way_many`, :func:`ccc_3way_noalloc`, ...
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libccc.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "ccc.h")

CCC_OK, CCC_ERR_ARG, CCC_ERR_RANGE, CCC_ERR_ALIGN = 0, -1, -2, -3
CCC_ERR_HIP, CCC_ERR_NOMEM, CCC_ERR_UNSUPPORTED = -4, -5, -6
CCC_PATH_AUTO, CCC_PATH_POPCOUNT, CCC_PATH_MFMA = 0, 1, 2
CCC_ACCUMULATE, CCC_FINALIZE = 1, 2
CCC_OPERANDS_AUTO, CCC_OPERANDS_FP4, CCC_OPERANDS_INT8 = 0, 4, 8
GAMMA = 2.0 / 3.0

_PATHS = {"auto": CCC_PATH_AUTO, "popcount": CCC_PATH_POPCOUNT, "mfma": CCC_PATH_MFMA,
          CCC_PATH_AUTO: CCC_PATH_AUTO, CCC_PATH_POPCOUNT: CCC_PATH_POPCOUNT,
          CCC_PATH_MFMA: CCC_PATH_MFMA}
_OPERANDS = {"auto": CCC_OPERANDS_AUTO, "fp4": CCC_OPERANDS_FP4, "int8": CCC_OPERANDS_INT8}


class CccError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_string(status)} (status {status})")


class ccc_opts(ctypes.Structure):
    _fields_ = [("path", ctypes.c_int), ("gamma", ctypes.c_double), ("flags", ctypes.c_uint),
                ("operands", ctypes.c_int)]


class ccc_selection(ctypes.Structure):
    _fields_ = [("index", ctypes.c_void_p), ("ccc", ctypes.c_void_p), ("tables", ctypes.c_void_p),
                ("cap", ctypes.c_int64), ("count", ctypes.c_void_p)]


class ccc_problem(ctypes.Structure):
    _fields_ = [("v", ctypes.c_void_p), ("n_v", ctypes.c_int64), ("n_f", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("tables", ctypes.c_void_p), ("ccc", ctypes.c_void_p),
                ("counts", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded libccc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1705_08213_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, cint = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int
        opts_p = ctypes.POINTER(ccc_opts)
        L.ccc_2way.argtypes = [vp, i64, i64, i64, vp, vp, vp, opts_p, vp]
        L.ccc_3way.argtypes = [vp, i64, i64, i64, vp, vp, vp, opts_p, vp]
        L.ccc_3way_noalloc.argtypes = [vp, i64, i64, i64, vp, vp, vp, opts_p, vp]
        L.ccc_2way_block.argtypes = [vp, i64, i64, vp, i64, i64, i64, vp, vp, vp, vp, opts_p, vp]
        L.ccc_2way_many.argtypes = [ctypes.POINTER(ccc_problem), cint, opts_p, vp]
        L.ccc_2way_rows.argtypes = [vp, i64, i64, i64, i64, i64, vp, vp, vp, opts_p, vp]
        L.ccc_3way_rows.argtypes = [vp, i64, i64, i64, i64, i64, vp, vp, vp, opts_p, vp]
        L.ccc_2way_multi.argtypes = [vp, i64, i64, i64, cint, vp, vp, vp, opts_p, vp]
        sel_p = ctypes.POINTER(ccc_selection)
        L.ccc_2way_select.argtypes = [vp, i64, i64, i64, ctypes.c_double, sel_p, vp, opts_p, vp]
        L.ccc_3way_select.argtypes = [vp, i64, i64, i64, ctypes.c_double, sel_p, vp, opts_p, vp]
        for f in (L.ccc_2way, L.ccc_3way, L.ccc_3way_noalloc, L.ccc_2way_block, L.ccc_2way_many, L.ccc_2way_rows,
                  L.ccc_3way_rows, L.ccc_2way_select, L.ccc_3way_select, L.ccc_2way_multi):
            f.restype = cint
        L.ccc_timing_enable.argtypes = [cint]
        L.ccc_timing_query.argtypes = [ctypes.c_char_p, ctypes.POINTER(cint)]
        L.ccc_timing_query.restype = ctypes.c_double
        L.ccc_status_string.argtypes = [cint]
        L.ccc_status_string.restype = ctypes.c_char_p
        L.ccc_version.restype = cint
        L.ccc_mfma_operands.argtypes = [i64]
        L.ccc_mfma_operands.restype = cint
        L.ccc_default_opts.restype = ccc_opts
        L.ccc_release_workspace.restype = None
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions declared in include/ccc.h."""
    text = open(HEADER_PATH).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ccc_[a-z0-9_]+)\s*\(", text)))


def status_string(status: int) -> str:
    return lib().ccc_status_string(status).decode()


def version() -> int:
    return lib().ccc_version()


def mfma_operands(n_f: int) -> str:
    """Operand format of an MFMA call over n_f fields: "fp4" or "int8"."""
    r = lib().ccc_mfma_operands(n_f)
    _raise(r if r < 0 else 0, "ccc_mfma_operands")
    return {4: "fp4", 8: "int8"}[r]


def release_workspace() -> None:
    lib().ccc_release_workspace()


def make_opts(path="auto", gamma=GAMMA, flags=0, operands="auto") -> ccc_opts:
    """Options struct; ``path`` ("auto", "popcount", "mfma") and ``operands``
    ("auto", "fp4", "int8": the MFMA operand format) are names or raw integers
    (passed through, so the library's own validation can be exercised)."""
    p = _PATHS[path] if isinstance(path, str) else int(path)
    o = _OPERANDS[operands] if isinstance(operands, str) else int(operands)
    return ccc_opts(p, float(gamma), int(flags), o)


# ---------------------------------------------------------------------------
# torch-facing wrappers
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_input(v, name="v"):
    torch = _torch()
    if not (isinstance(v, torch.Tensor) and v.is_cuda and v.dtype == torch.uint8 and v.dim() == 2
            and v.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous 2-D uint8 CUDA tensor [n, ld]")


def _check_out(t, shape, dtype, name):
    torch = _torch()
    if t is None:
        return
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()
            and tuple(t.shape) == tuple(shape)):
        raise TypeError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}")


def _raise(st, where):
    if st != CCC_OK:
        raise CccError(st, where)


def n_pairs(n: int) -> int:
    return n * (n - 1) // 2 if n >= 2 else 0


def n_triples(n: int) -> int:
    return n * (n - 1) * (n - 2) // 6 if n >= 3 else 0


def ccc_2way(v, n_f, tables=None, ccc=None, counts=None, path="auto", gamma=GAMMA,
             want_tables=True, want_ccc=True, stream=None, operands="auto"):
    """All pairs i<j: returns (tables int32 [P,4], ccc float64 [P,4], counts int32 [n_v,4])."""
    torch = _torch()
    _check_input(v)
    n_v, ld = v.shape
    P = n_pairs(n_v)
    dev = v.device
    if tables is None and want_tables:
        tables = torch.empty((P, 4), dtype=torch.int32, device=dev)
    if ccc is None and want_ccc:
        ccc = torch.empty((P, 4), dtype=torch.float64, device=dev)
    if counts is None:
        counts = torch.empty((n_v, 4), dtype=torch.int32, device=dev)
    _check_out(tables, (P, 4), torch.int32, "tables")
    _check_out(ccc, (P, 4), torch.float64, "ccc")
    _check_out(counts, (n_v, 4), torch.int32, "counts")
    o = make_opts(path, gamma, operands=operands)
    st = lib().ccc_2way(_ptr(v), n_v, n_f, ld, _ptr(tables), _ptr(ccc), _ptr(counts),
                        ctypes.byref(o), _stream(stream))
    _raise(st, "ccc_2way")
    return tables, ccc, counts


def ccc_2way_multi(v, n_f, s, tables=None, ccc=None, counts=None, path="auto", gamma=GAMMA,
                   want_tables=True, want_ccc=True, stream=None, operands="auto"):
    """Multi-allelic pairs i<j over s = 2..4 states (one byte per field, bits
    2a..2a+1 = copies of state a, 0 = missing): returns (tables int32 [P, s*s],
    ccc float64 [P, s*s], counts int32 [n_v, 8])."""
    torch = _torch()
    _check_input(v)
    n_v, ld = v.shape
    P = n_pairs(n_v)
    ss = s * s
    dev = v.device
    if tables is None and want_tables:
        tables = torch.empty((P, ss), dtype=torch.int32, device=dev)
    if ccc is None and want_ccc:
        ccc = torch.empty((P, ss), dtype=torch.float64, device=dev)
    if counts is None:
        counts = torch.empty((n_v, 8), dtype=torch.int32, device=dev)
    _check_out(tables, (P, ss), torch.int32, "tables")
    _check_out(ccc, (P, ss), torch.float64, "ccc")
    _check_out(counts, (n_v, 8), torch.int32, "counts")
    o = make_opts(path, gamma, operands=operands)
    st = lib().ccc_2way_multi(_ptr(v), n_v, n_f, ld, s, _ptr(tables), _ptr(ccc), _ptr(counts),
                              ctypes.byref(o), _stream(stream))
    _raise(st, "ccc_2way_multi")
    return tables, ccc, counts


def ccc_3way(v, n_f, tables=None, ccc=None, counts=None, path="auto", gamma=GAMMA,
             want_tables=True, want_ccc=True, stream=None, operands="auto"):
    """All triples i<j<k: returns (tables int32 [T,8], ccc float64 [T,8], counts)."""
    return _three_way("ccc_3way", v, n_f, tables, ccc, counts, path, gamma, want_tables,
                      want_ccc, stream, operands)


def ccc_3way_noalloc(v, n_f, tables=None, ccc=None, counts=None, path="auto", gamma=GAMMA,
                     want_tables=True, want_ccc=True, stream=None, operands="auto"):
    """As :func:`ccc_3way`, through the entry point whose scratch is the
    library's fixed per-device array (no device allocation inside the call;
    outputs the caller does not pass are still allocated here, by torch)."""
    return _three_way("ccc_3way_noalloc", v, n_f, tables, ccc, counts, path, gamma, want_tables,
                      want_ccc, stream, operands)


def _three_way(fn_name, v, n_f, tables, ccc, counts, path, gamma, want_tables, want_ccc, stream,
               operands):
    torch = _torch()
    _check_input(v)
    n_v, ld = v.shape
    T = n_triples(n_v)
    dev = v.device
    if tables is None and want_tables:
        tables = torch.empty((T, 8), dtype=torch.int32, device=dev)
    if ccc is None and want_ccc:
        ccc = torch.empty((T, 8), dtype=torch.float64, device=dev)
    if counts is None:
        counts = torch.empty((n_v, 4), dtype=torch.int32, device=dev)
    _check_out(tables, (T, 8), torch.int32, "tables")
    _check_out(ccc, (T, 8), torch.float64, "ccc")
    _check_out(counts, (n_v, 4), torch.int32, "counts")
    o = make_opts(path, gamma, operands=operands)
    st = getattr(lib(), fn_name)(_ptr(v), n_v, n_f, ld, _ptr(tables), _ptr(ccc), _ptr(counts),
                                 ctypes.byref(o), _stream(stream))
    _raise(st, fn_name)
    return tables, ccc, counts


def pair_run_length(n_v: int, i_begin: int, i_end: int) -> int:
    """Number of pairs (i, j), i_begin <= i < i_end, i < j < n_v."""
    return sum(max(n_v - 1 - i, 0) for i in range(i_begin, min(i_end, n_v)))


def triple_run_length(n_v: int, i_begin: int, i_end: int) -> int:
    """Number of triples (i, j, k), i_begin <= i < i_end, i < j < k < n_v."""
    return sum(n_pairs(n_v - 1 - i) for i in range(i_begin, min(i_end, n_v)))


def ccc_2way_rows(v, n_f, i_begin, i_end, tables=None, ccc=None, counts=None, path="auto",
                  gamma=GAMMA, want_tables=True, want_ccc=True, stream=None, operands="auto"):
    """Pairs with first index in [i_begin, i_end), in lexicographic order."""
    torch = _torch()
    _check_input(v)
    n_v, ld = v.shape
    P = pair_run_length(n_v, i_begin, i_end)
    dev = v.device
    if tables is None and want_tables:
        tables = torch.empty((P, 4), dtype=torch.int32, device=dev)
    if ccc is None and want_ccc:
        ccc = torch.empty((P, 4), dtype=torch.float64, device=dev)
    if counts is None:
        counts = torch.empty((n_v, 4), dtype=torch.int32, device=dev)
    _check_out(tables, (P, 4), torch.int32, "tables")
    _check_out(ccc, (P, 4), torch.float64, "ccc")
    o = make_opts(path, gamma, operands=operands)
    st = lib().ccc_2way_rows(_ptr(v), n_v, n_f, ld, i_begin, i_end, _ptr(tables), _ptr(ccc),
                             _ptr(counts), ctypes.byref(o), _stream(stream))
    _raise(st, "ccc_2way_rows")
    return tables, ccc, counts


def ccc_3way_rows(v, n_f, i_begin, i_end, tables=None, ccc=None, counts=None, path="auto",
                  gamma=GAMMA, want_tables=True, want_ccc=True, stream=None, operands="auto"):
    """Triples with first index in [i_begin, i_end), in lexicographic order."""
    torch = _torch()
    _check_input(v)
    n_v, ld = v.shape
    T = triple_run_length(n_v, i_begin, i_end)
    dev = v.device
    if tables is None and want_tables:
        tables = torch.empty((T, 8), dtype=torch.int32, device=dev)
    if ccc is None and want_ccc:
        ccc = torch.empty((T, 8), dtype=torch.float64, device=dev)
    if counts is None:
        counts = torch.empty((n_v, 4), dtype=torch.int32, device=dev)
    _check_out(tables, (T, 8), torch.int32, "tables")
    _check_out(ccc, (T, 8), torch.float64, "ccc")
    o = make_opts(path, gamma, operands=operands)
    st = lib().ccc_3way_rows(_ptr(v), n_v, n_f, ld, i_begin, i_end, _ptr(tables), _ptr(ccc),
                             _ptr(counts), ctypes.byref(o), _stream(stream))
    _raise(st, "ccc_3way_rows")
    return tables, ccc, counts


def _select(fn_name, width, v, n_f, threshold, cap, with_tables, counts, path, gamma, stream,
            operands="auto"):
    torch = _torch()
    _check_input(v)
    n_v, ld = v.shape
    dev = v.device
    index = torch.empty((max(cap, 1),), dtype=torch.int64, device=dev)
    cc = torch.empty((max(cap, 1), width), dtype=torch.float64, device=dev)
    tables = torch.empty((max(cap, 1), width), dtype=torch.int32, device=dev) if with_tables else None
    count = torch.zeros((2,), dtype=torch.int64, device=dev)  # 16-byte aligned counter
    if counts is None:
        counts = torch.empty((n_v, 4), dtype=torch.int32, device=dev)
    sel = ccc_selection(index.data_ptr(), cc.data_ptr(),
                        tables.data_ptr() if tables is not None else None, cap, count.data_ptr())
    o = make_opts(path, gamma, operands=operands)
    st = getattr(lib(), fn_name)(_ptr(v), n_v, n_f, ld, float(threshold), ctypes.byref(sel),
                                 _ptr(counts), ctypes.byref(o), _stream(stream))
    _raise(st, fn_name)
    n = int(count[0].item())
    k = min(n, cap)
    return n, index[:k], cc[:k], (tables[:k] if tables is not None else None)


def ccc_2way_select(v, n_f, threshold, cap, with_tables=True, counts=None, path="auto",
                    gamma=GAMMA, stream=None, operands="auto"):
    """Pairs with some CCC value >= threshold: (number found, pair index [k], CCC [k, 4],
    tables [k, 4]) with k = min(found, cap), in unspecified order.  Synchronises to read
    the count."""
    return _select("ccc_2way_select", 4, v, n_f, threshold, cap, with_tables, counts, path,
                   gamma, stream, operands)


def ccc_3way_select(v, n_f, threshold, cap, with_tables=True, counts=None, path="auto",
                    gamma=GAMMA, stream=None, operands="auto"):
    """Triples with some CCC value >= threshold (see ccc_2way_select)."""
    return _select("ccc_3way_select", 8, v, n_f, threshold, cap, with_tables, counts, path,
                   gamma, stream, operands)


def ccc_2way_block(va, vb, n_f, tables, counts_a, counts_b, ccc=None, accumulate=False,
                   finalize=True, path="auto", gamma=GAMMA, stream=None, field_offset=0,
                   operands="auto"):
    """Every (i in A, j in B) over one field chunk; tables/counts are the
    running state.  ``field_offset`` (bytes, a multiple of 16) selects the
    chunk inside wider rows: the chunk starts at byte ``field_offset`` of each
    row and the row stride stays ``v.shape[1]``."""
    torch = _torch()
    _check_input(va, "va")
    _check_input(vb, "vb")
    n_a, lda = va.shape
    n_b, ldb = vb.shape
    if field_offset % 16:
        raise ValueError("field_offset must be a multiple of 16 bytes")
    _check_out(tables, (n_a, n_b, 4), torch.int32, "tables")
    _check_out(counts_a, (n_a, 4), torch.int32, "counts_a")
    _check_out(counts_b, (n_b, 4), torch.int32, "counts_b")
    _check_out(ccc, (n_a, n_b, 4), torch.float64, "ccc")
    flags = (CCC_ACCUMULATE if accumulate else 0) | (CCC_FINALIZE if finalize else 0)
    o = make_opts(path, gamma, flags, operands)
    pa = ctypes.c_void_p(va.data_ptr() + field_offset)
    pb = ctypes.c_void_p(vb.data_ptr() + field_offset)
    st = lib().ccc_2way_block(pa, n_a, lda, pb, n_b, ldb, n_f, _ptr(tables), _ptr(counts_a),
                              _ptr(counts_b), _ptr(ccc), ctypes.byref(o), _stream(stream))
    _raise(st, "ccc_2way_block")
    return tables, ccc


def ccc_2way_many(problems, path="auto", gamma=GAMMA, stream=None, operands="auto"):
    """``problems``: sequence of dicts with keys v, n_f and optional tables,
    ccc, counts (outputs are allocated when absent).  Returns the list of
    (tables, ccc, counts)."""
    torch = _torch()
    arr = (ccc_problem * max(len(problems), 1))()
    outs = []
    for k, p in enumerate(problems):
        v = p["v"]
        _check_input(v)
        n_v, ld = v.shape
        P = n_pairs(n_v)
        t = p.get("tables")
        c = p.get("ccc")
        cnt = p.get("counts")
        if t is None and p.get("want_tables", True):
            t = torch.empty((P, 4), dtype=torch.int32, device=v.device)
        if c is None and p.get("want_ccc", True):
            c = torch.empty((P, 4), dtype=torch.float64, device=v.device)
        if cnt is None:
            cnt = torch.empty((n_v, 4), dtype=torch.int32, device=v.device)
        _check_out(t, (P, 4), torch.int32, "tables")
        _check_out(c, (P, 4), torch.float64, "ccc")
        _check_out(cnt, (n_v, 4), torch.int32, "counts")
        arr[k] = ccc_problem(v.data_ptr(), n_v, int(p["n_f"]), ld,
                             t.data_ptr() if t is not None else None,
                             c.data_ptr() if c is not None else None, cnt.data_ptr())
        outs.append((t, c, cnt))
    o = make_opts(path, gamma, operands=operands)
    st = lib().ccc_2way_many(arr, len(problems), ctypes.byref(o), _stream(stream))
    _raise(st, "ccc_2way_many")
    return outs
