"""The C ABI of libccc.so without a GPU: symbols, status codes and every
argument-validation path (validation runs before any HIP call, so these calls
enqueue nothing and touch no memory)."""
import ctypes

import pytest

import paper_1705_08213_amd as ccc

FAKE = 0x10000  # 16-byte aligned, never dereferenced by a failing call
I32MAX = 2**31 - 1


def test_library_exports_every_declared_function():
    L = ccc.lib()
    names = ccc.header_functions()
    assert {"ccc_2way", "ccc_3way", "ccc_2way_block", "ccc_2way_many",
            "ccc_status_string"} <= set(names)
    for name in names:
        assert hasattr(L, name), name


def test_status_strings_and_version():
    for st in (0, -1, -2, -3, -4, -5, -6):
        s = ccc.status_string(st)
        assert s and s != "unknown status"
    assert ccc.status_string(-99) == "unknown status"
    assert ccc.version() >= 200


def test_two_way_operand_format_query():
    # fp4 while every accumulated quarter-multiple (at most n_f) is exact in fp32
    assert ccc.mfma_operands(0) == "fp4"
    assert ccc.mfma_operands(65536) == "fp4"
    assert ccc.mfma_operands(1 << 22) == "fp4"
    assert ccc.mfma_operands((1 << 22) + 1) == "int8"
    assert ccc.lib().ccc_mfma_operands(-1) == ccc.CCC_ERR_ARG


def test_default_opts():
    o = ccc.lib().ccc_default_opts()
    assert o.path == ccc.CCC_PATH_AUTO and o.flags == 0
    assert o.gamma == 2.0 / 3.0
    assert o.operands == ccc.CCC_OPERANDS_AUTO


@pytest.mark.parametrize("fn", ["2way", "3way", "block", "multi", "many"])
def test_operand_format_option(fn):
    """Unknown formats and a format with the popcount path are argument
    errors; fp4 forced past 2^22 fields (where its fp32 sums stop being exact)
    is a range error.  All are caught before any device work."""
    L = ccc.lib()
    limit = 1 << 22

    def call(n_f, path="mfma", operands="auto"):
        o = ccc.make_opts(path, operands=operands)
        ld = (n_f + 3) // 4 // 16 * 16 + 16
        if fn == "2way":
            return L.ccc_2way(FAKE, 10, n_f, ld, FAKE, FAKE, None, ctypes.byref(o), None)
        if fn == "3way":
            return L.ccc_3way(FAKE, 10, n_f, ld, FAKE, FAKE, None, ctypes.byref(o), None)
        if fn == "block":
            o.flags = ccc.CCC_FINALIZE
            return L.ccc_2way_block(FAKE, 8, ld, FAKE, 9, ld, n_f, FAKE, FAKE, FAKE, FAKE,
                                    ctypes.byref(o), None)
        if fn == "multi":
            ldm = (n_f + 15) // 16 * 16
            return L.ccc_2way_multi(FAKE, 10, n_f, ldm, 3, FAKE, FAKE, None, ctypes.byref(o),
                                    None)
        P = ccc.ccc_problem
        arr = (P * 2)(P(FAKE, 10, 100, 32, FAKE, FAKE, FAKE),
                      P(FAKE, 10, n_f, ld, FAKE, FAKE, FAKE))
        return L.ccc_2way_many(arr, 2, ctypes.byref(o), None)

    assert call(100, operands=3) == ccc.CCC_ERR_ARG
    assert call(100, operands=-4) == ccc.CCC_ERR_ARG
    assert call(limit + 1, operands="fp4") == ccc.CCC_ERR_RANGE
    assert call(limit + 257, operands="fp4") == ccc.CCC_ERR_RANGE
    if fn != "multi":  # multi-allelic tallies have no popcount form
        assert call(100, path="popcount", operands="int8") == ccc.CCC_ERR_ARG
        assert call(100, path="popcount", operands="fp4") == ccc.CCC_ERR_ARG


def test_row_stride_and_field_count_limits():
    """ld beyond 2^28 bytes (the kernels' 32-bit block offsets) is a range
    error; so is any n_f whose table entries could pass INT32_MAX, even one so
    large that 4 n_f or 8 n_f would overflow int64."""
    big_ld = (1 << 28) + 16
    assert call2(ld=big_ld) == ccc.CCC_ERR_RANGE
    assert call3(ld=big_ld) == ccc.CCC_ERR_RANGE
    assert callb(lda=big_ld) == ccc.CCC_ERR_RANGE
    assert callb(ldb=big_ld) == ccc.CCC_ERR_RANGE
    assert call2(ld=1 << 28, n_f=4 << 28) == ccc.CCC_ERR_RANGE  # 4 n_f = 2^32
    for huge in ((1 << 62) + 1, (1 << 63) - 1, 1 << 61):
        # ld cannot hold such rows: the stride check fires before any product of n_f
        assert call2(n_f=huge, ld=1 << 28) == ccc.CCC_ERR_ARG
        assert call3(n_f=huge, ld=1 << 28) == ccc.CCC_ERR_ARG
    L = ccc.lib()
    o = ccc.make_opts()
    assert L.ccc_2way_multi(FAKE, 10, 100, big_ld, 3, FAKE, FAKE, None, ctypes.byref(o),
                            None) == ccc.CCC_ERR_RANGE
    assert L.ccc_2way_multi(FAKE, 10, (1 << 62) + 1, 1 << 28, 3, FAKE, FAKE, None,
                            ctypes.byref(o), None) == ccc.CCC_ERR_ARG
    P = ccc.ccc_problem
    arr = (P * 2)(P(FAKE, 10, 100, 32, FAKE, FAKE, FAKE),
                  P(FAKE, 10, 100, big_ld, FAKE, FAKE, FAKE))
    assert L.ccc_2way_many(arr, 2, None, None) == ccc.CCC_ERR_RANGE


def call2(v=FAKE, n_v=10, n_f=100, ld=32, tables=FAKE, cc=FAKE, counts=None, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return ccc.lib().ccc_2way(v, n_v, n_f, ld, tables, cc, counts, o, None)


def call3(v=FAKE, n_v=10, n_f=100, ld=32, tables=FAKE, cc=FAKE, counts=None, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return ccc.lib().ccc_3way(v, n_v, n_f, ld, tables, cc, counts, o, None)


def call3n(v=FAKE, n_v=10, n_f=100, ld=32, tables=FAKE, cc=FAKE, counts=None, opts=None):
    o = ctypes.byref(opts) if opts is not None else None
    return ccc.lib().ccc_3way_noalloc(v, n_v, n_f, ld, tables, cc, counts, o, None)


def callb(va=FAKE, n_a=8, lda=32, vb=FAKE, n_b=9, ldb=32, n_f=100, tables=FAKE, ca=FAKE,
          cb=FAKE, cc=FAKE, flags=ccc.CCC_FINALIZE, path=0):
    o = ccc.make_opts(path, flags=flags)
    return ccc.lib().ccc_2way_block(va, n_a, lda, vb, n_b, ldb, n_f, tables, ca, cb, cc,
                                    ctypes.byref(o), None)


@pytest.mark.parametrize("fn", [call2, call3, call3n])
def test_validation_errors_common(fn):
    assert fn(v=None) == ccc.CCC_ERR_ARG
    assert fn(n_v=-1) == ccc.CCC_ERR_ARG
    assert fn(n_f=-5) == ccc.CCC_ERR_ARG
    assert fn(ld=-16) == ccc.CCC_ERR_ARG
    assert fn(ld=24) == ccc.CCC_ERR_ALIGN            # ld % 16 != 0
    assert fn(ld=16) == ccc.CCC_ERR_ARG              # ld < ceil(100/4)
    assert fn(v=FAKE + 4) == ccc.CCC_ERR_ALIGN
    assert fn(tables=FAKE + 8) == ccc.CCC_ERR_ALIGN
    assert fn(cc=FAKE + 8) == ccc.CCC_ERR_ALIGN
    assert fn(counts=FAKE + 4) == ccc.CCC_ERR_ALIGN
    assert fn(tables=None, cc=None) == ccc.CCC_ERR_ARG
    assert fn(opts=ccc.make_opts(3)) == ccc.CCC_ERR_ARG
    assert fn(opts=ccc.make_opts(0, float("nan"))) == ccc.CCC_ERR_ARG
    assert fn(opts=ccc.make_opts(0, flags=ccc.CCC_ACCUMULATE)) == ccc.CCC_ERR_ARG
    assert fn(opts=ccc.make_opts(0, flags=64)) == ccc.CCC_ERR_ARG


def test_range_limits():
    big = I32MAX // 4 + 1  # 4 * n_f exceeds INT32_MAX
    assert call2(n_f=big, ld=(big + 3) // 4 // 16 * 16 + 16) == ccc.CCC_ERR_RANGE
    ok_2way_but_not_3way = I32MAX // 8 + 1
    ld = (ok_2way_but_not_3way + 3) // 4 // 16 * 16 + 16
    assert call3(n_f=ok_2way_but_not_3way, ld=ld) == ccc.CCC_ERR_RANGE
    assert callb(n_f=big, lda=(big + 3) // 4 // 16 * 16 + 16,
                 ldb=(big + 3) // 4 // 16 * 16 + 16) == ccc.CCC_ERR_RANGE


def test_noalloc_3way_validation_and_scratch_limit():
    """The no-allocation 3-way entry point validates like ccc_3way, and a
    problem whose work-unit offsets (8 bytes per tile pair of two grids of
    64-row tiles and one of 32-row tiles) cannot fit its fixed scratch is a
    range error, caught before any HIP call."""
    big = I32MAX // 8 + 1
    assert call3n(n_f=big, ld=(big + 3) // 4 // 16 * 16 + 16) == ccc.CCC_ERR_RANGE
    assert call3n(ld=(1 << 28) + 16) == ccc.CCC_ERR_RANGE
    assert call3n(n_v=2642246) == ccc.CCC_ERR_ARG  # C(n_v,3) * 8 past int64 indexing
    # 400000 rows: 6250 tiles, about 19.5 million tile pairs, 156 MB of offsets
    assert call3n(n_v=400000) == ccc.CCC_ERR_RANGE
    assert call3n(n_v=400000, counts=FAKE) == ccc.CCC_ERR_RANGE
    # 70000 rows: 1094 tiles of 64 rows and 2188 of 32 per side, 28.7 MB of offsets
    assert call3n(n_v=70000, counts=FAKE) == ccc.CCC_ERR_RANGE
    assert call3n(v=None, n_v=0) == ccc.CCC_OK
    assert call3n(n_v=2, tables=None, cc=None) == ccc.CCC_OK


def test_empty_problems_return_ok_without_work():
    assert call2(v=None, n_v=0, tables=None, cc=None) == ccc.CCC_OK
    assert call2(n_v=1, tables=None, cc=None, counts=None) == ccc.CCC_OK
    assert call3(v=None, n_v=0) == ccc.CCC_OK
    assert call3(n_v=2, tables=None, cc=None) == ccc.CCC_OK
    assert callb(n_a=0, va=None, tables=None, ca=None, cb=None, cc=None) == ccc.CCC_OK
    assert callb(n_b=0, vb=None, tables=None, ca=None, cb=None, cc=None) == ccc.CCC_OK
    assert ccc.lib().ccc_2way_many(None, 0, None, None) == ccc.CCC_OK


def test_block_validation():
    assert callb(tables=None) == ccc.CCC_ERR_ARG
    assert callb(ca=None) == ccc.CCC_ERR_ARG
    assert callb(cb=None) == ccc.CCC_ERR_ARG
    assert callb(cc=None) == ccc.CCC_ERR_ARG                    # FINALIZE needs ccc
    assert callb(lda=24) == ccc.CCC_ERR_ALIGN
    assert callb(ldb=16) == ccc.CCC_ERR_ARG
    assert callb(vb=FAKE + 1) == ccc.CCC_ERR_ALIGN
    assert callb(ca=FAKE + 4) == ccc.CCC_ERR_ALIGN
    assert callb(flags=8) == ccc.CCC_ERR_ARG
    assert callb(path=7) == ccc.CCC_ERR_ARG


def test_many_validation_checks_every_problem():
    P = ccc.ccc_problem
    good = P(FAKE, 10, 100, 32, FAKE, FAKE, FAKE)
    bad_ld = P(FAKE, 10, 100, 24, FAKE, FAKE, FAKE)
    bad_out = P(FAKE, 10, 100, 32, None, None, FAKE)
    big = I32MAX // 4 + 1
    bad_range = P(FAKE, 10, big, (big + 3) // 4 // 16 * 16 + 16, FAKE, FAKE, FAKE)
    L = ccc.lib()
    for bad, want in [(bad_ld, ccc.CCC_ERR_ALIGN), (bad_out, ccc.CCC_ERR_ARG),
                      (bad_range, ccc.CCC_ERR_RANGE)]:
        arr = (P * 3)(good, good, bad)
        assert L.ccc_2way_many(arr, 3, None, None) == want
    assert L.ccc_2way_many(None, 2, None, None) == ccc.CCC_ERR_ARG
    assert L.ccc_2way_many(None, -1, None, None) == ccc.CCC_ERR_ARG


def test_rows_and_select_validation():
    L = ccc.lib()
    o = ctypes.byref(ccc.make_opts())
    for fn in (L.ccc_2way_rows, L.ccc_3way_rows):
        assert fn(FAKE, 10, 100, 32, -1, 5, FAKE, FAKE, None, o, None) == ccc.CCC_ERR_ARG
        assert fn(FAKE, 10, 100, 32, 6, 5, FAKE, FAKE, None, o, None) == ccc.CCC_ERR_ARG
        assert fn(FAKE, 10, 100, 32, 0, 11, FAKE, FAKE, None, o, None) == ccc.CCC_ERR_ARG
        assert fn(FAKE, 10, 100, 32, 0, 5, None, None, None, o, None) == ccc.CCC_ERR_ARG
        assert fn(FAKE, 10, 100, 24, 0, 5, FAKE, FAKE, None, o, None) == ccc.CCC_ERR_ALIGN
        # an empty range needs no outputs and does no work
        assert fn(FAKE, 0, 100, 32, 0, 0, None, None, None, o, None) == ccc.CCC_OK
    S = ccc.ccc_selection
    good = S(FAKE, FAKE, FAKE, 10, FAKE)
    for fn in (L.ccc_2way_select, L.ccc_3way_select):
        assert fn(FAKE, 10, 100, 32, 0.1, None, None, o, None) == ccc.CCC_ERR_ARG
        assert fn(FAKE, 10, 100, 32, float("nan"), ctypes.byref(good), None, o,
                  None) == ccc.CCC_ERR_ARG
        for bad in (S(None, FAKE, FAKE, 10, FAKE), S(FAKE, None, FAKE, 10, FAKE),
                    S(FAKE, FAKE, FAKE, 10, None), S(FAKE, FAKE, FAKE, -1, FAKE)):
            assert fn(FAKE, 10, 100, 32, 0.1, ctypes.byref(bad), None, o, None) == ccc.CCC_ERR_ARG
        for bad in (S(FAKE + 8, FAKE, FAKE, 10, FAKE), S(FAKE, FAKE, FAKE + 4, 10, FAKE),
                    S(FAKE, FAKE, FAKE, 10, FAKE + 8)):
            assert fn(FAKE, 10, 100, 32, 0.1, ctypes.byref(bad), None, o,
                      None) == ccc.CCC_ERR_ALIGN
        assert fn(FAKE, 0, 100, 32, 0.1, ctypes.byref(good), None, o, None) == ccc.CCC_OK


def test_ranges_without_pairs_need_no_outputs():
    L = ccc.lib()
    o = ctypes.byref(ccc.make_opts())
    # the last row has no pair, the last two rows no triple: no outputs needed,
    # and with no counts requested nothing is launched
    assert L.ccc_2way_rows(FAKE, 10, 100, 32, 9, 10, None, None, None, o, None) == ccc.CCC_OK
    assert L.ccc_3way_rows(FAKE, 10, 100, 32, 8, 10, None, None, None, o, None) == ccc.CCC_OK
    assert L.ccc_2way_rows(FAKE, 10, 100, 32, 8, 10, None, None, None, o, None) == ccc.CCC_ERR_ARG


def test_multi_validation():
    L = ccc.lib()

    def callm(v=FAKE, n_v=10, n_f=100, ld=112, s=3, tables=FAKE, cc=FAKE, counts=None, path=0,
              flags=0):
        o = ccc.make_opts(path, flags=flags)
        return L.ccc_2way_multi(v, n_v, n_f, ld, s, tables, cc, counts, ctypes.byref(o), None)

    assert callm(s=1) == ccc.CCC_ERR_ARG
    assert callm(s=5) == ccc.CCC_ERR_ARG
    assert callm(ld=120) == ccc.CCC_ERR_ALIGN
    assert callm(ld=96) == ccc.CCC_ERR_ARG                 # ld < n_f
    assert callm(path=ccc.CCC_PATH_POPCOUNT) == ccc.CCC_ERR_UNSUPPORTED
    assert callm(flags=ccc.CCC_FINALIZE) == ccc.CCC_ERR_ARG
    assert callm(tables=None, cc=None) == ccc.CCC_ERR_ARG
    assert callm(v=None) == ccc.CCC_ERR_ARG
    assert callm(v=FAKE + 8) == ccc.CCC_ERR_ALIGN
    assert callm(tables=FAKE + 4) == ccc.CCC_ERR_ALIGN
    assert callm(cc=FAKE + 8) == ccc.CCC_ERR_ALIGN
    assert callm(counts=FAKE + 4) == ccc.CCC_ERR_ALIGN
    assert callm(n_v=-1) == ccc.CCC_ERR_ARG
    big = I32MAX // 4 + 1
    assert callm(n_f=big, ld=(big + 15) // 16 * 16) == ccc.CCC_ERR_RANGE
    # empty problems enqueue nothing
    assert callm(v=None, n_v=0, tables=None, cc=None) == ccc.CCC_OK
    assert callm(n_v=1, tables=None, cc=None) == ccc.CCC_OK
