// Host-side run of the library's C ABI without a GPU, built with
// AddressSanitizer and UndefinedBehaviorSanitizer on the host code (the
// library sources compiled host-only).  Every argument-validation path of
// every entry point is taken with fake device pointers (validation runs
// before any HIP call, so nothing is dereferenced), the empty problems that
// return without work, and the batched entry point's host planning (tune
// table parse, per-problem descriptors, largest-first work list, cache key)
// up to its first device allocation, which fails cleanly without a GPU.
// Prints "ok <checks>" and exits 0, or names the first failure.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "../../include/ccc.h"

static int g_checks = 0;

#define EXPECT(expr, want)                                                               \
  do {                                                                                   \
    const int got_ = (expr);                                                             \
    ++g_checks;                                                                          \
    if (got_ != (want)) {                                                                \
      printf("FAIL line %d: %s returned %d, want %d\n", __LINE__, #expr, got_, (want)); \
      exit(1);                                                                           \
    }                                                                                    \
  } while (0)

#define EXPECT_ANY2(expr, w1, w2)                                                        \
  do {                                                                                   \
    const int got_ = (expr);                                                             \
    ++g_checks;                                                                          \
    if (got_ != (w1) && got_ != (w2)) {                                                  \
      printf("FAIL line %d: %s returned %d\n", __LINE__, #expr, got_);                   \
      exit(1);                                                                           \
    }                                                                                    \
  } while (0)

static uint8_t* fake(uintptr_t off = 0) { return reinterpret_cast<uint8_t*>(0x10000 + off); }
template <typename T>
static T* fk(uintptr_t off = 0) {
  return reinterpret_cast<T*>(0x10000 + off);
}

static ccc_opts opts(int path, unsigned flags = 0, int operands = CCC_OPERANDS_AUTO,
                     double gamma = 2.0 / 3.0) {
  ccc_opts o = ccc_default_opts();
  o.path = path;
  o.flags = flags;
  o.operands = operands;
  o.gamma = gamma;
  return o;
}

int main() {
  const int64_t I32 = 2147483647;
  // status strings, version, defaults, operand query
  for (int s = -10; s <= 3; ++s) {
    const char* t = ccc_status_string(s);
    ++g_checks;
    if (!t || !strlen(t)) return printf("FAIL status string %d\n", s), 1;
  }
  EXPECT(ccc_version() >= 200, 1);
  EXPECT(ccc_mfma_operands(-1), CCC_ERR_ARG);
  EXPECT(ccc_mfma_operands(INT64_MAX), CCC_OPERANDS_INT8);
  EXPECT(ccc_mfma_operands(1 << 22), CCC_OPERANDS_FP4);

  const ccc_opts dflt = ccc_default_opts();
  for (int path = -1; path <= 3; ++path)
    for (int operands : {-1, 0, 3, 4, 8, 9}) {
      ccc_opts o = opts(path, 0, operands);
      const bool ok = path >= 0 && path <= 2 && (operands == 0 || operands == 4 || operands == 8) &&
                      !(path == CCC_PATH_POPCOUNT && operands != 0);
      // invalid option structs are rejected before anything else is looked at
      if (!ok) {
        EXPECT(ccc_2way(fake(), 10, 100, 32, fk<int32_t>(), fk<double>(), nullptr, &o, nullptr),
               CCC_ERR_ARG);
        EXPECT(ccc_3way(fake(), 10, 100, 32, fk<int32_t>(), fk<double>(), nullptr, &o, nullptr),
               CCC_ERR_ARG);
      }
    }
  ccc_opts nan_gamma = opts(0, 0, 0, strtod("nan", nullptr));
  EXPECT(ccc_2way(fake(), 10, 100, 32, fk<int32_t>(), fk<double>(), nullptr, &nan_gamma, nullptr),
         CCC_ERR_ARG);

  // 2-way / 3-way / rows / select validation
  // way 4: the no-allocation 3-way entry point
  for (int way = 2; way <= 4; ++way) {
    auto call = [&](const uint8_t* v, int64_t n, int64_t nf, int64_t ld, int32_t* t, double* c,
                    int32_t* cnt, const ccc_opts* o) {
      return way == 2   ? ccc_2way(v, n, nf, ld, t, c, cnt, o, nullptr)
             : way == 3 ? ccc_3way(v, n, nf, ld, t, c, cnt, o, nullptr)
                        : ccc_3way_noalloc(v, n, nf, ld, t, c, cnt, o, nullptr);
    };
    int32_t* T = fk<int32_t>();
    double* C = fk<double>();
    EXPECT(call(nullptr, 10, 100, 32, T, C, nullptr, &dflt), CCC_ERR_ARG);
    EXPECT(call(fake(), -1, 100, 32, T, C, nullptr, &dflt), CCC_ERR_ARG);
    EXPECT(call(fake(), 10, -1, 32, T, C, nullptr, &dflt), CCC_ERR_ARG);
    EXPECT(call(fake(), 10, 100, 24, T, C, nullptr, &dflt), CCC_ERR_ALIGN);
    EXPECT(call(fake(), 10, 100, 16, T, C, nullptr, &dflt), CCC_ERR_ARG);
    EXPECT(call(fake(4), 10, 100, 32, T, C, nullptr, &dflt), CCC_ERR_ALIGN);
    EXPECT(call(fake(), 10, 100, 32, fk<int32_t>(8), C, nullptr, &dflt), CCC_ERR_ALIGN);
    EXPECT(call(fake(), 10, 100, 32, nullptr, nullptr, nullptr, &dflt), CCC_ERR_ARG);
    EXPECT(call(fake(), 10, 100, (int64_t(1) << 28) + 16, T, C, nullptr, &dflt), CCC_ERR_RANGE);
    EXPECT(call(fake(), 10, INT64_MAX, int64_t(1) << 28, T, C, nullptr, &dflt), CCC_ERR_ARG);
    EXPECT(call(fake(), 10, I32 / 4 + 1, int64_t(1) << 28, T, C, nullptr, &dflt), CCC_ERR_RANGE);
    ccc_opts f4 = opts(CCC_PATH_MFMA, 0, CCC_OPERANDS_FP4);
    EXPECT(call(fake(), 10, (1 << 22) + 1, (1 << 20) + 16, T, C, nullptr, &f4), CCC_ERR_RANGE);
    ccc_opts accum = opts(0, CCC_ACCUMULATE);
    EXPECT(call(fake(), 10, 100, 32, T, C, nullptr, &accum), CCC_ERR_ARG);
    EXPECT(call(nullptr, 0, 100, 32, nullptr, nullptr, nullptr, &dflt), CCC_OK);
    EXPECT(call(fake(), way == 2 ? 1 : 2, 100, 32, nullptr, nullptr, nullptr, &dflt), CCC_OK);
  }
  for (int way = 2; way <= 3; ++way) {
    auto rows = [&](int64_t n, int64_t i0, int64_t i1, int32_t* t, double* c) {
      return way == 2 ? ccc_2way_rows(fake(), n, 100, 32, i0, i1, t, c, nullptr, &dflt, nullptr)
                      : ccc_3way_rows(fake(), n, 100, 32, i0, i1, t, c, nullptr, &dflt, nullptr);
    };
    EXPECT(rows(10, -1, 5, fk<int32_t>(), fk<double>()), CCC_ERR_ARG);
    EXPECT(rows(10, 6, 5, fk<int32_t>(), fk<double>()), CCC_ERR_ARG);
    EXPECT(rows(10, 0, 11, fk<int32_t>(), fk<double>()), CCC_ERR_ARG);
    EXPECT(rows(10, 0, 5, nullptr, nullptr), CCC_ERR_ARG);
    EXPECT(rows(10, 10 - way + 1, 10, nullptr, nullptr), CCC_OK);  // no pair/triple in range
    ccc_selection good{fk<int64_t>(), fk<double>(), fk<int32_t>(), 10,
                       fk<unsigned long long>()};
    ccc_selection bads[] = {
        {nullptr, fk<double>(), fk<int32_t>(), 10, fk<unsigned long long>()},
        {fk<int64_t>(), nullptr, fk<int32_t>(), 10, fk<unsigned long long>()},
        {fk<int64_t>(), fk<double>(), fk<int32_t>(), 10, nullptr},
        {fk<int64_t>(), fk<double>(), fk<int32_t>(), -1, fk<unsigned long long>()}};
    auto sel = [&](const ccc_selection* s, double thr, int64_t n) {
      return way == 2 ? ccc_2way_select(fake(), n, 100, 32, thr, s, nullptr, &dflt, nullptr)
                      : ccc_3way_select(fake(), n, 100, 32, thr, s, nullptr, &dflt, nullptr);
    };
    EXPECT(sel(nullptr, 0.1, 10), CCC_ERR_ARG);
    EXPECT(sel(&good, strtod("inf", nullptr), 10), CCC_ERR_ARG);
    for (auto& b : bads) EXPECT(sel(&b, 0.1, 10), CCC_ERR_ARG);
    ccc_selection mis{fk<int64_t>(8), fk<double>(), fk<int32_t>(), 10, fk<unsigned long long>()};
    EXPECT(sel(&mis, 0.1, 10), CCC_ERR_ALIGN);
    EXPECT(sel(&good, 0.1, 0), CCC_OK);
  }

  // block
  auto blk = [&](const uint8_t* va, int64_t na, int64_t lda, const uint8_t* vb, int64_t nb,
                 int64_t ldb, int64_t nf, int32_t* t, int32_t* ca, int32_t* cb, double* c,
                 unsigned flags, int path = 0, int operands = 0) {
    ccc_opts o = opts(path, flags, operands);
    return ccc_2way_block(va, na, lda, vb, nb, ldb, nf, t, ca, cb, c, &o, nullptr);
  };
  int32_t* T = fk<int32_t>();
  double* C = fk<double>();
  EXPECT(blk(fake(), 8, 32, fake(), 9, 32, 100, nullptr, T, T, C, CCC_FINALIZE), CCC_ERR_ARG);
  EXPECT(blk(fake(), 8, 32, fake(), 9, 32, 100, T, nullptr, T, C, CCC_FINALIZE), CCC_ERR_ARG);
  EXPECT(blk(fake(), 8, 32, fake(), 9, 32, 100, T, T, T, nullptr, CCC_FINALIZE), CCC_ERR_ARG);
  EXPECT(blk(fake(), 8, 24, fake(), 9, 32, 100, T, T, T, C, 0), CCC_ERR_ALIGN);
  EXPECT(blk(fake(), 8, 32, fake(1), 9, 32, 100, T, T, T, C, 0), CCC_ERR_ALIGN);
  EXPECT(blk(fake(), 8, 32, fake(), 9, 32, 100, T, T, T, C, 8), CCC_ERR_ARG);
  EXPECT(blk(fake(), 8, 32, fake(), 9, 32, 100, T, T, T, C, 0, 7), CCC_ERR_ARG);
  EXPECT(blk(fake(), 8, 32, fake(), 9, (int64_t(1) << 28) + 16, 100, T, T, T, C, 0),
         CCC_ERR_RANGE);
  EXPECT(blk(fake(), 8, (1 << 20) + 16, fake(), 9, (1 << 20) + 16, (1 << 22) + 1, T, T, T, C, 0,
             CCC_PATH_MFMA, CCC_OPERANDS_FP4),
         CCC_ERR_RANGE);
  EXPECT(blk(nullptr, 0, 32, fake(), 9, 32, 100, nullptr, nullptr, nullptr, nullptr, 0), CCC_OK);

  // multi-allelic
  auto mul = [&](int64_t n, int64_t nf, int64_t ld, int s, int path = 0, unsigned flags = 0) {
    ccc_opts o = opts(path, flags);
    return ccc_2way_multi(fake(), n, nf, ld, s, T, C, nullptr, &o, nullptr);
  };
  EXPECT(mul(10, 100, 112, 1), CCC_ERR_ARG);
  EXPECT(mul(10, 100, 112, 5), CCC_ERR_ARG);
  EXPECT(mul(10, 100, 120, 3), CCC_ERR_ALIGN);
  EXPECT(mul(10, 100, 96, 3), CCC_ERR_ARG);
  EXPECT(mul(10, 100, 112, 3, CCC_PATH_POPCOUNT), CCC_ERR_UNSUPPORTED);
  EXPECT(mul(10, 100, 112, 3, 0, CCC_FINALIZE), CCC_ERR_ARG);
  EXPECT(mul(10, 100, (int64_t(1) << 28) + 16, 3), CCC_ERR_RANGE);

  // batched: validation of every problem, then (valid batches) the host
  // planning up to the first device allocation
  std::vector<ccc_problem> probs;
  uint64_t seed = 0x9E3779B97F4A7C15ull;
  auto rnd = [&](int64_t lo, int64_t hi) {
    seed = seed * 6364136223846793005ull + 1442695040888963407ull;
    return lo + (int64_t)((seed >> 33) % (uint64_t)(hi - lo + 1));
  };
  for (int k = 0; k < 64; ++k) {
    const int64_t n = rnd(0, 5000), nf = rnd(0, 60000);
    probs.push_back(ccc_problem{fake(), n, nf, ((nf + 3) / 4 + 15) / 16 * 16, T, C,
                                (k % 3) ? T : nullptr});
  }
  std::vector<ccc_problem> bad = probs;
  bad[17].ld = 24;
  EXPECT(ccc_2way_many(bad.data(), (int)bad.size(), nullptr, nullptr), CCC_ERR_ALIGN);
  bad = probs;
  bad[63].n_f = I32 / 4 + 1;
  bad[63].ld = (bad[63].n_f + 3) / 4 / 16 * 16 + 16;
  EXPECT(ccc_2way_many(bad.data(), (int)bad.size(), nullptr, nullptr), CCC_ERR_RANGE);
  EXPECT(ccc_2way_many(nullptr, 3, nullptr, nullptr), CCC_ERR_ARG);
  EXPECT(ccc_2way_many(probs.data(), 0, nullptr, nullptr), CCC_OK);
  // tune table with malformed and out-of-range lines
  const char* tune = "/tmp/ccc_abi_sanitize_tune.txt";
  if (FILE* f = fopen(tune, "w")) {
    fputs("# comment\n\n garbage line\n1024 100000 mfma 1\n999999999999999999999 5 mfma 0\n"
          "512 2 popcount 9\n-5 -5 mfma -1\n4096 60000 mfma 0\n7 7 bogus 1\n"
          "2048 4096 mfma 2 3\n8192 100 mfma 3 999\n100 100 oneshot 1\n5000 5000 oneshot 7\n",
          f);
    fclose(f);
    setenv("CCC_TUNE_FILE", tune, 1);
  }
  for (int path : {CCC_PATH_AUTO, CCC_PATH_POPCOUNT})
    for (int operands : {CCC_OPERANDS_AUTO, CCC_OPERANDS_INT8}) {
      if (path == CCC_PATH_POPCOUNT && operands) continue;
      ccc_opts o = opts(path, 0, operands);
      // without a GPU the planned batch's first allocation (or device query) fails
      EXPECT_ANY2(ccc_2way_many(probs.data(), (int)probs.size(), &o, nullptr), CCC_ERR_NOMEM,
                  CCC_ERR_HIP);
    }
  remove(tune);

  // no-allocation 3-way: scratch limit, then (valid call) the device
  // lookup of the scratch array, which fails cleanly without a GPU
  EXPECT(ccc_3way_noalloc(fake(), 400000, 100, 32, fk<int32_t>(), fk<double>(), nullptr, &dflt,
                          nullptr),
         CCC_ERR_RANGE);
  EXPECT(ccc_3way_noalloc(fake(), 10, 100, 32, fk<int32_t>(), fk<double>(), nullptr, &dflt,
                          nullptr),
         CCC_ERR_HIP);

  // timing hooks with nothing recorded
  ccc_timing_enable(1);
  ccc_timing_enable(0);
  int cnt = -1;
  ++g_checks;
  if (ccc_timing_query(nullptr, &cnt) != 0.0 || cnt != 0) return printf("FAIL timing\n"), 1;
  ccc_timing_reset();
  printf("ok %d\n", g_checks);
  return 0;
}
