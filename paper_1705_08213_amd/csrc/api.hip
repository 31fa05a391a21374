// api.hip -- the C ABI declared in include/ccc.h: argument validation, the
// per-device workspace, and dispatch to the kernels.
//
// Validation is pure host logic and runs before any HIP call, so every error
// path returns with nothing enqueued and outputs untouched.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "../../include/ccc.h"
#include "kernels.h"
#include "many.h"

namespace {

constexpr int64_t kInt32Max = 2147483647;
// Largest row stride: the kernels address a 16-row block of the input with
// 32-bit byte offsets (15 ld + 64 < 2^32).
constexpr int64_t kMaxLd = int64_t(1) << 28;
// Largest row count whose complete-data Gram matrix (4 B per entry) the
// 3-way MFMA path keeps in the workspace (4 GiB); beyond it every unit takes
// the general path.
constexpr int64_t kGramMaxRows = 32768;

struct Workspace {
  void* ptr = nullptr;
  size_t bytes = 0;
};

std::mutex g_mu;
std::vector<Workspace> g_ws;  // indexed by device ordinal

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int resolve_opts(const ccc_opts* opts, ccc_opts* out) {
  *out = ccc_default_opts();
  if (!opts) return CCC_OK;
  if (opts->path < CCC_PATH_AUTO || opts->path > CCC_PATH_MFMA) return CCC_ERR_ARG;
  if (!isfinite(opts->gamma)) return CCC_ERR_ARG;
  if (opts->flags & ~(unsigned)(CCC_ACCUMULATE | CCC_FINALIZE)) return CCC_ERR_ARG;
  if (opts->operands != CCC_OPERANDS_AUTO && opts->operands != CCC_OPERANDS_FP4 &&
      opts->operands != CCC_OPERANDS_INT8)
    return CCC_ERR_ARG;
  if (opts->path == CCC_PATH_POPCOUNT && opts->operands != CCC_OPERANDS_AUTO) return CCC_ERR_ARG;
  *out = *opts;
  return CCC_OK;
}

// fp4 operands for an MFMA call whose largest per-call field count is n_f
// (1), int8 (0), or CCC_ERR_RANGE when fp4 is forced beyond its exact range.
int use_fp4(const ccc_opts& o, int64_t n_f) {
  if (o.operands == CCC_OPERANDS_INT8) return 0;
  if (o.operands == CCC_OPERANDS_FP4) return n_f <= ccc::kF4MaxFields ? 1 : CCC_ERR_RANGE;
  return n_f <= ccc::kF4MaxFields ? 1 : 0;
}

// Table entries are at most 4 n_f (2-way) or 8 n_f (3-way): `mult` = 4 or 8.
// Compared by division first, so that no product of a huge n_f overflows.
bool fields_in_range(int64_t n_f, int64_t mult) { return n_f <= kInt32Max / mult; }

int check_input(const uint8_t* v, int64_t n, int64_t n_f, int64_t ld) {
  if (n < 0 || n_f < 0 || ld < 0) return CCC_ERR_ARG;
  if (n > kInt32Max) return CCC_ERR_ARG;
  if (ld % 16 != 0) return CCC_ERR_ALIGN;
  if (ld > kMaxLd) return CCC_ERR_RANGE;
  if (n_f / 4 >= ld + (n_f % 4 == 0)) return CCC_ERR_ARG;  // ld < ceil(n_f/4), overflow-free
  if (n > 0 && !v) return CCC_ERR_ARG;
  if (v && !aligned16(v)) return CCC_ERR_ALIGN;
  return CCC_OK;
}

}  // namespace

namespace ccc {

// Workspace of at least `bytes` on the current device (grown on demand).
int workspace(size_t bytes, void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CCC_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  Workspace& w = g_ws[dev];
  if (w.bytes < bytes) {
    if (w.ptr) {
      // the old buffer may still be in use by enqueued work
      if (hipDeviceSynchronize() != hipSuccess) return CCC_ERR_HIP;
      (void)hipFree(w.ptr);
      w.ptr = nullptr;
      w.bytes = 0;
    }
    size_t want = bytes < (1u << 20) ? (1u << 20) : bytes;
    if (hipMalloc(&w.ptr, want) != hipSuccess) {
      (void)hipGetLastError();
      return CCC_ERR_NOMEM;
    }
    w.bytes = want;
  }
  *out = w.ptr;
  return CCC_OK;
}

static int run_pair2(const Pair2Args& a, int path, hipStream_t stream) {
  hipError_t e = path == CCC_PATH_POPCOUNT ? launch_pop2(a, stream) : launch_mfma2(a, stream);
  return e == hipSuccess ? CCC_OK : CCC_ERR_HIP;
}

}  // namespace ccc

extern "C" {

ccc_opts ccc_default_opts(void) {
  ccc_opts o;
  o.path = CCC_PATH_AUTO;
  o.gamma = 2.0 / 3.0;
  o.flags = 0;
  o.operands = CCC_OPERANDS_AUTO;
  return o;
}

int ccc_version(void) { return 200; }

int ccc_mfma_operands(int64_t n_f) {
  if (n_f < 0) return CCC_ERR_ARG;
  return n_f <= ccc::kF4MaxFields ? CCC_OPERANDS_FP4 : CCC_OPERANDS_INT8;
}

const char* ccc_status_string(int status) {
  switch (status) {
    case CCC_OK: return "ok";
    case CCC_ERR_ARG: return "invalid argument";
    case CCC_ERR_RANGE: return "a table entry could exceed the int32 range";
    case CCC_ERR_ALIGN: return "pointer not 16-byte aligned or row stride not a multiple of 16";
    case CCC_ERR_HIP: return "HIP call or kernel launch failed";
    case CCC_ERR_NOMEM: return "workspace allocation failed";
    case CCC_ERR_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

}  // extern "C"

namespace {

// All 2-way variants: dense rows [i_begin, i_end) (tables/ccc) or selection.
int two_way(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i_begin,
            int64_t i_end, int32_t* tables, double* ccc, const ccc_selection* sel,
            double threshold, int32_t* counts, const ccc_opts* opts, hipStream_t stream) {
  ccc_opts o;
  int st = resolve_opts(opts, &o);
  if (st) return st;
  if (o.flags != 0) return CCC_ERR_ARG;
  if ((st = check_input(v, n_v, n_f, ld))) return st;
  if (!fields_in_range(n_f, 4)) return CCC_ERR_RANGE;
  const int f4 = o.path == CCC_PATH_POPCOUNT ? 0 : use_fp4(o, n_f);
  if (f4 < 0) return f4;
  if (i_begin < 0 || i_end < i_begin || i_end > n_v) return CCC_ERR_ARG;
  if (sel) {
    if (!sel->index || !sel->ccc || !sel->count || sel->cap < 0) return CCC_ERR_ARG;
    if (!isfinite(threshold)) return CCC_ERR_ARG;
    if (!aligned16(sel->index) || !aligned16(sel->ccc) || !aligned16(sel->tables) ||
        !aligned16(sel->count))
      return CCC_ERR_ALIGN;
  } else if ((i_end < n_v - 1 ? i_end : n_v - 1) > i_begin && !tables && !ccc) {
    return CCC_ERR_ARG;  // the range holds pairs but there is nowhere to put them
  }
  if (!aligned16(tables) || !aligned16(ccc) || !aligned16(counts)) return CCC_ERR_ALIGN;
  if (n_v == 0) return CCC_OK;
  unsigned long long* zero = sel ? sel->count : nullptr;
  const int64_t row_end = i_end < n_v - 1 ? i_end : n_v - 1;  // the last row has no pair
  if (row_end <= i_begin && !counts && !zero) return CCC_OK;  // nothing to compute or write
  if (n_v == 1) {
    if (!counts && !zero) return CCC_OK;
    if (!counts) {  // only the selection counter to clear
      void* ws = nullptr;
      if ((st = ccc::workspace(16, &ws))) return st;
      counts = static_cast<int32_t*>(ws);
    }
    return ccc::launch_count1_zero(v, ld, n_v, n_f, counts, 0, zero, stream) == hipSuccess
               ? CCC_OK
               : CCC_ERR_HIP;
  }
  // workspace: the counts (unless the caller's), then the MFMA path's
  // complete-data flag
  const size_t cnt_bytes = counts ? 0 : ((size_t)n_v * 16 + 255) / 256 * 256;
  void* ws = nullptr;
  if ((st = ccc::workspace(cnt_bytes + 256, &ws))) return st;
  int32_t* cnt = counts ? counts : static_cast<int32_t*>(ws);
  if (ccc::launch_count1_zero(v, ld, n_v, n_f, cnt, 0, zero, stream) != hipSuccess)
    return CCC_ERR_HIP;
  if (row_end <= i_begin) return CCC_OK;
  ccc::Pair2Args a{};
  a.complete = reinterpret_cast<int*>(static_cast<char*>(ws) + cnt_bytes);
  a.va = v; a.lda = ld; a.n_a = n_v;
  a.vb = v; a.ldb = ld; a.n_b = n_v;
  a.n_f = n_f;
  a.f4 = f4;
  a.tri = 1;
  a.accumulate = 0;
  a.tables = tables;
  a.ccc = ccc;
  a.counts_a = cnt;
  a.counts_b = cnt;
  a.chunk_a = cnt;
  a.chunk_b = cnt;
  a.gamma = o.gamma;
  a.row_begin = i_begin;
  a.row_end = row_end;
  a.p_base = i_begin * n_v - i_begin * (i_begin + 1) / 2;  // p(i_begin, i_begin + 1)
  a.sel = sel ? ccc::Select{sel->count, sel->cap, threshold, sel->index, sel->ccc, sel->tables}
              : ccc::Select{nullptr, 0, 0.0, nullptr, nullptr, nullptr};
  return ccc::run_pair2(a, o.path, stream);
}

int64_t choose3(int64_t n) { return n < 3 ? 0 : n * (n - 1) / 2 * (n - 2) / 3; }
int64_t choose2(int64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }

// Scratch of ccc_3way_noalloc: a fixed device array, one copy per device,
// held until the process ends.  Host code never uses its name as an address:
// the device address of each device's copy is looked up once (with that
// device current) and kept in g_scratch.
static __device__ __align__(256) unsigned char scratch[CCC_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch;  // indexed by device ordinal; null until looked up

int noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CCC_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return CCC_ERR_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return CCC_OK;
}

// The no-allocation form of a call: its scratch is the fixed array above
// (`bytes` of it) instead of the library workspace.
struct FixedScratch {
  size_t bytes;
};

// All 3-way variants: dense first-index rows [i_begin, i_end) or selection.
// With `fixed`, the scratch comes from there instead of the workspace: the
// call returns CCC_ERR_RANGE if the unit offsets and counts do not fit, and
// leaves the Gram matrix out (every unit then takes the general form, same
// results) when it does not fit beside them.
int three_way(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i_begin,
              int64_t i_end, int32_t* tables, double* ccc, const ccc_selection* sel,
              double threshold, int32_t* counts, const ccc_opts* opts, hipStream_t stream,
              const FixedScratch* fixed = nullptr) {
  ccc_opts o;
  int st = resolve_opts(opts, &o);
  if (st) return st;
  if (o.flags != 0) return CCC_ERR_ARG;
  if ((st = check_input(v, n_v, n_f, ld))) return st;
  if (!fields_in_range(n_f, 8)) return CCC_ERR_RANGE;
  const int f4 = o.path == CCC_PATH_POPCOUNT ? 0 : use_fp4(o, n_f);
  if (f4 < 0) return f4;
  if (i_begin < 0 || i_end < i_begin || i_end > n_v) return CCC_ERR_ARG;
  if (sel) {
    if (!sel->index || !sel->ccc || !sel->count || sel->cap < 0) return CCC_ERR_ARG;
    if (!isfinite(threshold)) return CCC_ERR_ARG;
    if (!aligned16(sel->index) || !aligned16(sel->ccc) || !aligned16(sel->tables) ||
        !aligned16(sel->count))
      return CCC_ERR_ALIGN;
  } else if ((i_end < n_v - 2 ? i_end : n_v - 2) > i_begin && !tables && !ccc) {
    return CCC_ERR_ARG;  // the range holds triples but there is nowhere to put them
  }
  if (!aligned16(tables) || !aligned16(ccc) || !aligned16(counts)) return CCC_ERR_ALIGN;
  if (n_v > 2642245) return CCC_ERR_ARG;  // C(n_v,3) * 8 must fit int64 indexing
  if (n_v == 0) return CCC_OK;
  unsigned long long* zero = sel ? sel->count : nullptr;
  const int64_t row_end = i_end < n_v - 2 ? i_end : n_v - 2;  // first index below n_v - 2
  if (row_end <= i_begin && !counts && !zero) return CCC_OK;  // nothing to compute or write
  // workspace: offsets of the tetrahedral work units (per tile pair; the
  // one-j grid, the grid of the complete-data kernel's runs of j, the fp4
  // general kernel's grid of 32-row tiles), then (if needed) counts, then
  // (MFMA path) the complete-data flag and the rho(1) Gram matrix of rows
  // [g0, n_v) used by complete-data units; g0 is i_begin rounded down to the
  // unit tile
  const ccc::UnitGrid ug = ccc::unit_grid(n_v, ccc::kUnitTile, i_begin, row_end);
  const size_t offs_bytes = ((size_t)(ccc::grid_pairs(ug) + 1) * 8 + 255) / 256 * 256;
  const ccc::UnitGrid ug32 = ccc::unit_grid(n_v, ccc::kRunTile, i_begin, row_end);
  const size_t gen_bytes = ((size_t)(ccc::grid_pairs(ug32) + 1) * 8 + 255) / 256 * 256;
  const size_t cnt_bytes = counts ? 0 : ((size_t)n_v * 16 + 255) / 256 * 256;
  // offsets (one-j grid, runs grid, 32-row runs grid), counts, flag
  const size_t head_bytes = 2 * offs_bytes + gen_bytes + cnt_bytes + 256;
  const int64_t g0 = i_begin / ccc::kUnitTile * ccc::kUnitTile, ng = n_v - g0;
  bool use_gram = o.path != CCC_PATH_POPCOUNT && ng <= kGramMaxRows && i_begin < row_end;
  if (fixed) {
    if (head_bytes > fixed->bytes) return CCC_ERR_RANGE;
    if (use_gram && (size_t)ng * (size_t)ng * 4 > fixed->bytes - head_bytes) use_gram = false;
  }
  const size_t gram_bytes = use_gram ? (size_t)ng * (size_t)ng * 4 : 0;
  void* ws = nullptr;
  if ((st = fixed ? noalloc_scratch(&ws) : ccc::workspace(head_bytes + gram_bytes, &ws)))
    return st;
  char* wsb = static_cast<char*>(ws);
  int32_t* cnt = counts ? counts : reinterpret_cast<int32_t*>(wsb + 2 * offs_bytes + gen_bytes);
  if (n_v < 3)
    return ccc::launch_count1_zero(v, ld, n_v, n_f, cnt, 0, zero, stream) == hipSuccess
               ? CCC_OK
               : CCC_ERR_HIP;
  if (ccc::launch_count1_zero(v, ld, n_v, n_f, cnt, 0, zero, stream) != hipSuccess)
    return CCC_ERR_HIP;
  if (row_end <= i_begin) return CCC_OK;
  ccc::Triple3Args a{};
  a.v = v; a.ld = ld; a.n = n_v; a.n_f = n_f;
  a.f4 = f4;
  a.tables = tables;
  a.ccc = ccc;
  a.counts = cnt;
  a.gamma = o.gamma;
  a.offs = static_cast<int64_t*>(ws);
  a.i_begin = i_begin;
  a.i_end = row_end;
  a.t_base = choose3(n_v) - choose3(n_v - i_begin);  // T(i_begin, i_begin+1, i_begin+2)
  a.sel = sel ? ccc::Select{sel->count, sel->cap, threshold, sel->index, sel->ccc, sel->tables}
              : ccc::Select{nullptr, 0, 0.0, nullptr, nullptr, nullptr};
  a.gram = use_gram ? reinterpret_cast<int32_t*>(wsb + head_bytes) : nullptr;
  a.g0 = g0;
  a.ng = use_gram ? ng : 0;
  // the complete-data kernel (fp4 operands, with the Gram matrix)
  a.complete = use_gram && f4 ? reinterpret_cast<int*>(wsb + 2 * offs_bytes + gen_bytes + cnt_bytes)
                              : nullptr;
  a.offs_run = reinterpret_cast<int64_t*>(wsb + offs_bytes);
  a.offs_gen = reinterpret_cast<int64_t*>(wsb + 2 * offs_bytes);
  hipError_t e = o.path == CCC_PATH_POPCOUNT ? ccc::launch_pop3(a, stream)
                                             : ccc::launch_mfma3(a, stream);
  return e == hipSuccess ? CCC_OK : CCC_ERR_HIP;
}

}  // namespace

extern "C" {

int ccc_2way(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int32_t* tables,
             double* ccc, int32_t* counts, const ccc_opts* opts, hipStream_t stream) {
  return two_way(v, n_v, n_f, ld, 0, n_v < 0 ? 0 : n_v, tables, ccc, nullptr, 0.0, counts, opts,
                 stream);
}

int ccc_2way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i_begin,
                  int64_t i_end, int32_t* tables, double* ccc, int32_t* counts,
                  const ccc_opts* opts, hipStream_t stream) {
  return two_way(v, n_v, n_f, ld, i_begin, i_end, tables, ccc, nullptr, 0.0, counts, opts,
                 stream);
}

int ccc_2way_select(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, double threshold,
                    const ccc_selection* out, int32_t* counts, const ccc_opts* opts,
                    hipStream_t stream) {
  if (!out) return CCC_ERR_ARG;
  return two_way(v, n_v, n_f, ld, 0, n_v < 0 ? 0 : n_v, nullptr, nullptr, out, threshold,
                 counts, opts, stream);
}

int ccc_3way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i_begin,
                  int64_t i_end, int32_t* tables, double* ccc, int32_t* counts,
                  const ccc_opts* opts, hipStream_t stream) {
  return three_way(v, n_v, n_f, ld, i_begin, i_end, tables, ccc, nullptr, 0.0, counts, opts,
                   stream);
}

int ccc_3way_select(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, double threshold,
                    const ccc_selection* out, int32_t* counts, const ccc_opts* opts,
                    hipStream_t stream) {
  if (!out) return CCC_ERR_ARG;
  return three_way(v, n_v, n_f, ld, 0, n_v < 0 ? 0 : n_v, nullptr, nullptr, out, threshold,
                   counts, opts, stream);
}

int ccc_3way(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int32_t* tables,
             double* ccc, int32_t* counts, const ccc_opts* opts, hipStream_t stream) {
  return three_way(v, n_v, n_f, ld, 0, n_v < 0 ? 0 : n_v, tables, ccc, nullptr, 0.0, counts,
                   opts, stream);
}

int ccc_2way_block(const uint8_t* va, int64_t n_a, int64_t lda, const uint8_t* vb, int64_t n_b,
                   int64_t ldb, int64_t n_f, int32_t* tables, int32_t* counts_a,
                   int32_t* counts_b, double* ccc, const ccc_opts* opts, hipStream_t stream) {
  ccc_opts o;
  int st = resolve_opts(opts, &o);
  if (st) return st;
  if ((st = check_input(va, n_a, n_f, lda))) return st;
  if ((st = check_input(vb, n_b, n_f, ldb))) return st;
  if (!fields_in_range(n_f, 4)) return CCC_ERR_RANGE;
  const int f4 = o.path == CCC_PATH_POPCOUNT ? 0 : use_fp4(o, n_f);
  if (f4 < 0) return f4;
  const bool acc = (o.flags & CCC_ACCUMULATE) != 0, fin = (o.flags & CCC_FINALIZE) != 0;
  if (n_a > 0 && n_b > 0) {
    if (!tables || !counts_a || !counts_b) return CCC_ERR_ARG;
    if (fin && !ccc) return CCC_ERR_ARG;
  }
  if (!aligned16(tables) || !aligned16(ccc) || !aligned16(counts_a) || !aligned16(counts_b))
    return CCC_ERR_ALIGN;
  if (n_a == 0 || n_b == 0) return CCC_OK;
  // workspace: an accumulating call's own chunk counts, or else the MFMA
  // path's complete-data flag
  int32_t* chunk_a = counts_a;
  int32_t* chunk_b = counts_b;
  void* ws = nullptr;
  if ((st = ccc::workspace(acc ? (size_t)(n_a + n_b) * 16 : 256, &ws))) return st;
  if (acc) {
    chunk_a = static_cast<int32_t*>(ws);
    chunk_b = chunk_a + 4 * n_a;
    if (ccc::launch_count1(va, lda, n_a, n_f, chunk_a, 0, stream) != hipSuccess ||
        ccc::launch_count1(vb, ldb, n_b, n_f, chunk_b, 0, stream) != hipSuccess)
      return CCC_ERR_HIP;
  }
  if (ccc::launch_count1(va, lda, n_a, n_f, counts_a, acc, stream) != hipSuccess)
    return CCC_ERR_HIP;
  if (ccc::launch_count1(vb, ldb, n_b, n_f, counts_b, acc, stream) != hipSuccess)
    return CCC_ERR_HIP;
  ccc::Pair2Args a{};
  a.va = va; a.lda = lda; a.n_a = n_a;
  a.vb = vb; a.ldb = ldb; a.n_b = n_b;
  a.n_f = n_f;
  a.f4 = f4;
  a.tri = 0;
  a.accumulate = acc ? 1 : 0;
  a.tables = tables;
  a.ccc = fin ? ccc : nullptr;
  a.counts_a = counts_a;
  a.counts_b = counts_b;
  a.chunk_a = chunk_a;
  a.chunk_b = chunk_b;
  a.gamma = o.gamma;
  a.row_begin = 0;
  a.row_end = n_a;
  a.p_base = 0;
  a.sel = ccc::Select{nullptr, 0, 0.0, nullptr, nullptr, nullptr};
  a.complete = acc ? nullptr : static_cast<int*>(ws);
  return ccc::run_pair2(a, o.path, stream);
}

int ccc_2way_multi(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s,
                   int32_t* tables, double* ccc, int32_t* counts, const ccc_opts* opts,
                   hipStream_t stream) {
  ccc_opts o;
  int st = resolve_opts(opts, &o);
  if (st) return st;
  if (o.flags != 0) return CCC_ERR_ARG;
  if (o.path == CCC_PATH_POPCOUNT) return CCC_ERR_UNSUPPORTED;
  if (s < 2 || s > 4) return CCC_ERR_ARG;
  if (n_v < 0 || n_f < 0 || ld < 0 || n_v > kInt32Max) return CCC_ERR_ARG;
  if (ld % 16 != 0) return CCC_ERR_ALIGN;
  if (ld > kMaxLd) return CCC_ERR_RANGE;
  if (ld < n_f) return CCC_ERR_ARG;
  if (n_v > 0 && !v) return CCC_ERR_ARG;
  if (!aligned16(v) || !aligned16(tables) || !aligned16(ccc) || !aligned16(counts))
    return CCC_ERR_ALIGN;
  if (!fields_in_range(n_f, 4)) return CCC_ERR_RANGE;
  const int f4 = use_fp4(o, n_f);
  if (f4 < 0) return f4;
  if (n_v >= 2 && !tables && !ccc) return CCC_ERR_ARG;
  if (n_v == 0 || (n_v == 1 && !counts)) return CCC_OK;
  int32_t* cnt = counts;
  if (!cnt) {
    void* ws = nullptr;
    if ((st = ccc::workspace((size_t)n_v * 32, &ws))) return st;
    cnt = static_cast<int32_t*>(ws);
  }
  if (ccc::launch_multi_count(v, ld, n_v, n_f, s, cnt, stream) != hipSuccess) return CCC_ERR_HIP;
  if (n_v < 2) return CCC_OK;
  return ccc::launch_multi2(v, ld, n_v, n_f, s, tables, ccc, cnt, o.gamma, f4, stream) ==
                 hipSuccess
             ? CCC_OK
             : CCC_ERR_HIP;
}

int ccc_2way_many(const ccc_problem* probs, int n_probs, const ccc_opts* opts,
                  hipStream_t stream) {
  ccc_opts o;
  int st = resolve_opts(opts, &o);
  if (st) return st;
  if (o.flags != 0) return CCC_ERR_ARG;
  if (n_probs < 0 || (n_probs > 0 && !probs)) return CCC_ERR_ARG;
  int64_t nf_max = 0;
  for (int p = 0; p < n_probs; ++p) {
    const ccc_problem& q = probs[p];
    if ((st = check_input(q.v, q.n_v, q.n_f, q.ld))) return st;
    if (!fields_in_range(q.n_f, 4)) return CCC_ERR_RANGE;
    if (q.n_f > nf_max) nf_max = q.n_f;
    if (q.n_v >= 2 && !q.tables && !q.ccc) return CCC_ERR_ARG;
    if (!aligned16(q.tables) || !aligned16(q.ccc) || !aligned16(q.counts)) return CCC_ERR_ALIGN;
  }
  const int f4 = o.path == CCC_PATH_POPCOUNT ? 0 : use_fp4(o, nf_max);
  if (f4 < 0) return f4;
  if (n_probs == 0) return CCC_OK;
  return ccc::run_many(probs, n_probs, o, f4 != 0, stream);
}

int ccc_3way_noalloc(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int32_t* tables,
                     double* ccc, int32_t* counts, const ccc_opts* opts, hipStream_t stream) {
  const FixedScratch fs{CCC_NOALLOC_SCRATCH_BYTES};
  return three_way(v, n_v, n_f, ld, 0, n_v < 0 ? 0 : n_v, tables, ccc, nullptr, 0.0, counts,
                   opts, stream, &fs);
}

void ccc_release_workspace(void) {
  ccc::release_many_cache();
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = 0;
  bool have_cur = hipGetDevice(&cur) == hipSuccess;
  for (size_t d = 0; d < g_ws.size(); ++d) {
    if (!g_ws[d].ptr) continue;
    if (hipSetDevice((int)d) == hipSuccess) {
      (void)hipDeviceSynchronize();
      (void)hipFree(g_ws[d].ptr);
    }
    g_ws[d] = Workspace{};
  }
  if (have_cur) (void)hipSetDevice(cur);
}

}  // extern "C"
