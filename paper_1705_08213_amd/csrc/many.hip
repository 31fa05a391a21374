// many.hip -- many independent 2-way problems in one persistent launch.
//
// Host side: every problem gets a tile variant from the tune table (by its
// size class), its tiles become work items (problem, tile), and the items are
// ordered longest first (cost ~ tile pairs x n_f: the LPT rule), so the tail
// of the launch is made of the cheapest tiles.  Descriptors and items live in
// a device buffer owned by a cache entry keyed on the batch (every descriptor
// field, the path and gamma).  On first sight of a batch the two launches
// below are captured into a HIP graph; later calls with the same batch only
// replay the graph on the caller's stream.
//
// Device side:
//   1. count_many_kernel: 1-way counts of every row of every problem (one
//      wave per row), and the persistent work counter reset to 0 (a kernel
//      store, so graphs hold no memset node);
//   2. many_*_kernel, one persistent launch per tile variant in the batch: a
//      grid of a few workgroups per compute unit (the tune table's figure
//      for the variant's problems, else 2); each workgroup takes the next
//      item of its variant's list with an atomic on that list's counter and
//      computes the tile with the same device code as the one-shot kernels
//      (tile2.h), until the list is exhausted.  The variants run on forked
//      graph branches, concurrently.
//
// Tile variants (mfma path), workgroup tile (wave tile): 0 = 128 x 64
// (64 x 32), 1 = 64 x 32 (32 x 16), 2 = 64 x 64 (32 x 32), 3 = 32 x 32
// (16 x 16).  A triangle is cut into squares of the workgroup tile's height,
// each one or two workgroup tiles.  The popcount path has one shape
// (64 x 64).
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "many.h"
#include "tile2.h"

namespace ccc {

namespace {

struct ProbDesc {
  const uint8_t* v;
  int64_t ld, n_v, n_f;
  int32_t* tables;
  double* ccc;
  int32_t* counts;
  int64_t row_begin;  // first row of this problem in the concatenated row range
  int32_t variant;
  int32_t tiles_side;  // square tiles per side for the variant
};

struct WorkItem {
  int32_t prob;
  int32_t tile;  // index into the problem's halves-of-squares triangle enumeration
};

constexpr int kVariants = 4;
// wave tiles in 16-row blocks per mfma variant, and what follows from them
constexpr int kWM[kVariants] = {4, 2, 2, 1}, kWN[kVariants] = {2, 1, 2, 1};
constexpr int kSquare[kVariants] = {32 * kWM[0], 32 * kWM[1], 32 * kWM[2], 32 * kWM[3]};
constexpr int kHalves[kVariants] = {kWM[0] / kWN[0], kWM[1] / kWN[1], kWM[2] / kWN[2],
                                    kWM[3] / kWN[3]};  // workgroup tiles per square
// workgroups per compute unit each variant's kernel is built for (its
// register budget), the most a launch may ask
constexpr int kMaxWg[kVariants] = {2, 4, 2, 4};
constexpr int kDefaultWg = 2;
constexpr int kPopTile = 64;

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void count_many_kernel(const ProbDesc* __restrict__ d,
                                                         int n_probs, int64_t total_rows,
                                                         unsigned* __restrict__ counters) {
  if (blockIdx.x == 0 && threadIdx.x < kVariants) counters[threadIdx.x] = 0u;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= total_rows) return;
  int lo = 0, hi = n_probs;  // d[lo].row_begin <= row < d[hi].row_begin
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (d[mid].row_begin <= row) lo = mid; else hi = mid;
  }
  const ProbDesc& p = d[lo];
  const int64_t r = row - p.row_begin;
  count_row_wave(p.v + r * p.ld, p.n_f, p.counts + 4 * r, 0);
}

__device__ __forceinline__ Pair2Args pair_args(const ProbDesc& p, double gamma) {
  Pair2Args a;
  a.va = p.v; a.lda = p.ld; a.n_a = p.n_v;
  a.vb = p.v; a.ldb = p.ld; a.n_b = p.n_v;
  a.n_f = p.n_f;
  a.f4 = 0;  // the operand format is the kernel's template argument
  a.tri = 1;
  a.accumulate = 0;
  a.tables = p.tables;
  a.ccc = p.ccc;
  a.counts_a = p.counts;
  a.counts_b = p.counts;
  a.chunk_a = p.counts;
  a.chunk_b = p.counts;
  a.gamma = gamma;
  a.row_begin = 0;
  a.row_end = p.n_v;
  a.p_base = 0;
  a.sq_offset = 0;
  a.sel = Select{nullptr, 0, 0.0, nullptr, nullptr, nullptr};
  a.complete = nullptr;
  return a;
}

// Next work item for the whole workgroup (thread 0 takes it, all read it).
__device__ __forceinline__ int next_item(unsigned* counter, int* slot) {
  if (threadIdx.x == 0) *slot = (int)atomicAdd(counter, 1u);
  __syncthreads();
  int it = *slot;
  __syncthreads();
  return it;
}

template <int WM, int WN, bool F4>
__device__ __forceinline__ void mfma_item(const Pair2Args& a, int64_t tiles_side, int tile,
                                          u4 (*stage)[2 * WM + 2 * WN][64]) {
  constexpr int BM = 32 * WM, BN = 32 * WN, HALVES = WM / WN;
  static_assert(BM == HALVES * BN, "a square is whole workgroup tiles");
  const int wave = threadIdx.x >> 6;
  int64_t sq_i, sq_j;
  tri_tile(tile / HALVES, tiles_side, sq_i, sq_j);
  const int64_t I = sq_i, J = HALVES * sq_j + tile % HALVES;
  tile2::mfma2_wave_tile<WM, WN, F4>(a, I * BM + (wave & 1) * 16 * WM,
                                     J * BN + (wave >> 1) * 16 * WN, stage);
}

// One persistent launch per tile variant present in the batch (each variant's
// items form their own list and counter), so every kernel keeps the register
// budget of its own tile shape.  F4: fp4 operands (every problem of the batch
// has n_f <= kF4MaxFields), else int8.
template <int WM, int WN, bool F4, int MIN_WG>
__global__ __launch_bounds__(256, MIN_WG) void many_mfma_kernel(const ProbDesc* __restrict__ d,
                                                           const WorkItem* __restrict__ items,
                                                           int n_items,
                                                           unsigned* __restrict__ counter,
                                                           double gamma) {
  __shared__ int slot;
  __shared__ u4 stage[2][2 * WM + 2 * WN][64];  // the workgroup's two fp4 stage buffers
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= n_items) break;
    const WorkItem w = items[it];
    const ProbDesc p = d[w.prob];
    mfma_item<WM, WN, F4>(pair_args(p, gamma), p.tiles_side, w.tile, stage);
  }
}

__global__ __launch_bounds__(256) void many_pop_kernel(const ProbDesc* __restrict__ d,
                                                       const WorkItem* __restrict__ items,
                                                       int n_items, unsigned* __restrict__ counter,
                                                       double gamma) {
  __shared__ int slot;
  __shared__ tile2::Pop2Smem sm;
  for (;;) {
    const int it = next_item(counter, &slot);
    if (it >= n_items) break;
    const WorkItem w = items[it];
    const ProbDesc p = d[w.prob];
    int64_t I, J;
    tri_tile(w.tile, p.tiles_side, I, J);
    tile2::pop2_block_tile(pair_args(p, gamma), I, J, sm);
  }
}

// Tile variant and workgroups per CU of a problem from the kernel-shape
// table (tune.hip).
TuneChoice pick_variant(int64_t n_v, int64_t n_f, int path) {
  return tune_pick(path == CCC_PATH_POPCOUNT ? kTuneManyPopcount : kTuneManyMfma, n_v, n_f,
                   kVariants);
}

// ---------------------------------------------------------------------------
// Batch cache
// ---------------------------------------------------------------------------

struct Entry {
  std::vector<unsigned char> key;
  void* dbuf = nullptr;  // descriptors | items | counter | counts scratch
  hipGraphExec_t exec = nullptr;
  hipStream_t capture = nullptr;
  uint64_t last_use = 0;
  // direct-launch parameters (used when graphs are disabled)
  ProbDesc* d = nullptr;
  WorkItem* items = nullptr;      // per-variant lists, back to back
  unsigned* counters = nullptr;   // one per variant
  int n_probs = 0;
  int item_begin[kVariants] = {}, n_items[kVariants] = {};
  int64_t total_rows = 0;
  int path = 0;
  bool f4 = true;                 // fp4 operands (every n_f <= kF4MaxFields), else int8
  double gamma = 0;
  int grid[kVariants] = {};
  // capture streams of the variants after the first (concurrent branches)
  hipStream_t fork[kVariants] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kVariants] = {};
};

std::mutex g_mu;
std::vector<Entry*> g_cache;
uint64_t g_clock = 0;
constexpr size_t kMaxEntries = 8;

void destroy(Entry* e) {
  if (e->exec) (void)hipGraphExecDestroy(e->exec);
  if (e->capture) (void)hipStreamDestroy(e->capture);
  for (int v = 0; v < kVariants; ++v) {
    if (e->fork[v]) (void)hipStreamDestroy(e->fork[v]);
    if (e->ev_join[v]) (void)hipEventDestroy(e->ev_join[v]);
  }
  if (e->ev_fork) (void)hipEventDestroy(e->ev_fork);
  if (e->dbuf) (void)hipFree(e->dbuf);
  delete e;
}

std::vector<unsigned char> make_key(const ccc_problem* probs, int n, const ccc_opts& o,
                                    bool f4) {
  std::vector<unsigned char> k(sizeof(ccc_problem) * n + sizeof(int) + sizeof(double) + 64);
  size_t off = 0;
  memcpy(k.data(), probs, sizeof(ccc_problem) * n);
  off += sizeof(ccc_problem) * n;
  memcpy(k.data() + off, &o.path, sizeof(int));
  off += sizeof(int);
  memcpy(k.data() + off, &o.gamma, sizeof(double));
  off += sizeof(double);
  int dev = 0;
  (void)hipGetDevice(&dev);
  memcpy(k.data() + off, &dev, sizeof(int));
  off += sizeof(int);
  // the choices can be forced from the environment; make them part of the key
  for (const char* name : {"CCC_MANY_VARIANT", "CCC_MANY_WG"}) {
    const char* env = getenv(name);
    const int forced = env ? atoi(env) + 1 : 0;
    memcpy(k.data() + off, &forced, sizeof(int));
    off += sizeof(int);
  }
  const int operands = f4 ? 4 : 8;
  memcpy(k.data() + off, &operands, sizeof(int));
  off += sizeof(int);
  k.resize(off);
  return k;
}

template <int V, bool F4>
void launch_mfma(const Entry& e, const WorkItem* items, hipStream_t stream) {
  hipLaunchKernelGGL((many_mfma_kernel<kWM[V], kWN[V], F4, kMaxWg[V]>), dim3(e.grid[V]),
                     dim3(256), 0, stream, e.d, items, e.n_items[V], e.counters + V, e.gamma);
}

hipError_t launch_variant(const Entry& e, int v, hipStream_t stream) {
  const WorkItem* items = e.items + e.item_begin[v];
  if (e.path == CCC_PATH_POPCOUNT) {
    hipLaunchKernelGGL(many_pop_kernel, dim3(e.grid[v]), dim3(256), 0, stream, e.d, items,
                       e.n_items[v], e.counters + v, e.gamma);
    return hipGetLastError();
  }
  switch (v * 2 + (e.f4 ? 1 : 0)) {
    case 0: launch_mfma<0, false>(e, items, stream); break;
    case 1: launch_mfma<0, true>(e, items, stream); break;
    case 2: launch_mfma<1, false>(e, items, stream); break;
    case 3: launch_mfma<1, true>(e, items, stream); break;
    case 4: launch_mfma<2, false>(e, items, stream); break;
    case 5: launch_mfma<2, true>(e, items, stream); break;
    case 6: launch_mfma<3, false>(e, items, stream); break;
    default: launch_mfma<3, true>(e, items, stream); break;
  }
  return hipGetLastError();
}

// The batch's launches.  With `fork` (graph capture), every variant after
// the first non-empty one runs on a forked stream joined back before the
// end, so the variants' kernels can share the GPU.
hipError_t enqueue(const Entry& e, hipStream_t stream, bool fork) {
  hipLaunchKernelGGL(count_many_kernel, dim3((unsigned)((e.total_rows + 3) / 4)), dim3(256), 0,
                     stream, e.d, e.n_probs, e.total_rows, e.counters);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  int first = -1, forked = 0;
  for (int v = 0; v < kVariants; ++v) {
    if (e.n_items[v] == 0) continue;
    if (first < 0 || !fork) {
      if (first < 0) first = v;
      if (!fork && (err = launch_variant(e, v, stream)) != hipSuccess) return err;
      continue;
    }
    if (forked++ == 0 && (err = hipEventRecord(e.ev_fork, stream)) != hipSuccess) return err;
    if ((err = hipStreamWaitEvent(e.fork[v], e.ev_fork, 0)) != hipSuccess) return err;
    if ((err = launch_variant(e, v, e.fork[v])) != hipSuccess) return err;
    if ((err = hipEventRecord(e.ev_join[v], e.fork[v])) != hipSuccess) return err;
  }
  if (!fork || first < 0) return hipSuccess;
  if ((err = launch_variant(e, first, stream)) != hipSuccess) return err;
  for (int v = first + 1; v < kVariants; ++v)
    if (e.n_items[v] > 0 && (err = hipStreamWaitEvent(stream, e.ev_join[v], 0)) != hipSuccess)
      return err;
  return hipSuccess;
}

// Build descriptors and the LPT-ordered work list; allocate and upload.
int build_entry(const ccc_problem* probs, int n, const ccc_opts& o, bool f4, Entry* e) {
  e->f4 = f4;
  std::vector<ProbDesc> d(n);
  std::vector<WorkItem> items[kVariants];
  std::vector<int64_t> cost[kVariants];
  int wg[kVariants] = {};  // largest workgroups-per-CU figure among each variant's problems
  int64_t rows = 0, scratch_counts = 0;
  for (int p = 0; p < n; ++p) {
    const ccc_problem& q = probs[p];
    ProbDesc& x = d[p];
    x.v = q.v;
    x.ld = q.ld;
    x.n_v = q.n_v;
    x.n_f = q.n_f;
    x.tables = q.tables;
    x.ccc = q.ccc;
    x.counts = q.counts;
    x.row_begin = rows;
    const bool pop = o.path == CCC_PATH_POPCOUNT;
    const TuneChoice tc = pick_variant(q.n_v, q.n_f, pop ? CCC_PATH_POPCOUNT : CCC_PATH_MFMA);
    x.variant = pop ? 0 : tc.variant;
    const int side = pop ? kPopTile : kSquare[x.variant];
    const int halves = pop ? 1 : kHalves[x.variant];
    const int64_t T = (q.n_v + side - 1) / side;
    if (T > 65536 || halves * (T * (T + 1) / 2) > 0x7FFFFFFF)
      return CCC_ERR_ARG;  // item indices must fit int32
    x.tiles_side = (int32_t)T;
    rows += q.n_v;
    if (!q.counts) scratch_counts += q.n_v;
    if (q.n_v < 2) continue;
    wg[x.variant] = std::max(wg[x.variant], tc.wg_per_cu);
    const int64_t ntiles = halves * (T * (T + 1) / 2);
    const int64_t tile_pairs = (int64_t)side * side / halves;
    for (int64_t t = 0; t < ntiles; ++t) {
      items[x.variant].push_back(WorkItem{p, (int32_t)t});
      cost[x.variant].push_back(tile_pairs * (q.n_f + 256));
    }
  }
  // LPT: longest items first within each variant's list (stable sort)
  std::vector<WorkItem> sorted;
  for (int v = 0; v < kVariants; ++v) {
    if (items[v].size() > 0x3FFFFFFF) return CCC_ERR_ARG;
    std::vector<size_t> order(items[v].size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](size_t x, size_t y) { return cost[v][x] > cost[v][y]; });
    e->item_begin[v] = (int)sorted.size();
    e->n_items[v] = (int)items[v].size();
    for (size_t i : order) sorted.push_back(items[v][i]);
  }

  const size_t d_bytes = (sizeof(ProbDesc) * n + 255) / 256 * 256;
  const size_t i_bytes = (sizeof(WorkItem) * sorted.size() + 255) / 256 * 256;
  const size_t c_bytes = 256;
  const size_t s_bytes = (size_t)scratch_counts * 16;
  if (hipMalloc(&e->dbuf, d_bytes + i_bytes + c_bytes + s_bytes) != hipSuccess) {
    (void)hipGetLastError();
    return CCC_ERR_NOMEM;
  }
  char* base = static_cast<char*>(e->dbuf);
  e->d = reinterpret_cast<ProbDesc*>(base);
  e->items = reinterpret_cast<WorkItem*>(base + d_bytes);
  e->counters = reinterpret_cast<unsigned*>(base + d_bytes + i_bytes);
  int32_t* scratch = reinterpret_cast<int32_t*>(base + d_bytes + i_bytes + c_bytes);
  for (int p = 0; p < n; ++p)
    if (!d[p].counts) {
      d[p].counts = scratch;
      scratch += 4 * d[p].n_v;
    }
  if (hipMemcpy(e->d, d.data(), sizeof(ProbDesc) * n, hipMemcpyHostToDevice) != hipSuccess ||
      (sorted.size() && hipMemcpy(e->items, sorted.data(), sizeof(WorkItem) * sorted.size(),
                                  hipMemcpyHostToDevice) != hipSuccess))
    return CCC_ERR_HIP;
  e->n_probs = n;
  e->total_rows = rows;
  e->path = o.path == CCC_PATH_POPCOUNT ? CCC_PATH_POPCOUNT : CCC_PATH_MFMA;
  e->gamma = o.gamma;
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  for (int v = 0; v < kVariants; ++v) {
    const int per_cu = std::min(wg[v] > 0 ? wg[v] : kDefaultWg,
                                e->path == CCC_PATH_POPCOUNT ? kDefaultWg : kMaxWg[v]);
    e->grid[v] = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * per_cu,
                                                             e->n_items[v]));
  }
  return CCC_OK;
}

bool graphs_enabled() {
  const char* env = getenv("CCC_MANY_GRAPH");
  return !(env && env[0] == '0');
}

}  // namespace

int run_many(const ccc_problem* probs, int n_probs, const ccc_opts& opts, bool f4,
             hipStream_t stream) {
  int64_t rows = 0;
  for (int p = 0; p < n_probs; ++p) rows += probs[p].n_v;
  if (rows == 0) return CCC_OK;
  std::vector<unsigned char> key = make_key(probs, n_probs, opts, f4);
  std::lock_guard<std::mutex> lk(g_mu);
  Entry* e = nullptr;
  for (Entry* c : g_cache)
    if (c->key == key) e = c;
  const bool use_graph = graphs_enabled();
  if (!e) {
    if (g_cache.size() >= kMaxEntries) {
      auto oldest = std::min_element(g_cache.begin(), g_cache.end(),
                                     [](Entry* x, Entry* y) { return x->last_use < y->last_use; });
      if (hipDeviceSynchronize() != hipSuccess) return CCC_ERR_HIP;
      destroy(*oldest);
      g_cache.erase(oldest);
    }
    const auto t0 = std::chrono::steady_clock::now();
    e = new Entry();
    e->key = key;
    int st = build_entry(probs, n_probs, opts, f4, e);
    if (st != CCC_OK) {
      destroy(e);
      return st;
    }
    if (use_graph) {
      hipGraph_t graph = nullptr;
      bool ok = hipStreamCreateWithFlags(&e->capture, hipStreamNonBlocking) == hipSuccess &&
                hipEventCreateWithFlags(&e->ev_fork, hipEventDisableTiming) == hipSuccess;
      for (int v = 0; v < kVariants && ok; ++v)
        ok = hipStreamCreateWithFlags(&e->fork[v], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&e->ev_join[v], hipEventDisableTiming) == hipSuccess;
      ok = ok && hipStreamBeginCapture(e->capture, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        hipError_t le = enqueue(*e, e->capture, true);
        ok = hipStreamEndCapture(e->capture, &graph) == hipSuccess && le == hipSuccess &&
             hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0) == hipSuccess;
      }
      if (graph) (void)hipGraphDestroy(graph);
      if (!ok) {
        (void)hipGetLastError();
        destroy(e);
        return CCC_ERR_HIP;
      }
    }
    g_cache.push_back(e);
    timing_host("many_setup", std::chrono::duration<double, std::milli>(
                                  std::chrono::steady_clock::now() - t0).count());
  }
  e->last_use = ++g_clock;
  timing_begin("many", stream);
  hipError_t err = e->exec ? hipGraphLaunch(e->exec, stream) : enqueue(*e, stream, false);
  timing_end(stream);
  return err == hipSuccess ? CCC_OK : CCC_ERR_HIP;
}

void release_many_cache() {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_cache.empty()) (void)hipDeviceSynchronize();
  for (Entry* e : g_cache) destroy(e);
  g_cache.clear();
}

}  // namespace ccc
