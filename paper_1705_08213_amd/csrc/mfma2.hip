// mfma2.hip -- 2-way tallies on the matrix cores (fp4 or int8 operands): the
// one-shot kernel over the triangle (ccc_2way) or the rectangle
// (ccc_2way_block).  The tile body and its design notes are in tile2.h.
#include "tile2.h"

namespace ccc {

namespace {

// *flag = 1 if every row of A and B has all n_f fields present (one
// workgroup; its threads read the counts with a stride).
__global__ __launch_bounds__(1024) void complete_flag_kernel(const int32_t* __restrict__ ca,
                                                             int64_t n_a,
                                                             const int32_t* __restrict__ cb,
                                                             int64_t n_b, int64_t n_f,
                                                             int* __restrict__ flag) {
  bool ok = n_f > 0;
  for (int64_t r = threadIdx.x; r < n_a && ok; r += blockDim.x)
    ok = reinterpret_cast<const v4i*>(ca)[r].z == n_f;
  for (int64_t r = threadIdx.x; r < n_b && ok; r += blockDim.x)
    ok = reinterpret_cast<const v4i*>(cb)[r].z == n_f;
  ok = __syncthreads_and(ok ? 1 : 0) != 0;
  if (threadIdx.x == 0) *flag = ok ? 1 : 0;
}

// Workgroup tile (I, J) of `b` in a grid of tiles of BM x BN pairs
// (triangle: BM / BN tiles per square, squares in strips of H square rows).
template <int BM, int BN, int H = kStripRows>
__device__ __forceinline__ void tile_of(const Pair2Args& a, int64_t b, int64_t tiles_side,
                                        int64_t tiles_n, int64_t& I, int64_t& J) {
  constexpr int HALVES = BM / BN;
  static_assert(BM == HALVES * BN, "a square splits into whole tiles");
  if (a.tri) {
    int64_t sq_i, sq_j;
    strip_square(b / HALVES, tiles_side, a.row_begin / BM, (a.row_end + BM - 1) / BM, sq_i,
                 sq_j, H);
    I = sq_i;
    J = HALVES * sq_j + b % HALVES;
  } else {
    I = b / tiles_n;
    J = b % tiles_n;
  }
}

// Square rows per strip of the complete-data kernel's triangle order: its
// squares are twice the height of the general kernel's.
constexpr int kCompleteStripRows = 4;

// Calls whose every row is complete: 2 x 2 waves of (16 WM) x (16 WN) pairs
// (mfma2_complete_wave_tile); a workgroup exits at once when the flag says
// that some row is not complete (mfma2_kernel then covers the call).
template <int WM, int WN, bool F4>
__global__ __launch_bounds__(256, 2) void mfma2_complete_kernel(Pair2Args a,
                                                                int64_t tiles_side,
                                                                int64_t tiles_n) {
  if (*a.complete == 0) return;  // uniform
  constexpr int BM = 32 * WM, BN = 32 * WN, NB = 2 * WM + 2 * WN;
  const int wave = threadIdx.x >> 6;
  int64_t I, J;
  tile_of<BM, BN, kCompleteStripRows>(a, xcd_unit(blockIdx.x, gridDim.x), tiles_side, tiles_n, I,
                                      J);
  __shared__ u4 stage[2][NB][64];
  __shared__ u4 outs[4][128];
  tile2::mfma2_complete_wave_tile<WM, WN, F4>(a, I * BM + (wave & 1) * 16 * WM,
                                              J * BN + (wave >> 1) * 16 * WN, stage, outs[wave]);
}

// The general kernel: 2 x 2 waves of (16 WM) x (16 WN) pairs.  Workgroups
// of the 128 x 64 shape whose rows are all complete compute their tile
// together in the one-plane form (mfma2_coop_complete).
template <int WM, int WN, bool F4, int MIN_WG>
__global__ __launch_bounds__(256, MIN_WG) void mfma2_kernel(Pair2Args a, int64_t tiles_side,
                                                            int64_t tiles_n) {
  if (a.complete && *a.complete) return;  // uniform: mfma2_complete_kernel covers the call
  constexpr int BM = 32 * WM, BN = 32 * WN, NB = 2 * WM + 2 * WN;
  constexpr bool kCoop = WM == 4 && WN == 2;
  const int wave = threadIdx.x >> 6;
  // XCD-contiguous runs of tiles (triangle: in strip order, so that a run
  // shares row and column blocks in one L2)
  int64_t I, J;
  tile_of<BM, BN>(a, xcd_unit(blockIdx.x, gridDim.x), tiles_side, tiles_n, I, J);
  // the cooperative form's partial tiles (64 KB), or else the workgroup's
  // two stage buffers of NB row blocks
  __shared__ u4 smem[kCoop ? 4 * 16 * 64 : 2 * NB * 64];
  static_assert(sizeof(smem) >= 2 * NB * 64 * sizeof(u4), "stage buffers fit");
  if constexpr (kCoop) {
    if (tile2::workgroup_complete<WM, WN>(a, I * BM, J * BN)) {
      tile2::mfma2_coop_complete<WM, WN, F4>(a, I * BM, J * BN,
                                             reinterpret_cast<v4i(*)[16][64]>(smem));
      return;
    }
  }
  tile2::mfma2_wave_tile<WM, WN, F4>(a, I * BM + (wave & 1) * 16 * WM,
                                     J * BN + (wave >> 1) * 16 * WN,
                                     reinterpret_cast<u4(*)[NB][64]>(smem));
}

// Grid of BM x BN workgroup tiles: tiles along a side (rows, columns) and
// the tile count (triangle: the squares of the row range, BM / BN tiles
// each); 0 tiles when there is nothing to do.
template <int BM, int BN>
int64_t tile_grid(const Pair2Args& a, int64_t& tm, int64_t& tn) {
  tm = (a.n_a + BM - 1) / BM;
  tn = (a.n_b + BN - 1) / BN;
  if (!a.tri) return tm * tn;
  const int64_t s0 = a.row_begin / BM, s1 = (a.row_end + BM - 1) / BM;
  return BM / BN * (s1 * tm - s1 * (s1 - 1) / 2 - (s0 * tm - s0 * (s0 - 1) / 2));
}

template <int WM, int WN, bool F4, int MIN_WG>
hipError_t launch_shape(const Pair2Args& a, hipStream_t stream) {
  int64_t tm, tn;
  const int64_t ntiles = tile_grid<32 * WM, 32 * WN>(a, tm, tn);
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL((mfma2_kernel<WM, WN, F4, MIN_WG>), dim3((unsigned)ntiles), dim3(256), 0,
                     stream, a, tm, tn);
  return hipGetLastError();
}

// Shapes of the general kernel, picked per call by the kernel-shape table
// (kind oneshot): 0 = 128 x 64 workgroup tiles (waves 64 x 32), 1 = 64 x 32
// (32 x 16), 2 = 64 x 64 (32 x 32).  Smaller tiles give small calls more
// workgroups.
constexpr int kOneShotVariants = 3;

template <bool F4>
hipError_t launch_general(const Pair2Args& a, hipStream_t stream) {
  const int64_t n = a.n_a > a.n_b ? a.n_a : a.n_b;
  switch (tune_pick(kTuneOneShot, n, a.n_f, kOneShotVariants).variant) {
    case 1: return launch_shape<2, 1, F4, 4>(a, stream);
    case 2: return launch_shape<2, 2, F4, 2>(a, stream);
    default: return launch_shape<4, 2, F4, 2>(a, stream);
  }
}

// The complete-data kernel's wave tile: 128 x 64 pairs (8 x 4 blocks of 16).
constexpr int kCWM = 8, kCWN = 4;

template <bool F4>
hipError_t launch_complete(const Pair2Args& a, hipStream_t stream) {
  int64_t tm, tn;
  const int64_t ntiles = tile_grid<32 * kCWM, 32 * kCWN>(a, tm, tn);
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  hipLaunchKernelGGL((mfma2_complete_kernel<kCWM, kCWN, F4>), dim3((unsigned)ntiles), dim3(256),
                     0, stream, a, tm, tn);
  return hipGetLastError();
}

template <bool F4>
hipError_t launch_f(const Pair2Args& a, hipStream_t stream) {
  if (a.complete) {
    // the flag first, then both kernels: each exits at once unless the flag
    // picks it
    hipLaunchKernelGGL(complete_flag_kernel, dim3(1), dim3(1024), 0, stream, a.counts_a, a.n_a,
                       a.counts_b, a.n_b, a.n_f, a.complete);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_complete<F4>(a, stream)) != hipSuccess) return e;
  }
  return launch_general<F4>(a, stream);
}

}  // namespace

hipError_t launch_mfma2(const Pair2Args& a, hipStream_t stream) {
  if (a.complete && a.accumulate) return hipErrorInvalidValue;
  timing_begin("mfma2", stream);
  const hipError_t e = a.f4 ? launch_f<true>(a, stream) : launch_f<false>(a, stream);
  timing_end(stream);
  return e;
}

}  // namespace ccc
