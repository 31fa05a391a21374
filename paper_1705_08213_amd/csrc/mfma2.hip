// mfma2.hip -- 2-way tallies on the matrix cores (fp4 or int8 operands): the
// one-shot kernel over the triangle (ccc_2way) or the rectangle
// (ccc_2way_block).  The tile body and its design notes are in tile2.h.
#include "tile2.h"

namespace ccc {

namespace {

template <int WM, int WN, bool F4>
__global__ __launch_bounds__(256, 2) void mfma2_kernel(Pair2Args a, int64_t tiles_side,
                                                       int64_t tiles_n) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  static_assert(BM == 2 * BN, "triangle split assumes BM = 2 BN");
  const int wave = threadIdx.x >> 6;
  // XCD-contiguous runs of tiles (triangle: in strip order, so that a run
  // shares row and column blocks in one L2)
  const int64_t b = xcd_unit(blockIdx.x, gridDim.x);
  int64_t I, J;
  if (a.tri) {
    int64_t sq_i, sq_j;
    strip_square(b >> 1, tiles_side, a.row_begin / BM, (a.row_end + BM - 1) / BM, sq_i, sq_j);
    I = sq_i;
    J = 2 * sq_j + (b & 1);
  } else {
    I = b / tiles_n;
    J = b % tiles_n;
  }
  // 64 KB: the complete-data form's partial tiles, or else the workgroup's
  // two fp4 stage buffers of 2 WM + 2 WN row blocks
  __shared__ v4i part[4][16][64];
  static_assert(sizeof(part) >= 2 * (2 * WM + 2 * WN) * 64 * sizeof(u4), "stage buffers fit");
  if (tile2::workgroup_complete<WM, WN>(a, I * BM, J * BN)) {
    tile2::mfma2_coop_complete<WM, WN, F4>(a, I * BM, J * BN, part);
    return;
  }
  tile2::mfma2_wave_tile<WM, WN, F4>(
      a, I * BM + (wave & 1) * 16 * WM, J * BN + (wave >> 1) * 16 * WN,
      reinterpret_cast<u4(*)[2 * WM + 2 * WN][64]>(&part[0][0][0]));
}

template <int WM, int WN>
hipError_t launch_shape(const Pair2Args& a, hipStream_t stream) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  int64_t tm = (a.n_a + BM - 1) / BM, tn = (a.n_b + BN - 1) / BN;
  int64_t ntiles = tm * tn;
  Pair2Args b = a;
  if (a.tri) {  // squares of the row range, two halves each
    const int64_t s0 = a.row_begin / BM, s1 = (a.row_end + BM - 1) / BM;
    ntiles = 2 * (s1 * tm - s1 * (s1 - 1) / 2 - (s0 * tm - s0 * (s0 - 1) / 2));
  }
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  timing_begin("mfma2", stream);
  if (a.f4)
    hipLaunchKernelGGL((mfma2_kernel<WM, WN, true>), dim3((unsigned)ntiles), dim3(256), 0, stream,
                       b, tm, tn);
  else
    hipLaunchKernelGGL((mfma2_kernel<WM, WN, false>), dim3((unsigned)ntiles), dim3(256), 0,
                       stream, b, tm, tn);
  timing_end(stream);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mfma2(const Pair2Args& a, hipStream_t stream) {
  return launch_shape<4, 2>(a, stream);
}

}  // namespace ccc
