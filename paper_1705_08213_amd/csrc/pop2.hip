// pop2.hip -- 2-way tallies by bitwise AND + population count: the one-shot
// kernel over the triangle or the rectangle.  The tile body and its design
// notes are in tile2.h.
#include "tile2.h"

namespace ccc {

namespace {

__global__ __launch_bounds__(256) void pop2_kernel(Pair2Args a, int64_t tiles_side,
                                                   int64_t tiles_n) {
  __shared__ tile2::Pop2Smem sm;
  int64_t I, J;
  if (a.tri) {
    tri_tile(blockIdx.x + a.sq_offset, tiles_side, I, J);
  } else {
    I = blockIdx.x / tiles_n;
    J = blockIdx.x % tiles_n;
  }
  tile2::pop2_block_tile(a, I, J, sm);
}

}  // namespace

hipError_t launch_pop2(const Pair2Args& a, hipStream_t stream) {
  int64_t tm = (a.n_a + tile2::kTile - 1) / tile2::kTile, tn = (a.n_b + tile2::kTile - 1) / tile2::kTile;
  int64_t ntiles = tm * tn;
  Pair2Args b = a;
  if (a.tri) {  // square tiles of the row range
    const int64_t s0 = a.row_begin / tile2::kTile, s1 = (a.row_end + tile2::kTile - 1) / tile2::kTile;
    b.sq_offset = s0 * tm - s0 * (s0 - 1) / 2;
    ntiles = s1 * tm - s1 * (s1 - 1) / 2 - b.sq_offset;
  }
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  timing_begin("pop2", stream);
  hipLaunchKernelGGL(pop2_kernel, dim3((unsigned)ntiles), dim3(256), 0, stream, b, tm, tn);
  timing_end(stream);
  return hipGetLastError();
}

}  // namespace ccc
