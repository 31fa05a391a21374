// count1.hip -- per-vector allele counts n_i(0), n_i(1) and present-field
// count m_i (the ingredients of f_i(a), Sec. 2.1 Eq. (1)).
//
// One wave per row; each lane reads 16-byte pieces (64 fields) with a
// 1 KiB stride, so a wave streams its row fully coalesced.  The counts come
// from population counts on the two bit-planes of the codes:
//   b0 = low bits  (set for 01 and 11)   -> rho(1) >= 1
//   b1 = high bits (set for 11 and 10)
//   n(1) = pop(b0) + pop(b0 & b1),  missing = pop(b1 & ~b0),
//   m = fields - missing,  n(0) = 2m - n(1).
#include "common.h"
#include "kernels.h"

namespace ccc {

__global__ __launch_bounds__(256) void count1_kernel(const uint8_t* __restrict__ v, int64_t ld,
                                                     int64_t n, int64_t n_f,
                                                     int32_t* __restrict__ counts,
                                                     int accumulate,
                                                     unsigned long long* __restrict__ zero) {
  if (zero && blockIdx.x == 0 && threadIdx.x == 0) *zero = 0ull;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  count_row_wave(v + row * ld, n_f, counts + 4 * row, accumulate);
}

hipError_t launch_count1_zero(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f,
                              int32_t* counts, int accumulate, unsigned long long* zero,
                              hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 3) / 4));
  timing_begin("count1", stream);
  hipLaunchKernelGGL(count1_kernel, grid, dim3(256), 0, stream, v, ld, n, n_f, counts,
                     accumulate, zero);
  timing_end(stream);
  return hipGetLastError();
}

hipError_t launch_count1(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int32_t* counts,
                         int accumulate, hipStream_t stream) {
  return launch_count1_zero(v, ld, n, n_f, counts, accumulate, nullptr, stream);
}

}  // namespace ccc
