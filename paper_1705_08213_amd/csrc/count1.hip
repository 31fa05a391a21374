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
                                                     int accumulate) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const uint8_t* r = v + row * ld;
  const int64_t nbytes = (n_f + 3) / 4;
  int n1 = 0, miss = 0;
  for (int64_t ob = (int64_t)lane * 16; ob < nbytes; ob += 64 * 16) {
    u4 w = load_fields64(r, ob, n_f);
    unsigned ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      unsigned b0 = ws[s] & kEven, b1 = (ws[s] >> 1) & kEven;
      n1 += __popc(b0) + __popc(b0 & b1);
      miss += __popc(b1 & ~b0);
    }
  }
  // fields covered by the loop minus missing ones (masked tails count as missing)
  int64_t covered = 0;
  {
    int64_t first = (int64_t)lane * 16;
    if (first < nbytes) covered = ((nbytes - 1 - first) / (64 * 16) + 1) * 64;
  }
  int present = (int)(covered - miss);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    n1 += __shfl_xor(n1, off);
    present += __shfl_xor(present, off);
  }
  if (lane == 0) {
    v4i c = v4i{2 * present - n1, n1, present, 0};
    v4i* out = reinterpret_cast<v4i*>(counts) + row;
    if (accumulate) {
      v4i o = *out;
      c = v4i{o.x + c.x, o.y + c.y, o.z + c.z, 0};
    }
    *out = c;
  }
}

hipError_t launch_count1(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int32_t* counts,
                         int accumulate, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  dim3 grid((unsigned)((n + 3) / 4));
  timing_begin("count1", stream);
  hipLaunchKernelGGL(count1_kernel, grid, dim3(256), 0, stream, v, ld, n, n_f, counts,
                     accumulate);
  timing_end(stream);
  return hipGetLastError();
}

}  // namespace ccc
