// mfma2.hip -- 2-way tallies on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// The tally is a GEMM whose scalar product became a 2x2 table (Sec. 3.1):
//   C(a,b) = R_a R_b^T,  R_a[i][q] = rho_{i,q}(a) in {0,1,2}.
// With per-allele counts as int8 operands and int32 accumulation the four
// products are exact integer GEMMs, so the matrix cores compute the tables
// directly (4 MACs per comparison).
//
// Design (gfx950, wave64):
//  * No LDS: each lane loads 16 packed bytes (64 fields) of one row per
//    super-step straight into registers and unpacks them there.  A lane of the
//    16x16x64 operand holds 16 k-values of one row; since the contraction
//    only needs A and B to share the k order, lane (row r, group g) takes the
//    16 fields of packed word s of its 16 bytes for MFMA step s, in the byte
//    order produced by the unpack below.  Both operands use the same order.
//  * Unpack of one packed word (16 fields): four shift+mask steps give bytes
//    holding one 2-bit code each; v_perm_b32 then looks each code up in a
//    4-byte table (rho(0) = 2,1,0,0 and rho(1) = 0,1,0,2 for codes 00,01,10,11).
//  * A wave owns a (16 WM) x (16 WN) tile of pairs with 4 accumulator sets
//    (one per (a,b)); a workgroup is 2 x 2 waves.  With WM = 4, WN = 2 the
//    accumulators (128 registers) and operands stay in the 256 arch VGPRs, so
//    two waves share each SIMD and one's unpack overlaps the other's MFMAs.
//  * Triangle: the row-major upper triangle of (2*BN)-wide square tiles is
//    enumerated, each square split into two BN-wide column halves (one
//    workgroup each); waves with no pair i < j return at once.
//  * Fields past n_f and whole 16-byte pieces past the row stride are turned
//    into the missing code, which unpacks to zero in both planes.
#include "common.h"
#include "kernels.h"

namespace ccc {

namespace {

constexpr unsigned kRho0Table = 0x00000102u;  // code 0,1,2,3 -> 2,1,0,0
constexpr unsigned kRho1Table = 0x02000100u;  // code 0,1,2,3 -> 0,1,0,2
constexpr unsigned kLow2 = 0x03030303u;

__device__ __forceinline__ void unpack16(unsigned w, v4i& r0, v4i& r1) {
  unsigned c0 = w & kLow2, c1 = (w >> 2) & kLow2, c2 = (w >> 4) & kLow2, c3 = (w >> 6) & kLow2;
  r0 = v4i{(int)__builtin_amdgcn_perm(0u, kRho0Table, c0),
           (int)__builtin_amdgcn_perm(0u, kRho0Table, c1),
           (int)__builtin_amdgcn_perm(0u, kRho0Table, c2),
           (int)__builtin_amdgcn_perm(0u, kRho0Table, c3)};
  r1 = v4i{(int)__builtin_amdgcn_perm(0u, kRho1Table, c0),
           (int)__builtin_amdgcn_perm(0u, kRho1Table, c1),
           (int)__builtin_amdgcn_perm(0u, kRho1Table, c2),
           (int)__builtin_amdgcn_perm(0u, kRho1Table, c3)};
}

__device__ __forceinline__ unsigned word_of(const u4& x, int s) {
  return s == 0 ? x.x : (s == 1 ? x.y : (s == 2 ? x.z : x.w));
}

template <int WM, int WN>
__device__ __forceinline__ void mma_superstep(const u4 (&pa)[WM], const u4 (&pb)[WN],
                                              v4i (&acc)[WM][WN][4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    v4i a0[WM], a1[WM], b0[WN], b1[WN];
#pragma unroll
    for (int m = 0; m < WM; ++m) unpack16(word_of(pa[m], s), a0[m], a1[m]);
#pragma unroll
    for (int n = 0; n < WN; ++n) unpack16(word_of(pb[n], s), b0[n], b1[n]);
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int n = 0; n < WN; ++n) {
        acc[m][n][0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0[m], b0[n], acc[m][n][0], 0, 0, 0);
        acc[m][n][1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0[m], b1[n], acc[m][n][1], 0, 0, 0);
        acc[m][n][2] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1[m], b0[n], acc[m][n][2], 0, 0, 0);
        acc[m][n][3] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1[m], b1[n], acc[m][n][3], 0, 0, 0);
      }
  }
}

template <int WM, int WN>
__global__ __launch_bounds__(256, 2) void mfma2_kernel(Pair2Args a, int64_t tiles_side,
                                                       int64_t tiles_n) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  static_assert(BM == 2 * BN, "triangle split assumes BM = 2 BN");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t I, J;
  if (a.tri) {
    int64_t sq_i, sq_j;
    tri_tile(blockIdx.x >> 1, tiles_side, sq_i, sq_j);
    I = sq_i;
    J = 2 * sq_j + (blockIdx.x & 1);
  } else {
    I = blockIdx.x / tiles_n;
    J = blockIdx.x % tiles_n;
  }
  const int64_t row0 = I * BM + (wave & 1) * 16 * WM;
  const int64_t col0 = J * BN + (wave >> 1) * 16 * WN;
  if (row0 >= a.n_a || col0 >= a.n_b) return;
  if (a.tri && row0 >= col0 + 16 * WN - 1) return;  // no pair i < j in this wave tile

  const int g = lane >> 4, rl = lane & 15;
  const uint8_t* pa[WM];
  const uint8_t* pb[WN];
#pragma unroll
  for (int m = 0; m < WM; ++m) {
    int64_t r = row0 + 16 * m + rl;
    pa[m] = a.va + (r < a.n_a ? r : a.n_a - 1) * a.lda + 16 * g;
  }
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    int64_t r = col0 + 16 * n + rl;
    pb[n] = a.vb + (r < a.n_b ? r : a.n_b - 1) * a.ldb + 16 * g;
  }

  v4i acc[WM][WN][4];
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int n = 0; n < WN; ++n)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[m][n][e] = v4i{0, 0, 0, 0};

  // Super-steps of 256 fields (64 bytes per row).  The first nfull are
  // entirely inside n_f (so inside the row stride); one masked step follows.
  const int64_t nfull = a.n_f / 256;
  const int64_t nbytes = (a.n_f + 3) / 4;
  u4 ca[WM], cb[WN];
  if (nfull > 0) {
#pragma unroll
    for (int m = 0; m < WM; ++m) ca[m] = *reinterpret_cast<const u4*>(pa[m]);
#pragma unroll
    for (int n = 0; n < WN; ++n) cb[n] = *reinterpret_cast<const u4*>(pb[n]);
  }
  for (int64_t s = 0; s < nfull; ++s) {
    u4 na[WM], nb[WN];
    const int64_t kn = (s + 1) * 64;
    if (s + 1 < nfull) {
#pragma unroll
      for (int m = 0; m < WM; ++m) na[m] = *reinterpret_cast<const u4*>(pa[m] + kn);
#pragma unroll
      for (int n = 0; n < WN; ++n) nb[n] = *reinterpret_cast<const u4*>(pb[n] + kn);
    }
    mma_superstep<WM, WN>(ca, cb, acc);
#pragma unroll
    for (int m = 0; m < WM; ++m) ca[m] = na[m];
#pragma unroll
    for (int n = 0; n < WN; ++n) cb[n] = nb[n];
  }
  const int64_t kt = nfull * 64;
  if (kt < nbytes) {
    // row pointers already include the lane's 16*g byte offset
#pragma unroll
    for (int m = 0; m < WM; ++m) ca[m] = load_fields64(pa[m] - 16 * g, kt + 16 * g, a.n_f);
#pragma unroll
    for (int n = 0; n < WN; ++n) cb[n] = load_fields64(pb[n] - 16 * g, kt + 16 * g, a.n_f);
    mma_superstep<WM, WN>(ca, cb, acc);
  }

  // Epilogue: lane holds rows 4g + e (e = 0..3) of column rl of each 16x16 block.
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int n = 0; n < WN; ++n)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = row0 + 16 * m + 4 * g + e;
        const int64_t j = col0 + 16 * n + rl;
        if (i >= a.n_a || j >= a.n_b || (a.tri && i >= j)) continue;
        v4i t = v4i{acc[m][n][0][e], acc[m][n][1][e], acc[m][n][2][e], acc[m][n][3][e]};
        int64_t p = a.tri ? pair_index(a.n_a, i, j) : i * a.n_b + j;
        if (a.accumulate) t = t + *reinterpret_cast<const v4i*>(a.tables + 4 * p);
        v4i ci = reinterpret_cast<const v4i*>(a.counts_a)[i];
        v4i cj = reinterpret_cast<const v4i*>(a.counts_b)[j];
        store_pair(p, t, ci, cj, a.gamma, a.tables, a.ccc);
      }
}

template <int WM, int WN>
hipError_t launch_shape(const Pair2Args& a, hipStream_t stream) {
  constexpr int BM = 32 * WM, BN = 32 * WN;
  int64_t tm = (a.n_a + BM - 1) / BM, tn = (a.n_b + BN - 1) / BN;
  int64_t ntiles = a.tri ? tm * (tm + 1) : tm * tn;  // triangle: two halves per square
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  timing_begin("mfma2", stream);
  hipLaunchKernelGGL((mfma2_kernel<WM, WN>), dim3((unsigned)ntiles), dim3(256), 0, stream, a, tm,
                     tn);
  timing_end(stream);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mfma2(const Pair2Args& a, hipStream_t stream) {
  return launch_shape<4, 2>(a, stream);
}

}  // namespace ccc
