// mfma3.hip -- 3-way tallies on the int8 matrix cores (v_mfma_i32_16x16x64_i8).
//
// For a fixed middle vector j (Sec. 2.2, Eq. (5)):
//   C_ijk(a,b,c) = sum_q rho_i(a) * (rho_j(b) rho_k(c))
// i.e. a 2-way product of the i-side planes R_a against j-modulated k-side
// planes M_bc[k][q] = rho_{j,q}(b) rho_{k,q}(c) in {0,1,2,4}.  This plays the
// role of the paper's X_{j,xi} construction (Table 1), which restricts a 2-way
// tally by the genotype of v_j; here the restriction is folded into the
// operand values, so one pass over the fields gives all 8 entries
// (8 int8 MACs per comparison).
//
// Building M_bc costs one v_perm_b32 per 4 bytes: the selector is
// code_k | J_b(code_j), with J_b = 0 where rho_j(b) = 1 (pick rho_k(c) from
// the low table), 4 where rho_j(b) = 2 (pick 2 rho_k(c) from the high
// table) and 8 where rho_j(b) = 0 (selectors 8..11 replicate the sign bit of
// a table byte, and every table byte is below 0x80, so they give 0).
//
// Schedule: a work unit is (I tile, K tile, j) with I tile rows below j and K
// tile columns above j (tetrahedral: only i < j < k is ever stored).  A
// workgroup is 2 x 2 waves over a (32 WI) x (32 WK) tile for one j; waves
// whose whole tile has no valid (i, k) exit at once.
#include "tile3.h"

namespace ccc {

namespace {

constexpr unsigned kRho0Table = 0x00000102u;   // code -> rho(0): 2,1,0,0
constexpr unsigned kRho1Table = 0x02000100u;   // code -> rho(1): 0,1,0,2
constexpr unsigned kRho0Twice = 0x00000204u;   // 2 rho(0)
constexpr unsigned kRho1Twice = 0x04000200u;   // 2 rho(1)
constexpr unsigned kSelJ0 = 0x08080004u;       // code_j -> J_0: rho_j(0)=2,1,0,0 -> 4,0,8,8
constexpr unsigned kSelJ1 = 0x04080008u;       // code_j -> J_1: rho_j(1)=0,1,0,2 -> 8,0,8,4
constexpr unsigned kLow2 = 0x03030303u;

constexpr int WI = 2;  // 16-row blocks per wave along i
constexpr int WK = 2;  // 16-column blocks per wave along k
constexpr int BI = 32 * WI;
constexpr int BK = 32 * WK;

__device__ __forceinline__ unsigned word_of(const u4& x, int s) {
  return s == 0 ? x.x : (s == 1 ? x.y : (s == 2 ? x.z : x.w));
}

__device__ __forceinline__ void codes4(unsigned w, unsigned (&c)[4]) {
  c[0] = w & kLow2;
  c[1] = (w >> 2) & kLow2;
  c[2] = (w >> 4) & kLow2;
  c[3] = (w >> 6) & kLow2;
}

__global__ __launch_bounds__(256, 2) void mfma3_kernel(Triple3Args a,
                                                       const int64_t* __restrict__ offs,
                                                       int64_t unit_base) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t n = a.n;
  const int64_t u = unit_base + blockIdx.x;
  int64_t j, it, kt;
  unit_coords(u, n, BI, BK, a.i_begin, a.i_end, offs, j, it, kt);

  const int64_t row0 = it * BI + (wave & 1) * 16 * WI;  // i range of this wave
  const int64_t col0 = kt * BK + (wave >> 1) * 16 * WK; // k range of this wave
  if (row0 >= j || col0 + 16 * WK - 1 <= j || col0 >= n) return;

  const int g = lane >> 4, rl = lane & 15;
  const uint8_t* pa[WI];
  const uint8_t* pk[WK];
#pragma unroll
  for (int m = 0; m < WI; ++m) {
    int64_t rr = row0 + 16 * m + rl;
    pa[m] = a.v + (rr < n ? rr : n - 1) * a.ld + 16 * g;
  }
#pragma unroll
  for (int c = 0; c < WK; ++c) {
    int64_t rr = col0 + 16 * c + rl;
    pk[c] = a.v + (rr < n ? rr : n - 1) * a.ld + 16 * g;
  }
  const uint8_t* pj = a.v + j * a.ld + 16 * g;

  v4i acc[WI][WK][8];
#pragma unroll
  for (int m = 0; m < WI; ++m)
#pragma unroll
    for (int c = 0; c < WK; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[m][c][e] = v4i{0, 0, 0, 0};

  const int64_t nbytes = (a.n_f + 3) / 4;
  for (int64_t kb = 0; kb < nbytes; kb += 64) {
    const bool full = (kb + 64) * 4 <= a.n_f;
    u4 xa[WI], xk[WK], xj;
    if (full) {
#pragma unroll
      for (int m = 0; m < WI; ++m) xa[m] = *reinterpret_cast<const u4*>(pa[m] + kb);
#pragma unroll
      for (int c = 0; c < WK; ++c) xk[c] = *reinterpret_cast<const u4*>(pk[c] + kb);
      xj = *reinterpret_cast<const u4*>(pj + kb);
    } else {
#pragma unroll
      for (int m = 0; m < WI; ++m) xa[m] = load_fields64(pa[m] - 16 * g, kb + 16 * g, a.n_f);
#pragma unroll
      for (int c = 0; c < WK; ++c) xk[c] = load_fields64(pk[c] - 16 * g, kb + 16 * g, a.n_f);
      xj = load_fields64(pj - 16 * g, kb + 16 * g, a.n_f);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      unsigned cj[4], sel0[4], sel1[4];
      codes4(word_of(xj, s), cj);
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        sel0[t] = __builtin_amdgcn_perm(0u, kSelJ0, cj[t]);
        sel1[t] = __builtin_amdgcn_perm(0u, kSelJ1, cj[t]);
      }
      v4i A0[WI], A1[WI];
#pragma unroll
      for (int m = 0; m < WI; ++m) {
        unsigned ca[4];
        codes4(word_of(xa[m], s), ca);
        A0[m] = v4i{(int)__builtin_amdgcn_perm(0u, kRho0Table, ca[0]),
                    (int)__builtin_amdgcn_perm(0u, kRho0Table, ca[1]),
                    (int)__builtin_amdgcn_perm(0u, kRho0Table, ca[2]),
                    (int)__builtin_amdgcn_perm(0u, kRho0Table, ca[3])};
        A1[m] = v4i{(int)__builtin_amdgcn_perm(0u, kRho1Table, ca[0]),
                    (int)__builtin_amdgcn_perm(0u, kRho1Table, ca[1]),
                    (int)__builtin_amdgcn_perm(0u, kRho1Table, ca[2]),
                    (int)__builtin_amdgcn_perm(0u, kRho1Table, ca[3])};
      }
#pragma unroll
      for (int c = 0; c < WK; ++c) {
        unsigned ck[4];
        codes4(word_of(xk[c], s), ck);
        v4i M[4];  // (b,c) = 00, 01, 10, 11
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          unsigned s0 = ck[t] | sel0[t], s1 = ck[t] | sel1[t];
          M[0][t] = (int)__builtin_amdgcn_perm(kRho0Twice, kRho0Table, s0);
          M[1][t] = (int)__builtin_amdgcn_perm(kRho1Twice, kRho1Table, s0);
          M[2][t] = (int)__builtin_amdgcn_perm(kRho0Twice, kRho0Table, s1);
          M[3][t] = (int)__builtin_amdgcn_perm(kRho1Twice, kRho1Table, s1);
        }
#pragma unroll
        for (int m = 0; m < WI; ++m) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            acc[m][c][e] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A0[m], M[e], acc[m][c][e], 0, 0, 0);
            acc[m][c][4 + e] =
                __builtin_amdgcn_mfma_i32_16x16x64_i8(A1[m], M[e], acc[m][c][4 + e], 0, 0, 0);
          }
        }
      }
    }
  }

  // Epilogue: entry 4a + 2b + c; lane holds rows 4g + e of column rl.
  double wj[2];
  vector_factors(a.counts, j, a.gamma, wj);
#pragma unroll
  for (int m = 0; m < WI; ++m)
#pragma unroll
    for (int c = 0; c < WK; ++c) {
      const int64_t k = col0 + 16 * c + rl;
      const bool kvalid = k > j && k < n;
      double wk[2];
      vector_factors(a.counts, kvalid ? k : j, a.gamma, wk);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = row0 + 16 * m + 4 * g + e;
        int t[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) t[x] = acc[m][c][x][e];
        emit_triple(a, kvalid && i < j, i, j, k, t, wj, wk);
      }
    }
}

}  // namespace

hipError_t launch_mfma3(const Triple3Args& a, hipStream_t stream) {
  return launch_units(mfma3_kernel, a, BI, BK, "mfma3", stream);
}

}  // namespace ccc
