// mfma3.hip -- 3-way tallies on the matrix cores (fp4 or int8 operands).
//
// For a fixed middle vector j (Sec. 2.2, Eq. (5)):
//   C_ijk(a,b,c) = sum_q rho_i(a) * (rho_j(b) rho_k(c))
// i.e. a 2-way product of i-side planes against j-modulated k-side planes.
// This plays the role of the paper's X_{j,xi} construction (Table 1), which
// restricts a 2-way tally by the genotype of v_j; here the restriction is
// folded into the operand values, so one pass over the fields gives all 8
// entries (8 MACs per comparison).
//
// Kernels:
//   mfma3_run_kernel       fp4, every call that is not complete: units of four
//                          consecutive j over a pair of 32-row tiles, one j per
//                          wave, the i and k planes shared through LDS;
//   mfma3_complete_kernel  fp4, calls whose every row is complete (a device
//                          flag picks it): one plane, units of four j over a
//                          pair of 64-row tiles;
//   mfma3_kernel           int8 operands: units of one j over a pair of 64-row
//                          tiles, 2 x 2 waves; a unit whose rows are complete
//                          takes the one-plane form together;
//   gram1_kernel           the rho(1) Gram matrix of the complete-data formula.
//
// int8 operands: M_bc[k][q] = rho_{j,q}(b) rho_{k,q}(c) in {0,1,2,4}, one
// v_perm_b32 per 4 bytes: the selector is code_k | J_b(code_j), with J_b = 0
// where rho_j(b) = 1 (pick rho_k(c) from the low table), 4 where rho_j(b) = 2
// (pick 2 rho_k(c) from the high table) and 8 where rho_j(b) = 0 (selectors
// 8..11 replicate the sign bit of a table byte, and every table byte is below
// 0x80, so they give 0).
//
// Schedule: a work unit is (I tile, K tile, j or a run of j) with I tile rows
// below j and K tile columns above j (tetrahedral: only i < j < k is ever
// stored).
//
// Complete data (every row of a unit, and v_j, has all n_f fields present, as
// the 1-way counts of the call say): with rho(0) = 2 - rho(1) on every field
// the 8 entries follow from the single triple sum
//   S_xyz = sum_q rho_i(1) rho_j(1) rho_k(1)
// together with the pair sums S_xy, S_xz, S_yz (one dense rho(1) Gram matrix
// G computed before the unit kernel), the allele counts n(1) and n_f:
//   C(1,1,1) = S_xyz,  C(1,1,0) = 2 S_xy - S_xyz, ...,
//   C(0,0,0) = 8 n_f - 4 (n_i + n_j + n_k) + 2 (S_xy + S_xz + S_yz) - S_xyz
// (expand the product of (2 - x) and x factors).  One MFMA plane replaces
// eight.
#include <type_traits>

#include "tile2.h"
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
static_assert(BI == kUnitTile && BK == kUnitTile, "work units are kUnitTile-row tile pairs");

__device__ __forceinline__ unsigned word_of(const u4& x, int s) {
  return s == 0 ? x.x : (s == 1 ? x.y : (s == 2 ? x.z : x.w));
}

__device__ __forceinline__ void codes4(unsigned w, unsigned (&c)[4]) {
  c[0] = w & kLow2;
  c[1] = (w >> 2) & kLow2;
  c[2] = (w >> 4) & kLow2;
  c[3] = (w >> 6) & kLow2;
}

// ---------------------------------------------------------------------------
// fp4 form (n_f <= kF4MaxFields; operands as in the 2-way fp4 form: a 2-bit
// value x in a nibble is the e2m1 number x / 2).  Planes rho(1) = R and P for
// i and k; D = rho(1) - P (values -1, 0, 1) and P for j.  The k-side operands
// are modulated by j field by field:
//   D_j Z_k: Z_k's nibble where D_j != 0, with the e2m1 sign bit set where
//            D_j = -1 (code 00): one v_bitop3, (z & m) ^ sign;
//   P_j Z_k: Z_k's nibble where P_j = 1: one AND.
// The eight sums S[x][y][z] = sum x_i y_j z_k (x, z in {R, P}, y in {D, P};
// each is 4x its fp32 accumulator, a multiple of 1/4 of magnitude <= n_f,
// exact) give the table through rho(1) = R, rho(0) = 2P - R on i and k and
// rho_j(1) = D + P, rho_j(0) = P - D.

// j's masks for the two operand registers (even, odd fields) of one packed
// word: y = both value bits where D != 0, sg = the sign bit where D = -1,
// p = both value bits where P = 1.  v_bitop3 tables on (a = w, b = w >> 1,
// c = field mask): 0x82 = c & ~(a ^ b), 0x02 = c & ~a & ~b, 0xA2 = c & (a | ~b).
__device__ __forceinline__ void j_masks_f4(unsigned w, unsigned* y, unsigned* sg, unsigned* p) {
  const unsigned s = w >> 1;
  unsigned t = __builtin_amdgcn_bitop3_b32(w, s, 0x11111111u, 0x82);
  y[0] = t | (t << 1);
  t = __builtin_amdgcn_bitop3_b32(w, s, 0x44444444u, 0x82) >> 2;
  y[1] = t | (t << 1);
  sg[0] = __builtin_amdgcn_bitop3_b32(w, s, 0x11111111u, 0x02) << 3;
  sg[1] = __builtin_amdgcn_bitop3_b32(w, s, 0x44444444u, 0x02) << 1;
  if (p) {
    t = __builtin_amdgcn_bitop3_b32(w, s, 0x11111111u, 0xA2);
    p[0] = t | (t << 1);
    t = __builtin_amdgcn_bitop3_b32(w, s, 0x44444444u, 0xA2) >> 2;
    p[1] = t | (t << 1);
  }
}

// j_masks_f4 of two words w0 (into y[0..1], sg[0..1], p[0..1]) and w1 (into
// y[2..3] ...), with the shifts paired (twenty-five operations instead of
// thirty).  Crossing bits: s takes w1's bit 0 into bit 31, which every mask
// drops; the >> 2 moves bits that sit at 2 mod 4 (w1's bits 0-1 are zero);
// the << 3 and << 1 move bits that sit at 0 mod 4 and 2 mod 4 (w0's bits
// 29-31 are zero).
__device__ __forceinline__ void j_masks32_f4(unsigned w0, unsigned w1, unsigned* y, unsigned* sg,
                                             unsigned* p) {
  unsigned s0, s1, a, b;
  tile2::shr_pair<1>(w0, w1, s0, s1);
  unsigned t0 = __builtin_amdgcn_bitop3_b32(w0, s0, 0x11111111u, 0x82);
  unsigned t1 = __builtin_amdgcn_bitop3_b32(w1, s1, 0x11111111u, 0x82);
  y[0] = t0 | (t0 << 1);
  y[2] = t1 | (t1 << 1);
  tile2::shr_pair<2>(__builtin_amdgcn_bitop3_b32(w0, s0, 0x44444444u, 0x82),
                     __builtin_amdgcn_bitop3_b32(w1, s1, 0x44444444u, 0x82), a, b);
  y[1] = a | (a << 1);
  y[3] = b | (b << 1);
  tile2::shl_pair<3>(__builtin_amdgcn_bitop3_b32(w0, s0, 0x11111111u, 0x02),
                     __builtin_amdgcn_bitop3_b32(w1, s1, 0x11111111u, 0x02), sg[0], sg[2]);
  tile2::shl_pair<1>(__builtin_amdgcn_bitop3_b32(w0, s0, 0x44444444u, 0x02),
                     __builtin_amdgcn_bitop3_b32(w1, s1, 0x44444444u, 0x02), sg[1], sg[3]);
  if (p) {
    t0 = __builtin_amdgcn_bitop3_b32(w0, s0, 0x11111111u, 0xA2);
    t1 = __builtin_amdgcn_bitop3_b32(w1, s1, 0x11111111u, 0xA2);
    p[0] = t0 | (t0 << 1);
    p[2] = t1 | (t1 << 1);
    tile2::shr_pair<2>(__builtin_amdgcn_bitop3_b32(w0, s0, 0x44444444u, 0xA2),
                       __builtin_amdgcn_bitop3_b32(w1, s1, 0x44444444u, 0xA2), a, b);
    p[1] = a | (a << 1);
    p[3] = b | (b << 1);
  }
}

// (z & m) ^ sg: z modulated by D_j.
__device__ __forceinline__ unsigned mod_d(unsigned z, unsigned m, unsigned sg) {
  return __builtin_amdgcn_bitop3_b32(z, m, sg, 0x6A);
}

// Table entry 4a + 2b + c from the eight sums (index 4x + 2y + z).
__device__ __forceinline__ void table3_f4(const int (&S)[8], int (&t)[8]) {
  int T[8], U[8];
#pragma unroll
  for (int xy = 0; xy < 4; ++xy) {  // k: rho(1) = R, rho(0) = 2P - R
    T[2 * xy + 1] = S[2 * xy];
    T[2 * xy] = 2 * S[2 * xy + 1] - S[2 * xy];
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)  // j: rho(1) = D + P, rho(0) = P - D
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      U[4 * x + 2 + c] = T[4 * x + c] + T[4 * x + 2 + c];
      U[4 * x + c] = T[4 * x + 2 + c] - T[4 * x + c];
    }
#pragma unroll
  for (int bc = 0; bc < 4; ++bc) {  // i: rho(1) = R, rho(0) = 2P - R
    t[4 + bc] = U[bc];
    t[bc] = 2 * U[4 + bc] - U[bc];
  }
}

// General unit, one wave, int8 operands: the (16 WI) x (16 WK) tile of
// (i, k) at rows row0.., columns col0.. for middle vector j, eight MFMA
// planes.  `active`: the tile holds a triple i < j < k; inactive waves return
// at once.
__device__ __forceinline__ void general_wave(const Triple3Args& a, int64_t j, int64_t row0,
                                             int64_t col0, bool active) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63;
  const int64_t n = a.n;
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

  if (!active) return;

  v4i acc[WI][WK][8];
#pragma unroll
  for (int m = 0; m < WI; ++m)
#pragma unroll
    for (int c = 0; c < WK; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[m][c][e] = v4i{0, 0, 0, 0};

  auto body = [&](const u4 (&xa)[WI], const u4 (&xk)[WK], const u4& xj) {
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
  };
  // Whole 256-field super-steps with plain loads, then the masked tail.
  const int64_t nfull = a.n_f / 256;
  for (int64_t st = 0; st < nfull; ++st) {
    const int64_t kb = st * 64;
    u4 xa[WI], xk[WK];
#pragma unroll
    for (int m = 0; m < WI; ++m) xa[m] = *reinterpret_cast<const u4*>(pa[m] + kb);
#pragma unroll
    for (int c = 0; c < WK; ++c) xk[c] = *reinterpret_cast<const u4*>(pk[c] + kb);
    body(xa, xk, *reinterpret_cast<const u4*>(pj + kb));
  }
  if (nfull * 256 < a.n_f) {
    const int64_t kb = nfull * 64 + 16 * g;
    u4 xa[WI], xk[WK];
#pragma unroll
    for (int m = 0; m < WI; ++m) xa[m] = load_fields64(pa[m] - 16 * g, kb, a.n_f);
#pragma unroll
    for (int c = 0; c < WK; ++c) xk[c] = load_fields64(pk[c] - 16 * g, kb, a.n_f);
    body(xa, xk, load_fields64(pj - 16 * g, kb, a.n_f));
  }

  // Epilogue: entry 4a + 2b + c; lane holds rows 4g + e of column rl.
  double wj[2], wk[WK][2];
  triple_factors(a, j, wj);
#pragma unroll
  for (int c = 0; c < WK; ++c) triple_factors(a, col0 + 16 * c + rl, wk[c]);
#pragma unroll
  for (int m = 0; m < WI; ++m)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = row0 + 16 * m + 4 * g + e;
      double wi[2];
      triple_factors(a, i, wi);
#pragma unroll
      for (int c = 0; c < WK; ++c) {
        const int64_t k = col0 + 16 * c + rl;
        int t[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) t[x] = acc[m][c][x][e];
        emit_triple(a, k > j && k < n && i < j, i, j, k, t, wi, wj, wk[c]);
      }
    }
}

// The 16 triples a lane holds in one 16-row block of a complete-data tile:
// rows ib + 4g + e (e = 0..3), columns k0 + 16c + rl (c = 0..3), middle
// vector j.  xyz[c][e] is S_xyz (fp4: the sum modulated by D_j, to which
// G[i][k] is added here); the pair sums come from the Gram matrix and the
// single counts from the 1-way counts.  fp4: the dense output is staged
// through `scratch` (384 x 16 bytes of this wave's LDS).
template <bool F4>
__device__ __forceinline__ void complete_block_row(const Triple3Args& a, int64_t j, int64_t ib,
                                                   int64_t k0, const v4i (&xyz)[4],
                                                   u4* scratch) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const int64_t n = a.n;
  const v4i* cnt = reinterpret_cast<const v4i*>(a.counts);
  const int64_t ng = a.ng, g0 = a.g0;
  const unsigned S8 = 8u * (unsigned)a.n_f, Y = (unsigned)cnt[j].y;
  const int32_t* grow_j = a.gram + (j - g0) * ng;
  double wj[2], wk[4][2];
  triple_factors(a, j, wj);
  unsigned Z[4], YZ[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t k = k0 + 16 * c + rl;
    const int64_t kk = k > j && k < n ? k : j;  // a valid row for invalid lanes
    triple_factors(a, kk, wk[c]);
    Z[c] = (unsigned)cnt[kk].y;
    YZ[c] = (unsigned)grow_j[kk - g0];
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int64_t i = ib + 4 * g + e;
    const int64_t ii = i < j ? i : j;  // a valid row for invalid lanes
    double wi[2];
    triple_factors(a, ii, wi);
    const unsigned X = (unsigned)cnt[ii].y;
    const int32_t* grow_i = a.gram + (ii - g0) * ng;
    const unsigned XY = (unsigned)grow_i[j - g0];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t k = k0 + 16 * c + rl;
      const bool valid = k > j && k < n && i < j;
      const int64_t kk = k > j && k < n ? k : j;
      const unsigned XZ = (unsigned)grow_i[kk - g0];
      // fp4: the partial sums hold sum rho_i(1) D_j rho_k(1)
      const unsigned XYZ = F4 ? XZ + (unsigned)xyz[c][e] : (unsigned)xyz[c][e];
      int t[8];
      t[7] = (int)XYZ;
      t[6] = (int)(2u * XY - XYZ);
      t[5] = (int)(2u * XZ - XYZ);
      t[3] = (int)(2u * YZ[c] - XYZ);
      t[4] = (int)(4u * X - 2u * XY - 2u * XZ + XYZ);
      t[2] = (int)(4u * Y - 2u * XY - 2u * YZ[c] + XYZ);
      t[1] = (int)(4u * Z[c] - 2u * XZ - 2u * YZ[c] + XYZ);
      t[0] = (int)(S8 - 4u * (X + Y + Z[c]) + 2u * (XY + XZ + YZ[c]) - XYZ);
      if constexpr (F4)
        emit_triple_staged(a, valid, i, j, k, t, wi, wj, wk[c], scratch);
      else
        emit_triple(a, valid, i, j, k, t, wi, wj, wk[c]);
    }
  }
}

// Complete-data unit of the int8 form (see the notes at the top): all four
// waves build the same 64 x 64 tile of S_xyz over a quarter of the 256-field
// super-steps each, the partial sums meet in LDS, and wave w finishes rows
// 16w..16w+15.
__device__ __forceinline__ void complete_unit(const Triple3Args& a, int64_t j, int64_t i0,
                                              int64_t k0, v4i (*part)[16][64]) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, rl = lane & 15;
  const int64_t n = a.n;
  const uint8_t* pa[4];
  const uint8_t* pk[4];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int64_t rr = i0 + 16 * m + rl;
    pa[m] = a.v + (rr < n ? rr : n - 1) * a.ld + 16 * g;
    rr = k0 + 16 * m + rl;
    pk[m] = a.v + (rr < n ? rr : n - 1) * a.ld + 16 * g;
  }
  const uint8_t* pj = a.v + j * a.ld + 16 * g;

  v4i acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[m][c] = v4i{0, 0, 0, 0};

  const int64_t steps = (a.n_f + 255) / 256;
  const int64_t s_begin = steps * wave / 4, s_end = steps * (wave + 1) / 4;
  for (int64_t st = s_begin; st < s_end; ++st) {
    const int64_t kb = st * 64;
    const bool full = (kb + 64) * 4 <= a.n_f;
    u4 xa[4], xk[4], xj;
    if (full) {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        xa[m] = *reinterpret_cast<const u4*>(pa[m] + kb);
        xk[m] = *reinterpret_cast<const u4*>(pk[m] + kb);
      }
      xj = *reinterpret_cast<const u4*>(pj + kb);
    } else {
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        xa[m] = load_fields64(pa[m] - 16 * g, kb + 16 * g, a.n_f);
        xk[m] = load_fields64(pk[m] - 16 * g, kb + 16 * g, a.n_f);
      }
      xj = load_fields64(pj - 16 * g, kb + 16 * g, a.n_f);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      unsigned cj[4], sel1[4];
      codes4(word_of(xj, s), cj);
#pragma unroll
      for (int t = 0; t < 4; ++t) sel1[t] = __builtin_amdgcn_perm(0u, kSelJ1, cj[t]);
      v4i A1[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) A1[m] = tile2::unpack16_rho1(word_of(xa[m], s));
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        unsigned ck[4];
        codes4(word_of(xk[c], s), ck);
        v4i M;  // rho_j(1) rho_k(1)
#pragma unroll
        for (int t = 0; t < 4; ++t)
          M[t] = (int)__builtin_amdgcn_perm(kRho1Twice, kRho1Table, ck[t] | sel1[t]);
#pragma unroll
        for (int m = 0; m < 4; ++m)
          acc[m][c] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A1[m], M, acc[m][c], 0, 0, 0);
      }
    }
  }

#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) part[wave][4 * m + c][lane] = acc[m][c];
  __syncthreads();

  v4i xyz[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    xyz[c] = part[0][4 * wave + c][lane] + part[1][4 * wave + c][lane] +
             part[2][4 * wave + c][lane] + part[3][4 * wave + c][lane];
  }
  complete_block_row<false>(a, j, i0 + 16 * wave, k0, xyz, nullptr);
}

// Middle vectors per unit of the complete-data kernel: one per wave.
constexpr int64_t kJRun = 4;

// Complete-data kernel, for calls whose every row has all n_f fields present
// (the flag set by complete3_flag_kernel picks it; it exits at once
// otherwise).  A workgroup takes a run of kJRun consecutive middle vectors j
// of one tile pair (I tile, K tile), one per wave, and each wave computes the
// whole 64 x 64 (i, k) tile of S_xyz = G[i][k] + sum rho_i(1) D_j rho_k(1)
// for its j over every field (4 x 4 blocks of one fp4 plane).
//
// The four waves need the same rho(1) operands of the unit's 4 i blocks and
// 4 k blocks; only D_j (and so the modulation of the k operands) is their
// own.  So per super-step the rows travel through the workgroup's LDS stage
// once (`raw`: 4 i blocks, 4 k blocks, and one block holding the run's j
// rows, lane l the row j0 + min(l & 15, jn - 1)), each wave turns two of the
// 8 row blocks into rho(1) nibbles and writes them to `planes`, and every
// wave reads all 8 back.  The steps are skewed by one: in step s a wave
// builds the planes of step s + 1 (and keeps its j word of step s + 1)
// while it multiplies those of step s, so one barrier per step covers both
// buffers: raw(s + 1) has landed, planes(s) are written, and the buffers of
// step s - 1 are free (raw(s + 2) goes into the buffer of raw(s), which was
// read in step s - 1).  The last, padded step takes plain loads.
__global__ __launch_bounds__(256, 3) void mfma3_complete_kernel(Triple3Args a, UnitGrid ug,
                                                                const int64_t* __restrict__ offs,
                                                                int64_t unit_base,
                                                                int64_t count) {
#pragma clang fp contract(off)
  if (*a.complete == 0) return;  // uniform
  constexpr int NB = 9, BPW = 3;  // raw row blocks per step; copies per wave (the last idle)
  __shared__ u4 raw[2][NB][64];        // 18 KB
  __shared__ u4 planes[2][8][2][64];   // 32 KB: [step & 1][block][half][lane]; then store staging
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int64_t n = a.n;
  const int64_t u = unit_base + xcd_unit(blockIdx.x, count);
  int64_t j0, it, kt, jlo, jhi;
  unit_coords(u, ug, offs, j0, it, kt);
  pair_j_range(ug, it, kt, jlo, jhi);
  const int64_t jn = jhi - j0 < kJRun ? jhi - j0 : kJRun;  // middle vectors of this run
  const int64_t j = j0 + (wave < jn ? wave : jn - 1);      // inactive waves repeat the last
  const bool active = wave < jn;
  const int64_t i0 = it * BI, k0 = kt * BK;

  // Copies: blocks 0-3 rows i, 4-7 rows k, 8 the run's j rows; a
  // wave-uniform base (the block's first row, clamped) plus a 32-bit lane
  // offset (r - rf < 16 rows of at most 2^28 bytes).
  gbytes base[BPW];
  uint32_t off[BPW];
#pragma unroll
  for (int t = 0; t < BPW; ++t) {
    const int b = BPW * wave + t < NB ? BPW * wave + t : NB - 1;
    int64_t r0, r1;
    if (b < 8) {
      r0 = (b < 4 ? i0 + 16 * b : k0 + 16 * (b - 4));
      r1 = r0 + rl;
    } else {
      r0 = j0;
      r1 = j0 + (rl < jn ? rl : jn - 1);
    }
    const int64_t rf = r0 < n ? r0 : n - 1, r = r1 < n ? r1 : n - 1;
    const uint64_t bp = (uint64_t)(a.v + rf * a.ld);
    base[t] = (gbytes)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bp >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)bp));
    off[t] = (uint32_t)((r - rf) * a.ld + 16 * g);
  }
  auto issue = [&](int64_t st, int buf) {
#pragma unroll
    for (int t = 0; t < BPW; ++t)
      if (BPW * wave + t < NB)
        tile2::stage_row((const uint8_t*)(base[t] + st * 64 + off[t]),
                         &raw[buf][BPW * wave + t][0]);
  };
  // this wave's share of the planes: blocks 2 wave and 2 wave + 1, both halves
  auto build = [&](int rbuf, int pbuf) {
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int b = 2 * wave + t;
      const u4 x = raw[rbuf][b][lane];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const v8i r = tile2::rho1_nibbles_complete(word_of(x, 2 * h), word_of(x, 2 * h + 1));
        planes[pbuf][b][h][lane] = u4{(unsigned)r[0], (unsigned)r[1], (unsigned)r[2],
                                      (unsigned)r[3]};
      }
    }
  };

  v4f acc[4][4];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[m][c] = v4f{0, 0, 0, 0};
  // the MFMAs of one half super-step from the 8 blocks' nibbles and j's word
  auto multiply = [&](const v8i (&A)[4], const v8i (&K)[4], unsigned wj0, unsigned wj1) {
    unsigned y[4], sg[4];
    j_masks_f4(wj0, y, sg, nullptr);
    j_masks_f4(wj1, y + 2, sg + 2, nullptr);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v8i B;
#pragma unroll
      for (int q = 0; q < 4; ++q) B[q] = (int)mod_d((unsigned)K[c][q], y[q], sg[q]);
#pragma unroll
      for (int q = 4; q < 8; ++q) B[q] = 0;
#pragma unroll
      for (int m = 0; m < 4; ++m) acc[m][c] = tile2::mfma_f4(A[m], B, acc[m][c]);
    }
  };
  auto as_v8 = [](const u4& x) { return v8i{(int)x.x, (int)x.y, (int)x.z, (int)x.w, 0, 0, 0, 0}; };

  const int64_t nfull = a.n_f / 256;
  u4 xj = u4{0, 0, 0, 0};  // this wave's j word of the step to multiply next
  if (nfull > 0) {
    issue(0, 0);
    if (nfull > 1) issue(1, 1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    build(0, 0);
    xj = raw[0][8][16 * g + wave];
  }
  for (int64_t st = 0; st < nfull; ++st) {
    const int buf = (int)(st & 1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // raw(st + 1) of this wave has landed
    __syncthreads();  // every wave's has; planes(st) are written; step st - 1's buffers are free
    const u4 xj_now = xj;
    if (st + 1 < nfull) {
      xj = raw[buf ^ 1][8][16 * g + wave];
      if (st + 2 < nfull) issue(st + 2, buf);
      build(buf ^ 1, buf ^ 1);
    }
    if (active) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v8i A[4], K[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          A[m] = as_v8(planes[buf][m][h][lane]);
          K[m] = as_v8(planes[buf][4 + m][h][lane]);
        }
        multiply(A, K, word_of(xj_now, 2 * h), word_of(xj_now, 2 * h + 1));
      }
    }
  }
  if (nfull * 256 < a.n_f && active) {
    const int64_t kb = nfull * 64 + 16 * g;
    u4 xa[4], xk[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      int64_t r = i0 + 16 * m + rl;
      xa[m] = load_fields64(a.v + (r < n ? r : n - 1) * a.ld, kb, a.n_f);
      r = k0 + 16 * m + rl;
      xk[m] = load_fields64(a.v + (r < n ? r : n - 1) * a.ld, kb, a.n_f);
    }
    const u4 xt = load_fields64(a.v + j * a.ld, kb, a.n_f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      v8i A[4], K[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        A[m] = tile2::nibbles32(tile2::rho1_16_f4<false>(word_of(xa[m], 2 * h)),
                                tile2::rho1_16_f4<false>(word_of(xa[m], 2 * h + 1)));
        K[m] = tile2::nibbles32(tile2::rho1_16_f4<false>(word_of(xk[m], 2 * h)),
                                tile2::rho1_16_f4<false>(word_of(xk[m], 2 * h + 1)));
      }
      multiply(A, K, word_of(xt, 2 * h), word_of(xt, 2 * h + 1));
    }
  }
  __syncthreads();  // every wave is done with `raw` and `planes`

  // The epilogue's inputs are read before any of its stores (a wait for a
  // load also waits for every store issued before it): the unit's Gram tile
  // G[i][k] into `raw` (one copy for the four waves), each wave's rows i
  // (their count n(1), G[i][j] and factors) into its 2 KB past the store
  // staging in `planes`, and its columns k and j into registers.
  const v4i* cnt = reinterpret_cast<const v4i*>(a.counts);
  const int64_t ng = a.ng, g0 = a.g0;
  int32_t(*gt)[64] = reinterpret_cast<int32_t(*)[64]>(&raw[0][0][0]);  // 16 KB of the 18
  {
    const int r = threadIdx.x >> 2, q = threadIdx.x & 3;  // row r, columns 16q ..
    const int64_t ir = (i0 + r < n ? i0 + r : n - 1) - g0;
    const int32_t* grow = a.gram + ir * ng;
    int32_t x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const int64_t k = k0 + 16 * q + t;
      x[t] = grow[(k < n ? k : n - 1) - g0];
    }
#pragma unroll
    for (int t = 0; t < 16; t += 4)
      *reinterpret_cast<v4i*>(&gt[r][16 * q + t]) = v4i{x[t], x[t + 1], x[t + 2], x[t + 3]};
  }
  struct RowIn {
    double w[2];
    int x, xy, pad0, pad1;
  };
  RowIn* rows = reinterpret_cast<RowIn*>(&planes[0][0][0][0] + 1536 + 128 * wave);  // 64 x 32 B
  if (active) {
    const int64_t i = i0 + lane, ii = i < n ? i : n - 1;
    RowIn ri;
    triple_factors(a, ii, ri.w);
    ri.x = cnt[ii].y;
    ri.xy = a.gram[(ii - g0) * ng + (j - g0)];
    ri.pad0 = ri.pad1 = 0;
    rows[lane] = ri;
  }
  const unsigned S8 = 8u * (unsigned)a.n_f, Y = (unsigned)cnt[j].y;
  double wj[2], wk[4][2];
  unsigned Z[4], YZ[4];
  triple_factors(a, j, wj);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t k = k0 + 16 * c + rl;
    const int64_t kk = k > j && k < n ? k : j;  // a valid row for invalid lanes
    triple_factors(a, kk, wk[c]);
    Z[c] = (unsigned)cnt[kk].y;
    YZ[c] = (unsigned)a.gram[(j - g0) * ng + (kk - g0)];
  }
  __syncthreads();  // the Gram tile is in place
  if (!active) return;

  // Epilogue: 4 block rows of 16 triples per lane for this wave's j
  // (S_xyz = G[i][k] + the modulated sums; the other pair sums from the Gram
  // matrix, the single counts from the 1-way counts).
  u4* outs = &planes[0][0][0][0] + 384 * wave;
  tile2::static_for<4>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = 16 * m + 4 * g + e;
      const int64_t i = i0 + r;
      const RowIn ri = rows[r];
      const unsigned X = (unsigned)ri.x, XY = (unsigned)ri.xy;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int64_t k = k0 + 16 * c + rl;
        const bool valid = k > j && k < n && i < j;
        const unsigned XZ = (unsigned)gt[r][16 * c + rl];
        const unsigned XYZ = XZ + (unsigned)tile2::f4_count(acc[m][c][e]);
        int t[8];
        t[7] = (int)XYZ;
        t[6] = (int)(2u * XY - XYZ);
        t[5] = (int)(2u * XZ - XYZ);
        t[3] = (int)(2u * YZ[c] - XYZ);
        t[4] = (int)(4u * X - 2u * XY - 2u * XZ + XYZ);
        t[2] = (int)(4u * Y - 2u * XY - 2u * YZ[c] + XYZ);
        t[1] = (int)(4u * Z[c] - 2u * XZ - 2u * YZ[c] + XYZ);
        t[0] = (int)(S8 - 4u * (X + Y + Z[c]) + 2u * (XY + XZ + YZ[c]) - XYZ);
        emit_triple_staged(a, valid, i, j, k, t, ri.w, wj, wk[c], outs);
      }
    }
  });
}

// General 3-way kernel on fp4 operands (calls that are not complete; it
// exits at once when the complete-data flag is set).  A workgroup takes a
// run of kJRun consecutive middle vectors j of one pair of 32-row tiles
// (I tile, K tile), one per wave; each wave computes the eight MFMA planes
// of the whole 32 x 32 (i, k) tile for its j over every field (2 x 2 blocks
// x 8 planes of accumulators).  The rho(1) and P planes of the unit's 2 i
// and 2 k blocks do not depend on j: per super-step the rows travel through
// the workgroup's LDS stage once (`raw`, wave w copying row block w: 2 i
// blocks, 2 k blocks), wave w turns row block w into its two planes and
// writes them to `planes`, and every wave reads all four back; only j's
// masks and the modulation of the k planes by D_j and P_j are each wave's
// own.  The steps are skewed by one as in mfma3_complete_kernel, so one
// barrier per step covers both buffers.
//
// j's masks are the same for the 16 lanes of a field group, so a wave makes
// them eight steps at a time: lane (g, l) turns the 32 fields of half l & 1
// of step 8b + (l >> 1) in group g into their masks and writes them to the
// wave's part of `jm`, and each half step reads its masks back (the 16
// lanes of a group read one address).  The words of batch b + 1 are loaded
// while batch b is multiplied.
__global__ __launch_bounds__(256, 2) void mfma3_run_kernel(Triple3Args a, UnitGrid ug,
                                                           const int64_t* __restrict__ offs,
                                                           int64_t unit_base, int64_t count) {
#pragma clang fp contract(off)
  if (a.complete && *a.complete) return;  // uniform: mfma3_complete_kernel covers the call
  __shared__ u4 raw[2][4][64];            // 8 KB: [step & 1][row block][lane]
  __shared__ u4 planes[2][4][2][2][64];   // 32 KB: [step & 1][block][half][rho(1), P][lane]
  __shared__ u4 jm[4][4][16][3];          // 12 KB: [wave][group][half step][y, sg, p]
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int64_t n = a.n;
  const int64_t u = unit_base + xcd_unit(blockIdx.x, count);
  int64_t j0, it, kt, jlo, jhi;
  unit_coords(u, ug, offs, j0, it, kt);
  pair_j_range(ug, it, kt, jlo, jhi);
  const int64_t jn = jhi - j0 < kJRun ? jhi - j0 : kJRun;  // middle vectors of this run
  const int64_t j = j0 + (wave < jn ? wave : jn - 1);      // inactive waves repeat the last
  const bool active = wave < jn;
  const int64_t i0 = it * kRunTile, k0 = kt * kRunTile;

  // Copies: wave w copies row block w (0-1 rows i, 2-3 rows k) from a
  // wave-uniform base (the block's first row, clamped) plus a 32-bit lane
  // offset (r - rf < 16 rows of at most 2^28 bytes).
  gbytes base;
  uint32_t off;
  {
    const int64_t r0 = wave < 2 ? i0 + 16 * wave : k0 + 16 * (wave - 2);
    const int64_t rf = r0 < n ? r0 : n - 1, r = r0 + rl < n ? r0 + rl : n - 1;
    const uint64_t bp = (uint64_t)(a.v + rf * a.ld);
    base = (gbytes)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bp >> 32)) << 32) |
                    (uint32_t)__builtin_amdgcn_readfirstlane((int)bp));
    off = (uint32_t)((r - rf) * a.ld + 16 * g);
  }
  auto issue = [&](int64_t st, int buf) {
    tile2::stage_row((const uint8_t*)(base + st * 64 + off), &raw[buf][wave][0]);
  };
  // the planes of one row block's 16 bytes: per half, rho(1) and P
  auto planes_of = [](const u4& x, int h, u4& R, u4& P) {
    unsigned r0[2], p0[2], r1[2], p1[2];
    tile2::planes32_f4(word_of(x, 2 * h), word_of(x, 2 * h + 1), r0, p0, r1, p1);
    R = u4{r0[0], r0[1], r1[0], r1[1]};
    P = u4{p0[0], p0[1], p1[0], p1[1]};
  };
  // this wave's share: row block `wave` (0-1 rows i, 2-3 rows k), both halves
  auto build_from = [&](const u4& x, int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u4 R, P;
      planes_of(x, h, R, P);
      planes[buf][wave][h][0][lane] = R;
      planes[buf][wave][h][1][lane] = P;
    }
  };
  auto build = [&](int buf) { build_from(raw[buf][wave][lane], buf); };

  v4f acc[2][2][8];
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) acc[m][c][e] = v4f{0, 0, 0, 0};
  auto as_v8 = [](const u4& x) { return v8i{(int)x.x, (int)x.y, (int)x.z, (int)x.w, 0, 0, 0, 0}; };
  // the MFMAs of one half super-step: planes of rows i (AR, AP) and k (KR,
  // KP), j's masks
  auto multiply_c = [&](const u4 (&AR)[2], const u4 (&AP)[2], const u4& KRc, const u4& KPc,
                        const u4& y, const u4& sg, const u4& pm, auto cc) {
    constexpr int c = decltype(cc)::value;
    {
      v8i B[4];  // y z = D R, D P, P R, P P
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const unsigned R = word_of(KRc, q), P = word_of(KPc, q);
        const unsigned yq = word_of(y, q), sq = word_of(sg, q), pq = word_of(pm, q);
        B[0][q] = (int)mod_d(R, yq, sq);
        B[1][q] = (int)mod_d(P, yq, sq);
        B[2][q] = (int)(R & pq);
        B[3][q] = (int)(P & pq);
      }
#pragma unroll
      for (int yz = 0; yz < 4; ++yz)
#pragma unroll
        for (int q = 4; q < 8; ++q) B[yz][q] = 0;
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const v8i ar = as_v8(AR[m]), ap = as_v8(AP[m]);
#pragma unroll
        for (int yz = 0; yz < 4; ++yz) {
          acc[m][c][yz] = tile2::mfma_f4(ar, B[yz], acc[m][c][yz]);
          acc[m][c][4 + yz] = tile2::mfma_f4(ap, B[yz], acc[m][c][4 + yz]);
        }
      }
    }
  };
  auto multiply = [&](const u4 (&AR)[2], const u4 (&AP)[2], const u4 (&KR)[2], const u4 (&KP)[2],
                      const u4& y, const u4& sg, const u4& pm) {
    multiply_c(AR, AP, KR[0], KP[0], y, sg, pm, std::integral_constant<int, 0>{});
    multiply_c(AR, AP, KR[1], KP[1], y, sg, pm, std::integral_constant<int, 1>{});
  };
  // j's masks of two packed words (even and odd fields of 16 each)
  auto masks_of = [](unsigned w0, unsigned w1, u4& y, u4& sg, u4& pm) {
    unsigned yy[4], ss[4], pp[4];
    j_masks32_f4(w0, w1, yy, ss, pp);
    y = u4{yy[0], yy[1], yy[2], yy[3]};
    sg = u4{ss[0], ss[1], ss[2], ss[3]};
    pm = u4{pp[0], pp[1], pp[2], pp[3]};
  };

  const int64_t nfull = a.n_f / 256;
  // this lane's two words of j's batch of eight steps from st0 (zero past
  // the whole steps); the wave's row j from a uniform base
  const uint64_t jp = (uint64_t)(a.v + j * a.ld);
  const gbytes jrow = (gbytes)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(jp >> 32))
                                << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)jp));
  const uint32_t joff = (uint32_t)(64 * (rl >> 1) + 16 * g + 8 * (rl & 1));
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  auto jwords = [&](int64_t st0) {
    u2 w = u2{0u, 0u};
    if (st0 + (rl >> 1) < nfull)
      w = *reinterpret_cast<const __attribute__((address_space(1))) u2*>(jrow + st0 * 64 + joff);
    return w;
  };
  u2 jw = u2{0u, 0u};
  if (nfull > 0) {
    issue(0, 0);
    if (nfull > 1) issue(1, 1);
    if (active) jw = jwords(0);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    build(0);
  }
  for (int64_t st = 0; st < nfull; ++st) {
    const int buf = (int)(st & 1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // raw(st + 1) of this wave has landed
    __syncthreads();  // every wave's has; planes(st) are written; step st - 1's buffers are free
    if (active && (st & 7) == 0) {  // uniform: the masks of steps st .. st + 7
      u4 y, sg, pm;
      masks_of(jw.x, jw.y, y, sg, pm);
      u4* d = &jm[wave][g][rl][0];
      d[0] = y;
      d[1] = sg;
      d[2] = pm;
      jw = jwords(st + 8);
    }
    const bool more = st + 1 < nfull;  // uniform
    if (more && st + 2 < nfull) issue(st + 2, buf);
    if (!active) {
      if (more) build(buf ^ 1);
    } else {
      // Every LDS read of the step goes out ahead of the MFMAs that need it:
      // the next step's row block and the first half's operands, then the
      // second half's while the first half's first block column is
      // multiplied (the fences keep the compiler to this order).  The next
      // step's planes are built between the two halves; on the last step
      // the build reads and writes buffers that no wave uses any more (no
      // branch, so that the compiler keeps the MFMAs where they are).
      const u4 xn = raw[buf ^ 1][wave][lane];
      u4 AR[2][2], AP[2][2], KR[2][2], KP[2][2], M[2][3];
      auto read_half = [&](int h) {
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          AR[h][m] = planes[buf][m][h][0][lane];
          AP[h][m] = planes[buf][m][h][1][lane];
          KR[h][m] = planes[buf][2 + m][h][0][lane];
          KP[h][m] = planes[buf][2 + m][h][1][lane];
        }
        const u4* ms = &jm[wave][g][2 * (st & 7) + h][0];
#pragma unroll
        for (int x = 0; x < 3; ++x) M[h][x] = ms[x];
      };
      read_half(0);
      __builtin_amdgcn_sched_barrier(0);
      multiply_c(AR[0], AP[0], KR[0][0], KP[0][0], M[0][0], M[0][1], M[0][2],
                 std::integral_constant<int, 0>{});
      __builtin_amdgcn_sched_barrier(0);
      read_half(1);
      __builtin_amdgcn_sched_barrier(0);
      multiply_c(AR[0], AP[0], KR[0][1], KP[0][1], M[0][0], M[0][1], M[0][2],
                 std::integral_constant<int, 1>{});
      build_from(xn, buf ^ 1);
      multiply(AR[1], AP[1], KR[1], KP[1], M[1][0], M[1][1], M[1][2]);
    }
  }
  if (nfull * 256 < a.n_f && active) {  // the padded last step: plain loads, all four blocks
    const int64_t kb = nfull * 64 + 16 * g;
    u4 xr[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t r = (b < 2 ? i0 + 16 * b : k0 + 16 * (b - 2)) + rl;
      xr[b] = load_fields64(a.v + (r < n ? r : n - 1) * a.ld, kb, a.n_f);
    }
    const u4 xt = load_fields64(a.v + j * a.ld, kb, a.n_f);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      u4 AR[2], AP[2], KR[2], KP[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        planes_of(xr[m], h, AR[m], AP[m]);
        planes_of(xr[2 + m], h, KR[m], KP[m]);
      }
      u4 y, sg, pm;
      masks_of(word_of(xt, 2 * h), word_of(xt, 2 * h + 1), y, sg, pm);
      multiply(AR, AP, KR, KP, y, sg, pm);
    }
  }
  __syncthreads();  // every wave is done with `planes`: it now stages the stores
  if (!active) return;

  // Epilogue: entry 4a + 2b + c; lane holds rows i0 + 16m + 4g + e of column
  // k0 + 16c + rl.  Every factor is read before the first store (a wait for
  // a load also waits for every store issued before it): the rows' into this
  // wave's 512 bytes past the store staging in `planes`, the others' into
  // registers.
  u4* outs = &planes[0][0][0][0][0] + 384 * wave;
  typedef double d2 __attribute__((ext_vector_type(2)));
  d2* wrow = reinterpret_cast<d2*>(&planes[0][0][0][0][0] + 1536) + 32 * wave;
  if (lane < 32) {
    double w[2];
    triple_factors(a, i0 + lane, w);
    wrow[lane] = d2{w[0], w[1]};
  }
  double wj[2], wk[2][2];
  triple_factors(a, j, wj);
#pragma unroll
  for (int c = 0; c < 2; ++c) triple_factors(a, k0 + 16 * c + rl, wk[c]);
  tile2::static_for<2>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = i0 + 16 * m + 4 * g + e;
      const d2 wv = wrow[16 * m + 4 * g + e];
      const double wi[2] = {wv.x, wv.y};
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int64_t k = k0 + 16 * c + rl;
        int S[8], t[8];
#pragma unroll
        for (int x = 0; x < 8; ++x) S[x] = tile2::f4_count(acc[m][c][x][e]);
        table3_f4(S, t);
        emit_triple_staged(a, k > j && k < n && i < j, i, j, k, t, wi, wj, wk[c], outs);
      }
    }
  });
}

// *flag = 1 if every row of [r0, n) has all n_f fields present (one
// workgroup; its threads read the counts with a stride).
__global__ __launch_bounds__(1024) void complete3_flag_kernel(const int32_t* __restrict__ counts,
                                                              int64_t r0, int64_t n, int64_t n_f,
                                                              int* __restrict__ flag) {
  bool ok = n_f > 0;
  for (int64_t r = r0 + threadIdx.x; r < n && ok; r += blockDim.x)
    ok = reinterpret_cast<const v4i*>(counts)[r].z == n_f;
  ok = __syncthreads_and(ok ? 1 : 0) != 0;
  if (threadIdx.x == 0) *flag = ok ? 1 : 0;
}

// The int8 form over one-j units: 2 x 2 waves over a 64 x 64 (i, k) tile
// for one middle vector j; a unit whose rows are all complete computes its
// tile together in the one-plane form (complete_unit).
__global__ __launch_bounds__(256, 2) void mfma3_kernel(Triple3Args a, UnitGrid ug,
                                                       const int64_t* __restrict__ offs,
                                                       int64_t unit_base, int64_t count) {
  __shared__ v4i part[4][16][64];  // 64 KB: the complete-data partial tiles
  const int wave = threadIdx.x >> 6;
  const int64_t n = a.n;
  const int64_t u = unit_base + xcd_unit(blockIdx.x, count);
  int64_t j, it, kt;
  unit_coords(u, ug, offs, j, it, kt);

  // Complete-data vote over the unit's 64 i rows, 64 k rows and v_j
  // (workgroup-uniform; rows past n repeat row n-1).
  if (a.gram && a.n_f > 0) {
    const int t = threadIdx.x;
    int64_t r = t < 64 ? it * BI + t : (t < 128 ? kt * BK + (t - 64) : j);
    r = r < n ? r : n - 1;
    const bool ok = reinterpret_cast<const v4i*>(a.counts)[r].z == a.n_f;
    if (__syncthreads_and(ok ? 1 : 0)) {
      complete_unit(a, j, it * BI, kt * BK, part);
      return;
    }
  }

  const int64_t row0 = it * BI + (wave & 1) * 16 * WI;  // i range of this wave
  const int64_t col0 = kt * BK + (wave >> 1) * 16 * WK; // k range of this wave
  const bool active = !(row0 >= j || col0 + 16 * WK - 1 <= j || col0 >= n);
  if (!active) return;
  general_wave(a, j, row0, col0, active);
}

// G[r][c] = sum_q rho_{g0+r,q}(1) rho_{g0+c,q}(1) for r, c < ng: the pair
// sums of the complete-data formula.  Waves of 64 x 32 entries, workgroups
// of 128 x 64.
__global__ __launch_bounds__(256, 2) void gram1_kernel(const uint8_t* __restrict__ v, int64_t ld,
                                                       int64_t g0, int64_t ng, int64_t n_f,
                                                       int32_t* __restrict__ gram) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, rl = lane & 15;
  const int64_t row0 = (int64_t)blockIdx.y * 128 + (wave & 1) * 64;
  const int64_t col0 = (int64_t)blockIdx.x * 64 + (wave >> 1) * 32;
  if (row0 >= ng || col0 >= ng) return;
  const uint8_t* pa[4];
  const uint8_t* pb[2];
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    int64_t r = row0 + 16 * m + rl;
    pa[m] = v + (g0 + (r < ng ? r : ng - 1)) * ld + 16 * g;
  }
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    int64_t r = col0 + 16 * c + rl;
    pb[c] = v + (g0 + (r < ng ? r : ng - 1)) * ld + 16 * g;
  }
  v4i acc[4][2];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[m][c] = v4i{0, 0, 0, 0};
  tile2::wave_loop<4, 2>(pa, pb, g, n_f, [&](const u4 (&ca)[4], const u4 (&cb)[2]) {
    tile2::mma_superstep_rho1<4, 2>(ca, cb, acc);
  });
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t r = row0 + 16 * m + 4 * g + e, col = col0 + 16 * c + rl;
        if (r < ng && col < ng) gram[r * ng + col] = acc[m][c][e];
      }
}

}  // namespace

hipError_t launch_mfma3(const Triple3Args& a, hipStream_t stream) {
  if (a.gram && a.ng > 0) {
    const dim3 grid((unsigned)((a.ng + 63) / 64), (unsigned)((a.ng + 127) / 128));
    hipLaunchKernelGGL(gram1_kernel, grid, dim3(256), 0, stream, a.v, a.ld, a.g0, a.ng, a.n_f,
                       a.gram);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  timing_begin("mfma3", stream);
  hipError_t e = hipSuccess;
  if (a.complete) {
    // the flag, then both kernels: each exits at once unless the flag picks it
    hipLaunchKernelGGL(complete3_flag_kernel, dim3(1), dim3(1024), 0, stream, a.counts, a.g0,
                       a.n, a.n_f, a.complete);
    if ((e = hipGetLastError()) == hipSuccess)
      e = launch_units(mfma3_complete_kernel, a, BI, nullptr, stream, kJRun, a.offs_run);
  }
  if (e == hipSuccess)
    e = a.f4 ? launch_units(mfma3_run_kernel, a, kRunTile, nullptr, stream, kJRun, a.offs_gen)
             : launch_units(mfma3_kernel, a, BI, nullptr, stream);
  timing_end(stream);
  return e;
}

}  // namespace ccc
