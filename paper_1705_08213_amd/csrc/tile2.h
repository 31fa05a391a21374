// tile2.h -- device bodies of the 2-way tally tiles, shared by the one-shot
// kernels (mfma2.hip, pop2.hip) and the persistent batched kernel (many.hip).
//
#pragma once

#include <type_traits>
#include <utility>

#include "common.h"
#include "kernels.h"

namespace ccc {
namespace tile2 {

// f(integral_constant<int, I>) for I = 0 .. N - 1, unrolled in the source:
// loops whose bodies index register arrays stay in registers whatever the
// compiler's unrolling limits (a loop it leaves rolled turns such an array
// into scratch memory).
template <typename F, int... I>
__device__ __forceinline__ void static_for_seq(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// Output of one pair (i, j) with table t (Eqs. (2)-(3)) and the factors wi,
// wj of its two vectors (read on valid lanes only).  Dense mode stores the
// table and/or CCC at entry p(i,j) - p_base (adding the old table first when
// accumulating); selection mode keeps the pair only if one of its CCC values
// reaches the threshold.  In selection mode every lane of the wave must call
// it (the slot is taken with one atomic per wave); `valid` says whether this
// lane holds a pair to emit.
__device__ __forceinline__ void emit_pair(const Pair2Args& a, bool valid, int64_t i, int64_t j,
                                          v4i t, const double (&wi)[2], const double (&wj)[2]) {
  valid = valid && i >= a.row_begin && i < a.row_end;
  if (a.sel.count) {
    double r[4] = {0.0, 0.0, 0.0, 0.0};
    bool keep = false;
    int64_t p = 0;
    if (valid) {
      p = a.tri ? pair_index(a.n_a, i, j) : i * a.n_b + j;
      pair_ccc(t, wi, wj, r);
      keep = r[0] >= a.sel.threshold || r[1] >= a.sel.threshold ||
             r[2] >= a.sel.threshold || r[3] >= a.sel.threshold;
    }
    const int64_t slot = select_slot(keep, a.sel.count);
    if (slot >= 0 && slot < a.sel.cap) {
      a.sel.index[slot] = p;
      double2* c = reinterpret_cast<double2*>(a.sel.ccc + 4 * slot);
      c[0] = double2{r[0], r[1]};
      c[1] = double2{r[2], r[3]};
      if (a.sel.tables) *reinterpret_cast<v4i*>(a.sel.tables + 4 * slot) = t;
    }
    return;
  }
  if (!valid) return;
  const int64_t p = a.tri ? pair_index(a.n_a, i, j) : i * a.n_b + j;
  if (a.accumulate) t = t + *reinterpret_cast<const v4i*>(a.tables + 4 * p);
  store_pair(p - a.p_base, t, wi, wj, a.tables, a.ccc);
}

// emit_pair with the CCC rows written through LDS, so that each store
// instruction covers 256 contiguous bytes.  Every lane of the wave must call
// it; lane (g, rl) holds pair (i, j) with j = j_base + rl for one i per
// 16-lane group g (consecutive entries when valid).  The group's 16 CCC rows
// (32 B each) go into `scratch` (wave-private, 128 x 16 B) in output order,
// then lane rl stores 16-byte piece rl of each 256-byte stretch.  Tables are
// stored directly (16 lanes x 16 B are already contiguous).  Selection and
// accumulating calls fall back to emit_pair.
__device__ __forceinline__ void emit_pair_staged(const Pair2Args& a, bool valid, int64_t i,
                                                 int64_t j, v4i t, const double (&wi)[2],
                                                 const double (&wj)[2], u4* scratch) {
  if (a.sel.count || a.accumulate) {
    emit_pair(a, valid, i, j, t, wi, wj);
    return;
  }
  valid = valid && i >= a.row_begin && i < a.row_end;
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const int64_t p = valid ? (a.tri ? pair_index(a.n_a, i, j) : i * a.n_b + j) - a.p_base : 0;
  // streaming stores: the dense output is written once and not read back here
  if (valid && a.tables)
    __builtin_nontemporal_store(t, reinterpret_cast<v4i*>(a.tables + 4 * p));
  if (!a.ccc) return;
  const unsigned gm = (unsigned)(__ballot(valid ? 1 : 0) >> (16 * g)) & 0xFFFFu;
  const int first = gm ? __ffs(gm) - 1 : 0;
  const int64_t p0 = __shfl(p - rl, 16 * g + first);  // entry of the group's lane 0
  double r[4] = {0.0, 0.0, 0.0, 0.0};
  if (valid) pair_ccc(t, wi, wj, r);
  u4* C = scratch + 32 * g;
  double2* Cd = reinterpret_cast<double2*>(C + 2 * rl);
  Cd[0] = double2{r[0], r[1]};
  Cd[1] = double2{r[2], r[3]};
  // the wave's LDS accesses run in program order; keep the compiler to it
  asm volatile("" ::: "memory");
  typedef unsigned v4u __attribute__((ext_vector_type(4)));
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int piece = 16 * q + rl;
    const u4 d = C[piece];
    if ((gm >> (piece >> 1)) & 1u)
      __builtin_nontemporal_store(v4u{d.x, d.y, d.z, d.w},
                                  reinterpret_cast<v4u*>(a.ccc + 4 * p0) + piece);
  }
  asm volatile("" ::: "memory");  // the scratch is reused by the next call
}

// Factors of row x of A (side 0) or B (side 1), clamped into range; only
// computed when some CCC value is produced.
__device__ __forceinline__ void side_factors(const Pair2Args& a, int side, int64_t x,
                                             double (&w)[2]) {
  if (a.ccc || a.sel.count) {
    const int64_t n = side ? a.n_b : a.n_a;
    vector_factors(side ? a.counts_b : a.counts_a, x < n ? x : n - 1, a.gamma, w);
  } else {
    w[0] = w[1] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// int8-MFMA path
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
// ---------------------------------------------------------------------------

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

// rho(1) of 16 fields (one packed word), as for unpack16.
__device__ __forceinline__ v4i unpack16_rho1(unsigned w) {
  unsigned c0 = w & kLow2, c1 = (w >> 2) & kLow2, c2 = (w >> 4) & kLow2, c3 = (w >> 6) & kLow2;
  return v4i{(int)__builtin_amdgcn_perm(0u, kRho1Table, c0),
             (int)__builtin_amdgcn_perm(0u, kRho1Table, c1),
             (int)__builtin_amdgcn_perm(0u, kRho1Table, c2),
             (int)__builtin_amdgcn_perm(0u, kRho1Table, c3)};
}

// Complete-data super-step: only C11 = sum rho_i(1) rho_j(1) (one plane).
template <int WM, int WN>
__device__ __forceinline__ void mma_superstep_rho1(const u4 (&pa)[WM], const u4 (&pb)[WN],
                                                   v4i (&acc)[WM][WN]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    v4i a1[WM], b1[WN];
#pragma unroll
    for (int m = 0; m < WM; ++m) a1[m] = unpack16_rho1(word_of(pa[m], s));
#pragma unroll
    for (int n = 0; n < WN; ++n) b1[n] = unpack16_rho1(word_of(pb[n], s));
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int n = 0; n < WN; ++n)
        acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1[m], b1[n], acc[m][n], 0, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// fp4 operands (e2m1, the 16x16x128 scaled MFMA at twice the int8 rate)
//
// A 2-bit value x in the low two bits of a nibble is the e2m1 number x / 2
// (0001 is the subnormal 1/2, 0010 is 1).  The planes used are rho(1) and
// the presence P (code != 10); from the code's bits lo, hi:
//   rho(1) = lo + (lo & hi)  (00 -> 0, 01 -> 1, 11 -> 2, 10 -> 0),
//   P      = lo | !hi,
// five operations per 16 fields, computed on the packed word, whose 2-bit
// fields then go to nibbles (even fields, then odd ones: A and B share the
// order).  Products are multiples of 1/4 and a sum over n_f fields is at most
// n_f, so fp32 accumulation is exact while n_f <= 2^22 (kF4MaxFields); the
// four sums S = sum rho_i rho_j, T = sum rho_i P_j, U = sum P_i rho_j,
// V = sum P_i P_j give the table:
//   C11 = S,  C10 = 2T - S,  C01 = 2U - S,  C00 = 4V - 2T - 2U + S
// (rho(0) = 2P - rho(1)); the general 2-way loop reaches them through the
// cheaper plane U = rho(1) + 2 [missing] (planes32_f4u).  Fields past n_f
// carry the missing code, which is zero in rho(1) and P.
// ---------------------------------------------------------------------------

constexpr unsigned kEven2 = 0x55555555u;  // bit 0 of every 2-bit field
constexpr unsigned kNib2 = 0x33333333u;   // low two bits of every nibble

// Shifts of a pair of words as one 64-bit shift (v_lshrrev_b64 /
// v_lshlrev_b64, as inline asm: the compiler would split them).  Callers
// use them only where the bits crossing between the words are zero or
// masked off afterwards.
template <int N>
__device__ __forceinline__ void shr_pair(unsigned a0, unsigned a1, unsigned& r0, unsigned& r1) {
  const unsigned long long x = ((unsigned long long)a1 << 32) | a0;
  unsigned long long y;
  asm("v_lshrrev_b64 %0, %1, %2" : "=v"(y) : "n"(N), "v"(x));
  r0 = (unsigned)y;
  r1 = (unsigned)(y >> 32);
}
template <int N>
__device__ __forceinline__ void shl_pair(unsigned a0, unsigned a1, unsigned& r0, unsigned& r1) {
  const unsigned long long x = ((unsigned long long)a1 << 32) | a0;
  unsigned long long y;
  asm("v_lshlrev_b64 %0, %1, %2" : "=v"(y) : "n"(N), "v"(x));
  r0 = (unsigned)y;
  r1 = (unsigned)(y >> 32);
}

// The rho(1) and P planes of two words w0, w1 as fp4 operand halves: r0 =
// (rho(1) of w0's even fields, of its odd fields), p0 likewise, r1 and p1
// for w1 (see nibbles32).  v_bitop3 truth tables 0x80 = a & b & c and
// 0xA2 = c & (a | ~b) (with a = w, b = w >> 1: bit 0 of a field is lo, of b
// is hi).  Seventeen operations, the shifts paired (twenty one word at a
// time).  Crossing bits: s takes
// w1's bit 0 into bit 31, which every mask drops; the >> 2 of r and of the
// odd P bits takes w1's bits 0-1 into bits 30-31, dropped by kNib2 for r and
// zero for P (its bits sit at 2 mod 4).
__device__ __forceinline__ void planes32_f4(unsigned w0, unsigned w1, unsigned (&r0)[2],
                                            unsigned (&p0)[2], unsigned (&r1)[2],
                                            unsigned (&p1)[2]) {
  unsigned s0, s1;
  shr_pair<1>(w0, w1, s0, s1);
  const unsigned a0 = (w0 & kEven2) + __builtin_amdgcn_bitop3_b32(w0, s0, kEven2, 0x80);
  const unsigned a1 = (w1 & kEven2) + __builtin_amdgcn_bitop3_b32(w1, s1, kEven2, 0x80);
  unsigned b0, b1;
  shr_pair<2>(a0, a1, b0, b1);
  r0[0] = a0 & kNib2;
  r0[1] = b0 & kNib2;
  r1[0] = a1 & kNib2;
  r1[1] = b1 & kNib2;
  p0[0] = __builtin_amdgcn_bitop3_b32(w0, s0, 0x11111111u, 0xA2);
  p1[0] = __builtin_amdgcn_bitop3_b32(w1, s1, 0x11111111u, 0xA2);
  shr_pair<2>(__builtin_amdgcn_bitop3_b32(w0, s0, 0x44444444u, 0xA2),
              __builtin_amdgcn_bitop3_b32(w1, s1, 0x44444444u, 0xA2), p0[1], p1[1]);
}

// Elements q, q + 1 of a register array as a two-element array.
__device__ __forceinline__ unsigned (&pair_of(unsigned (&x)[4], int q))[2] {
  return *reinterpret_cast<unsigned(*)[2]>(&x[q]);
}

// The 2-way planes U = rho(1) + 2 [missing] (codes 00, 01, 10, 11 -> 0, 1,
// 2, 2) and P of 16 fields (one word w) as fp4 nibbles, in seven operations: even fields
// in the low two bits of a nibble (e2m1 value = plane / 2), odd fields in
// its middle two bits (value = plane; U = 2 is the pattern 0100, never 0110).
// With s = w >> 1, h = s & kEven2 (hi at bit 0 of each field, 0 at bit 1)
// and q = h >> 1, truth tables 0x20 = c & a & ~b and 0xA2 = c & (a | ~b):
//   ue: bit 0 = lo & ~hi, bit 1 = hi         uo: the same at bits 1, 2
//   pe: bit 0 = lo | ~hi                     po: the same at bit 1
// Two words at once: the shifts s and q are taken on the 64-bit pair
// (shr_pair: the bit that crosses from the upper word lands in bit 31 of the
// lower one, which no mask keeps), six operations per word.
__device__ __forceinline__ void planes32_f4u(unsigned w0, unsigned w1, unsigned (&ue)[2],
                                             unsigned (&uo)[2], unsigned (&pe)[2],
                                             unsigned (&po)[2]) {
  unsigned s0, s1, q0, q1;
  shr_pair<1>(w0, w1, s0, s1);
  const unsigned h0 = s0 & kEven2, h1 = s1 & kEven2;
  shr_pair<1>(h0, h1, q0, q1);
  ue[0] = __builtin_amdgcn_bitop3_b32(w0, h0, 0x33333333u, 0x20);
  ue[1] = __builtin_amdgcn_bitop3_b32(w1, h1, 0x33333333u, 0x20);
  uo[0] = __builtin_amdgcn_bitop3_b32(s0, q0, 0x66666666u, 0x20);
  uo[1] = __builtin_amdgcn_bitop3_b32(s1, q1, 0x66666666u, 0x20);
  pe[0] = __builtin_amdgcn_bitop3_b32(w0, s0, 0x11111111u, 0xA2);
  pe[1] = __builtin_amdgcn_bitop3_b32(w1, s1, 0x11111111u, 0xA2);
  po[0] = __builtin_amdgcn_bitop3_b32(s0, q0, 0x22222222u, 0xA2);
  po[1] = __builtin_amdgcn_bitop3_b32(s1, q1, 0x22222222u, 0xA2);
}

// fp4 MFMA with both E8M0 scales 2^(e - 127).
template <int e>
__device__ __forceinline__ v4f mfma_f4s(const v8i& a, const v8i& b, v4f c) {
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 4, 4, 0, e, 0, e);
}

// rho(1) of 16 fields; `complete` words hold no missing code, where
// rho(1) = code - hi.
template <bool complete>
__device__ __forceinline__ unsigned rho1_16_f4(unsigned w) {
  if (complete) return w - ((w >> 1) & kEven2);
  const unsigned lo = w & kEven2;
  return lo + (lo & (w >> 1));
}

// Two words of 2-bit values -> one fp4 operand of 32 nibbles (4 registers).
__device__ __forceinline__ v8i nibbles32(unsigned x0, unsigned x1) {
  return v8i{(int)(x0 & kNib2), (int)((x0 >> 2) & kNib2), (int)(x1 & kNib2),
             (int)((x1 >> 2) & kNib2), 0, 0, 0, 0};
}

// nibbles32(rho1_16_f4<true>(w0), rho1_16_f4<true>(w1)) for words of
// complete data (codes 00, 01, 11), in nine operations instead of twelve:
// per field (hi, lo) -> (hi, lo & ~hi), one v_bitop3 (0x20 = c & a & ~b) of
// the word and its hi bits moved to the field's bit 0 (h); the odd fields
// are shifted down by two first, word and hi bits alike.  The pair shifts
// carry w1's low bits into bits 30-31 (31 for s) of the w0 results, which
// kEven2 and kNib2 drop.
__device__ __forceinline__ v8i rho1_nibbles_complete(unsigned w0, unsigned w1) {
  unsigned s0, s1, t0, t1, q0, q1;
  shr_pair<1>(w0, w1, s0, s1);
  const unsigned h0 = s0 & kEven2, h1 = s1 & kEven2;
  shr_pair<2>(w0, w1, t0, t1);
  shr_pair<2>(h0, h1, q0, q1);
  return v8i{(int)__builtin_amdgcn_bitop3_b32(w0, h0, kNib2, 0x20),
             (int)__builtin_amdgcn_bitop3_b32(t0, q0, kNib2, 0x20),
             (int)__builtin_amdgcn_bitop3_b32(w1, h1, kNib2, 0x20),
             (int)__builtin_amdgcn_bitop3_b32(t1, q1, kNib2, 0x20),
             0, 0, 0, 0};
}

__device__ __forceinline__ v8i operand_f4(const unsigned (&x0)[2], const unsigned (&x1)[2]) {
  return v8i{(int)x0[0], (int)x0[1], (int)x1[0], (int)x1[1], 0, 0, 0, 0};
}

__device__ __forceinline__ v4f mfma_f4(const v8i& a, const v8i& b, v4f c) {
  // formats 4 = e2m1 for A and B; E8M0 scales 127 = 2^0
  return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 4, 4, 0, 127, 0, 127);
}

__device__ __forceinline__ int f4_count(float x) { return (int)(4.0f * x); }

// Table (entry 2a+b) from the four sums of the U and P planes
// (planes32_f4u) over the K fields of the loop: rho(1) = U + 2P - 2 gives
//   S = UU + 2UP + 2PU + 4PP - 2 n_i(1) - 2 n_j(1) - 4K,
//   T = UP + 2PP - 2 m_j,  U' = PU + 2PP - 2 m_i,  V = PP
// (sum_q U_i = n_i(1) + 2 (K - m_i), sum_q P_i = m_i).
__device__ __forceinline__ v4i table_f4u(float uu, float up, float pu, float pp, const v4i& ci,
                                         const v4i& cj, int kpad) {
  const int UU = f4_count(uu), UP = f4_count(up), PU = f4_count(pu), PP = f4_count(pp);
  const int S = UU + 2 * UP + 2 * PU + 4 * PP - 2 * ci.y - 2 * cj.y - 4 * kpad;
  const int T = UP + 2 * PP - 2 * cj.z, U = PU + 2 * PP - 2 * ci.z, V = PP;
  return v4i{4 * V - 2 * T - 2 * U + S, 2 * U - S, 2 * T - S, S};
}

// One 256-field super-step of the four sums of the U and P planes
// (planes32_f4u): the MFMA step of the even fields of the lane's four words,
// then the one of the odd fields, whose nibble values are twice as large
// (scales 2^-1 on A and B).
template <int WM, int WN>
__device__ __forceinline__ void mma_superstep_f4u(const u4 (&xa)[WM], const u4 (&xb)[WN],
                                                  v4f (&acc)[WM][WN][4]) {
  v8i bu[2][WN], bp[2][WN];
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    unsigned ue[4], uo[4], pe[4], po[4];
#pragma unroll
    for (int q = 0; q < 4; q += 2)
      planes32_f4u(word_of(xb[n], q), word_of(xb[n], q + 1), pair_of(ue, q), pair_of(uo, q),
                   pair_of(pe, q), pair_of(po, q));
    bu[0][n] = v8i{(int)ue[0], (int)ue[1], (int)ue[2], (int)ue[3], 0, 0, 0, 0};
    bu[1][n] = v8i{(int)uo[0], (int)uo[1], (int)uo[2], (int)uo[3], 0, 0, 0, 0};
    bp[0][n] = v8i{(int)pe[0], (int)pe[1], (int)pe[2], (int)pe[3], 0, 0, 0, 0};
    bp[1][n] = v8i{(int)po[0], (int)po[1], (int)po[2], (int)po[3], 0, 0, 0, 0};
  }
#pragma unroll
  for (int m = 0; m < WM; ++m) {
    unsigned ue[4], uo[4], pe[4], po[4];
#pragma unroll
    for (int q = 0; q < 4; q += 2)
      planes32_f4u(word_of(xa[m], q), word_of(xa[m], q + 1), pair_of(ue, q), pair_of(uo, q),
                   pair_of(pe, q), pair_of(po, q));
    const v8i au0{(int)ue[0], (int)ue[1], (int)ue[2], (int)ue[3], 0, 0, 0, 0};
    const v8i ap0{(int)pe[0], (int)pe[1], (int)pe[2], (int)pe[3], 0, 0, 0, 0};
    const v8i au1{(int)uo[0], (int)uo[1], (int)uo[2], (int)uo[3], 0, 0, 0, 0};
    const v8i ap1{(int)po[0], (int)po[1], (int)po[2], (int)po[3], 0, 0, 0, 0};
#pragma unroll
    for (int n = 0; n < WN; ++n) {
      acc[m][n][0] = mfma_f4s<127>(au0, bu[0][n], acc[m][n][0]);
      acc[m][n][1] = mfma_f4s<127>(au0, bp[0][n], acc[m][n][1]);
      acc[m][n][2] = mfma_f4s<127>(ap0, bu[0][n], acc[m][n][2]);
      acc[m][n][3] = mfma_f4s<127>(ap0, bp[0][n], acc[m][n][3]);
    }
#pragma unroll
    for (int n = 0; n < WN; ++n) {
      acc[m][n][0] = mfma_f4s<126>(au1, bu[1][n], acc[m][n][0]);
      acc[m][n][1] = mfma_f4s<126>(au1, bp[1][n], acc[m][n][1]);
      acc[m][n][2] = mfma_f4s<126>(ap1, bu[1][n], acc[m][n][2]);
      acc[m][n][3] = mfma_f4s<126>(ap1, bp[1][n], acc[m][n][3]);
    }
  }
}

// 16 bytes per lane of one row copied straight into LDS (lane l's bytes at
// dst + 16 l), asynchronously: the wave's vector-memory counter covers it.
__device__ __forceinline__ void stage_row(const uint8_t* src, u4* dst) {
  __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
}

// The fp4 super-step loop of a workgroup of four waves: 2 x 2 wave tiles of
// (16 WM) x (16 WN) pairs, the workgroup tile at (I0, J0).  The waves share
// rows, so each step's 2 WM + 2 WN row blocks (16 rows x 64 bytes, one
// `global_load_lds_dwordx4` each: lane l's 16 bytes land at 16 l) travel
// into the workgroup's LDS stage once, split over the waves, while the
// previous step is unpacked and multiplied.  One barrier per step says that
// every block of the step has landed and that the buffer read one step
// earlier is free.  Every wave of the workgroup must call it; inactive
// waves only copy their blocks.  Then the masked tail step of the active
// waves from plain loads (pa, pb: this wave's rows, with the lane's 16g
// byte offset), taken by `tail` (whose fields past n_f read as missing).
template <int WM, int WN, typename Step, typename Tail>
__device__ __forceinline__ void wg_loop_f4(const Pair2Args& a, int64_t I0, int64_t J0,
                                           bool active, const uint8_t* const (&pa)[WM],
                                           const uint8_t* const (&pb)[WN],
                                           u4 (*stage)[2 * WM + 2 * WN][64], Step step,
                                           Tail tail) {
  constexpr int NB = 2 * WM + 2 * WN, BPW = (NB + 3) / 4;  // blocks, blocks per wave
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int g = lane >> 4, rl = lane & 15;
  // each copy: a wave-uniform base (the block's first row, clamped; its two
  // halves read from lane 0 so the compiler knows it is uniform) plus a
  // fixed 32-bit lane offset.  The LDS destinations become scalar (m0 set
  // without v_readfirstlane).
  const uint8_t* base[BPW];
  uint32_t off[BPW];
#pragma unroll
  for (int t = 0; t < BPW; ++t) {
    const int b = BPW * wave + t;  // blocks 0 .. 2 WM - 1 are rows i, then rows j
    const bool rows_i = b < 2 * WM;
    const int64_t n = rows_i ? a.n_a : a.n_b, ld = rows_i ? a.lda : a.ldb;
    const int64_t r0 = rows_i ? I0 + 16 * b : J0 + 16 * (b - 2 * WM);
    const int64_t rf = r0 < n ? r0 : n - 1, r = r0 + rl < n ? r0 + rl : n - 1;
    const uint64_t bp = (uint64_t)((rows_i ? a.va : a.vb) + rf * ld);  // uniform
    base[t] = (const uint8_t*)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bp >> 32))
                                << 32) |
                               (uint32_t)__builtin_amdgcn_readfirstlane((int)bp));
    off[t] = (uint32_t)((r - rf) * ld + 16 * g);
  }
  auto issue = [&](int64_t s, int buf) {
#pragma unroll
    for (int t = 0; t < BPW; ++t)
      if (BPW * wave + t < NB) stage_row(base[t] + s * 64 + off[t], &stage[buf][BPW * wave + t][0]);
  };
  const int ma = (wave & 1) * WM, nb = 2 * WM + (wave >> 1) * WN;
  const int64_t nfull = a.n_f / 256, nbytes = (a.n_f + 3) / 4;
  if (nfull > 0) issue(0, 0);
  for (int64_t s = 0; s < nfull; ++s) {
    const int buf = (int)(s & 1);
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's blocks have landed
    __syncthreads();                                   // every wave's have; buf ^ 1 is free
    // read before the next copy is issued (the compiler would otherwise wait
    // for that copy before the reads)
    u4 xa[WM], xb[WN];
    if (active) {
#pragma unroll
      for (int n = 0; n < WN; ++n) xb[n] = stage[buf][nb + n][lane];
#pragma unroll
      for (int m = 0; m < WM; ++m) xa[m] = stage[buf][ma + m][lane];
    }
    if (s + 1 < nfull) issue(s + 1, buf ^ 1);
    if (active) step(xa, xb);
  }
  const int64_t kt = nfull * 64;
  if (active && kt < nbytes) {
    u4 xa[WM], xb[WN];
#pragma unroll
    for (int m = 0; m < WM; ++m) xa[m] = load_fields64(pa[m] - 16 * g, kt + 16 * g, a.n_f);
#pragma unroll
    for (int n = 0; n < WN; ++n) xb[n] = load_fields64(pb[n] - 16 * g, kt + 16 * g, a.n_f);
    tail(xa, xb);
  }
}

// Complete-data super-step of S alone.
template <int WM, int WN, bool complete>
__device__ __forceinline__ void mma_superstep_rho1_f4(const u4 (&pa)[WM], const u4 (&pb)[WN],
                                                      v4f (&acc)[WM][WN]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    v8i a1[WM], b1[WN];
#pragma unroll
    for (int m = 0; m < WM; ++m)
      a1[m] = nibbles32(rho1_16_f4<complete>(word_of(pa[m], 2 * h)),
                        rho1_16_f4<complete>(word_of(pa[m], 2 * h + 1)));
#pragma unroll
    for (int n = 0; n < WN; ++n)
      b1[n] = nibbles32(rho1_16_f4<complete>(word_of(pb[n], 2 * h)),
                        rho1_16_f4<complete>(word_of(pb[n], 2 * h + 1)));
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int n = 0; n < WN; ++n) acc[m][n] = mfma_f4(a1[m], b1[n], acc[m][n]);
  }
}

// Run the super-step loop of a wave tile: `step` consumes the 16-byte pieces
// of every row (plain loads while all 256 fields are inside n_f, prefetched
// one super-step ahead; then one masked tail step).
template <int WM, int WN, typename Step>
__device__ __forceinline__ void wave_loop(const uint8_t* const (&pa)[WM],
                                          const uint8_t* const (&pb)[WN], int g, int64_t n_f,
                                          Step step) {
  const int64_t nfull = n_f / 256;
  const int64_t nbytes = (n_f + 3) / 4;
  // Two register sets in turn (no copies): set 0 holds even super-steps,
  // set 1 odd ones; each is refilled right after its MFMAs are issued.
  u4 ca[WM], cb[WN], da[WM], db[WN];
  auto load = [&](int64_t s, u4 (&xa)[WM], u4 (&xb)[WN]) {
#pragma unroll
    for (int m = 0; m < WM; ++m) xa[m] = *reinterpret_cast<const u4*>(pa[m] + s * 64);
#pragma unroll
    for (int n = 0; n < WN; ++n) xb[n] = *reinterpret_cast<const u4*>(pb[n] + s * 64);
  };
  if (nfull > 0) load(0, ca, cb);
  int64_t s = 0;
  for (; s + 1 < nfull; s += 2) {
    load(s + 1, da, db);
    step(ca, cb);
    if (s + 2 < nfull) load(s + 2, ca, cb);
    step(da, db);
  }
  if (s < nfull) step(ca, cb);
  const int64_t kt = nfull * 64;
  if (kt < nbytes) {
    // row pointers already include the lane's 16*g byte offset
#pragma unroll
    for (int m = 0; m < WM; ++m) ca[m] = load_fields64(pa[m] - 16 * g, kt + 16 * g, n_f);
#pragma unroll
    for (int n = 0; n < WN; ++n) cb[n] = load_fields64(pb[n] - 16 * g, kt + 16 * g, n_f);
    step(ca, cb);
  }
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

// One wave's (16 WM) x (16 WN) tile of pairs with first row row0 and first
// column col0 (see the design notes above); wave w of the workgroup holds
// the tile at (I0 + (w & 1) 16 WM, J0 + (w >> 1) 16 WN).  Both operand
// formats stage the rows for the workgroup (`stage`: two buffers of
// 2 WM + 2 WN row blocks of 1 KB), so every wave of the workgroup must call
// it; waves whose tile holds no pair to compute only take part in the
// copies.
template <int WM, int WN, bool F4>
__device__ __forceinline__ void mfma2_wave_tile(const Pair2Args& a, int64_t row0, int64_t col0,
                                                u4 (*stage)[2 * WM + 2 * WN][64]) {
  const int lane = threadIdx.x & 63;
  // no pair i < j in this wave tile
  const bool active = row0 < a.n_a && col0 < a.n_b && !(a.tri && row0 >= col0 + 16 * WN - 1);
  const int g = lane >> 4, rl = lane & 15;
  const int wave = threadIdx.x >> 6;
  const int64_t I0 = row0 - (wave & 1) * 16 * WM, J0 = col0 - (wave >> 1) * 16 * WN;
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

  // Complete data (every row of this wave tile has all n_f fields present,
  // as the 1-way counts of this call say): P = 1, so the table follows from
  // C11 = sum rho_i(1) rho_j(1) and the allele counts n(1):
  //   C10 = 2 n_i(1) - C11,  C01 = 2 n_j(1) - C11,
  //   C00 = 4 n_f - 2 n_i(1) - 2 n_j(1) + C11,
  // one MFMA plane instead of four.  The vote is wave-uniform.
  bool mine = active && !a.accumulate && a.n_f > 0;
#pragma unroll
  for (int m = 0; m < WM; ++m) {
    int64_t r = row0 + 16 * m + rl;
    r = r < a.n_a ? r : a.n_a - 1;
    mine = mine && reinterpret_cast<const v4i*>(a.counts_a)[r].z == a.n_f;
  }
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    int64_t r = col0 + 16 * n + rl;
    r = r < a.n_b ? r : a.n_b - 1;
    mine = mine && reinterpret_cast<const v4i*>(a.counts_b)[r].z == a.n_f;
  }
  if (__all(mine ? 1 : 0)) {
    using Acc = std::conditional_t<F4, v4f, v4i>;
    Acc acc1[WM][WN];
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int n = 0; n < WN; ++n) acc1[m][n] = Acc{0, 0, 0, 0};
    auto step1 = [&](const u4 (&ca)[WM], const u4 (&cb)[WN]) {
      if constexpr (F4)
        mma_superstep_rho1_f4<WM, WN, false>(ca, cb, acc1);
      else
        mma_superstep_rho1<WM, WN>(ca, cb, acc1);
    };
    wg_loop_f4<WM, WN>(a, I0, J0, true, pa, pb, stage, step1, step1);
    const int nf4 = (int)(4 * a.n_f);
    double wj[WN][2];
    int n1j[WN];
#pragma unroll
    for (int n = 0; n < WN; ++n) {
      const int64_t j = col0 + 16 * n + rl;
      side_factors(a, 1, j, wj[n]);
      n1j[n] = reinterpret_cast<const v4i*>(a.counts_b)[j < a.n_b ? j : a.n_b - 1].y;
    }
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = row0 + 16 * m + 4 * g + e;
        const int n1i = reinterpret_cast<const v4i*>(a.counts_a)[i < a.n_a ? i : a.n_a - 1].y;
        double wi[2];
        side_factors(a, 0, i, wi);
#pragma unroll
        for (int n = 0; n < WN; ++n) {
          const int64_t j = col0 + 16 * n + rl;
          int c11;
          if constexpr (F4)
            c11 = f4_count(acc1[m][n][e]);
          else
            c11 = acc1[m][n][e];
          const bool valid = i < a.n_a && j < a.n_b && !(a.tri && i >= j);
          emit_pair(a, valid, i, j,
                    v4i{nf4 - 2 * n1i - 2 * n1j[n] + c11, 2 * n1j[n] - c11, 2 * n1i - c11, c11},
                    wi, wj[n]);
        }
      }
    return;
  }

  using Acc = std::conditional_t<F4, v4f, v4i>;
  Acc acc[WM][WN][4];
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int n = 0; n < WN; ++n)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[m][n][e] = Acc{0, 0, 0, 0};
  auto step = [&](const u4 (&xa)[WM], const u4 (&xb)[WN]) {
    if constexpr (F4)
      mma_superstep_f4u<WM, WN>(xa, xb, acc);
    else
      mma_superstep<WM, WN>(xa, xb, acc);
  };
  wg_loop_f4<WM, WN>(a, I0, J0, active, pa, pb, stage, step, step);
  if (!active) return;

  // Epilogue: lane holds rows 4g + e (e = 0..3) of column rl of each 16x16 block.
  // The factors and (fp4) this call's counts of the wave's 16 WM rows and
  // 16 WN columns are read into its own LDS before the first store (a wait
  // for a load also waits for every store issued before it).
  struct SideIn {
    double w[2];
    v4i c;
  };
  static_assert(sizeof(SideIn) == 32, "two 16-byte halves");
  __shared__ SideIn side_in[4][16 * (WM + WN)];
  SideIn* rows = side_in[threadIdx.x >> 6];
  for (int t = lane; t < 16 * (WM + WN); t += 64) {
    const bool is_row = t < 16 * WM;
    const int64_t x = is_row ? row0 + t : col0 + (t - 16 * WM);
    const int64_t nx = is_row ? a.n_a : a.n_b;
    SideIn si;
    side_factors(a, is_row ? 0 : 1, x, si.w);
    si.c = v4i{0, 0, 0, 0};
    if constexpr (F4)
      si.c = reinterpret_cast<const v4i*>(is_row ? a.chunk_a : a.chunk_b)[x < nx ? x : nx - 1];
    rows[t] = si;
  }
  const int kpad = (int)((a.n_f + 255) / 256 * 256);  // fields the fp4 loop covers
#pragma unroll
  for (int m = 0; m < WM; ++m) {
#pragma unroll
    for (int n = 0; n < WN; ++n) {
      const int64_t j = col0 + 16 * n + rl;
      const SideIn sj = rows[16 * WM + 16 * n + rl];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = row0 + 16 * m + 4 * g + e;
        const SideIn si = rows[16 * m + 4 * g + e];
        const bool valid = i < a.n_a && j < a.n_b && !(a.tri && i >= j);
        v4i t;
        if constexpr (F4)
          t = table_f4u(acc[m][n][0][e], acc[m][n][1][e], acc[m][n][2][e], acc[m][n][3][e],
                        si.c, sj.c, kpad);
        else
          t = v4i{acc[m][n][0][e], acc[m][n][1][e], acc[m][n][2][e], acc[m][n][3][e]};
        emit_pair(a, valid, i, j, t, si.w, sj.w);
      }
    }
  }
}

// Wave tile of a call whose every row of A and B has all n_f fields
// present (P = 1 on every field): only C11 = sum rho_i(1) rho_j(1) is
// multiplied, and the table follows from the allele counts n(1):
//   C10 = 2 n_i(1) - C11,  C01 = 2 n_j(1) - C11,
//   C00 = 4 n_f - 2 n_i(1) - 2 n_j(1) + C11.
// One plane needs a quarter of the accumulators of the general form, so a
// wave holds a (16 WM) x (16 WN) tile four times the size, and a workgroup
// of 2 x 2 such waves stages 2 WM + 2 WN row blocks per step for four times
// the pairs: half the bytes per pair that travel from L2, and rho(1) of each
// staged block feeds 2 WN (rows i) or 2 WM (rows j) MFMAs per half step.
// Both operand formats stage through LDS.  Every wave of the workgroup must
// call it; `outs` is this wave's 2 KB of LDS for staging its CCC stores.
template <int WM, int WN, bool F4>
__device__ __forceinline__ void mfma2_complete_wave_tile(const Pair2Args& a, int64_t row0,
                                                         int64_t col0,
                                                         u4 (*stage)[2 * WM + 2 * WN][64],
                                                         u4* outs) {
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const int wave = threadIdx.x >> 6;
  // no pair i < j in this wave tile
  const bool active = row0 < a.n_a && col0 < a.n_b && !(a.tri && row0 >= col0 + 16 * WN - 1);
  const int64_t I0 = row0 - (wave & 1) * 16 * WM, J0 = col0 - (wave >> 1) * 16 * WN;
  const uint8_t* pa[WM];
  const uint8_t* pb[WN];
#pragma unroll
  for (int m = 0; m < WM; ++m) {
    const int64_t r = row0 + 16 * m + rl;
    pa[m] = a.va + (r < a.n_a ? r : a.n_a - 1) * a.lda + 16 * g;
  }
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    const int64_t r = col0 + 16 * n + rl;
    pb[n] = a.vb + (r < a.n_b ? r : a.n_b - 1) * a.ldb + 16 * g;
  }
  using Acc = std::conditional_t<F4, v4f, v4i>;
  Acc acc[WM][WN];
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int n = 0; n < WN; ++n) acc[m][n] = Acc{0, 0, 0, 0};
  // `complete`: every field of the step is inside n_f (no padding code)
  auto body = [&](const u4 (&xa)[WM], const u4 (&xb)[WN], auto complete) {
    if constexpr (F4) {
      auto rho1_pair = [&](unsigned w0, unsigned w1) {
        if constexpr (complete.value)
          return rho1_nibbles_complete(w0, w1);
        else
          return nibbles32(rho1_16_f4<false>(w0), rho1_16_f4<false>(w1));
      };
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v8i b1[WN];
#pragma unroll
        for (int n = 0; n < WN; ++n)
          b1[n] = rho1_pair(word_of(xb[n], 2 * h), word_of(xb[n], 2 * h + 1));
#pragma unroll
        for (int m = 0; m < WM; ++m) {
          const v8i a1 = rho1_pair(word_of(xa[m], 2 * h), word_of(xa[m], 2 * h + 1));
#pragma unroll
          for (int n = 0; n < WN; ++n) acc[m][n] = mfma_f4(a1, b1[n], acc[m][n]);
        }
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        v4i b1[WN];
#pragma unroll
        for (int n = 0; n < WN; ++n) b1[n] = unpack16_rho1(word_of(xb[n], q));
#pragma unroll
        for (int m = 0; m < WM; ++m) {
          const v4i a1 = unpack16_rho1(word_of(xa[m], q));
#pragma unroll
          for (int n = 0; n < WN; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b1[n], acc[m][n], 0, 0, 0);
        }
      }
    }
  };
  wg_loop_f4<WM, WN>(
      a, I0, J0, active, pa, pb, stage,
      [&](const u4 (&xa)[WM], const u4 (&xb)[WN]) { body(xa, xb, std::true_type{}); },
      [&](const u4 (&xa)[WM], const u4 (&xb)[WN]) { body(xa, xb, std::false_type{}); });

  // The epilogue's inputs are read before its first store (a wait for a
  // load also waits for every store issued before it): the columns' into
  // registers, the 16 WM rows' (n(1) and factors) into this wave's part of
  // the stage, which every wave is done with after the barrier.
  struct RowIn {
    double w[2];
    int n1, pad0, pad1, pad2;
  };
  static_assert(sizeof(RowIn) == 32, "two 16-byte halves");
  static_assert(4 * 16 * WM * sizeof(RowIn) <= sizeof(u4) * (2 * WM + 2 * WN) * 64 * 2,
                "the rows fit in the stage");
  __syncthreads();
  if (!active) return;
  RowIn* rows = reinterpret_cast<RowIn*>(&stage[0][0][0]) + 16 * WM * wave;
  for (int t = lane; t < 16 * WM; t += 64) {
    const int64_t i = row0 + t, ii = i < a.n_a ? i : a.n_a - 1;
    RowIn ri;
    side_factors(a, 0, ii, ri.w);
    ri.n1 = reinterpret_cast<const v4i*>(a.counts_a)[ii].y;
    ri.pad0 = ri.pad1 = ri.pad2 = 0;
    rows[t] = ri;
  }

  // Epilogue: lane holds rows 4g + e (e = 0..3) of column rl of each 16x16 block.
  const int nf4 = (int)(4 * a.n_f);
  double wj[WN][2];
  int n1j[WN];
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    const int64_t j = col0 + 16 * n + rl;
    side_factors(a, 1, j, wj[n]);
    n1j[n] = reinterpret_cast<const v4i*>(a.counts_b)[j < a.n_b ? j : a.n_b - 1].y;
  }
  static_for<WM>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t i = row0 + 16 * m + 4 * g + e;
      const RowIn ri = rows[16 * m + 4 * g + e];
      const int n1i = ri.n1;
      const double(&wi)[2] = ri.w;
#pragma unroll
      for (int n = 0; n < WN; ++n) {
        const int64_t j = col0 + 16 * n + rl;
        int c11;
        if constexpr (F4)
          c11 = f4_count(acc[m][n][e]);
        else
          c11 = acc[m][n][e];
        const bool valid = i < a.n_a && j < a.n_b && !(a.tri && i >= j);
        emit_pair_staged(a, valid, i, j,
                         v4i{nf4 - 2 * n1i - 2 * n1j[n] + c11, 2 * n1j[n] - c11, 2 * n1i - c11,
                             c11},
                         wi, wj[n], outs);
      }
    }
  });
}

// Complete-data workgroup tile (every one of its rows has all n_f fields
// present, as the workgroup has voted): the one-plane product C11 of the
// whole (32 WM) x (32 WN) tile is computed by all four waves together, each
// over a quarter of the 256-field super-steps.  A wave then holds
// (2 WM) x (2 WN) 16x16 blocks, so each unpacked operand word feeds 2 WN
// (A side) or 2 WM (B side) MFMAs: half the unpack per MFMA of the per-wave
// form, which is bound by that unpack.  The four partial tiles are added
// through LDS (`part`, 4 x 16 x 64 x 16 bytes) in two halves of 16 blocks;
// wave w keeps block rows 2w and 2w+1 and finishes their pairs.  Every thread
// of the workgroup must call it (barriers).
template <int WM, int WN, bool F4>
__device__ __forceinline__ void mfma2_coop_complete(const Pair2Args& a, int64_t I0, int64_t J0,
                                                    v4i (*part)[16][64]) {
  constexpr int TM = 2 * WM, TN = 2 * WN;  // 16x16 blocks of the workgroup tile
  static_assert(TM == 8 && TN == 4, "the LDS halves hold 4 x 4 blocks");
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform
  const int g = lane >> 4, rl = lane & 15;
  // The loads: a wave-uniform base per block (its first row,
  // clamped; halves read from lane 0 so that it lives in scalar registers)
  // plus a 32-bit lane offset (r - rf < 16 rows of at most 2^28 bytes), so
  // that each load takes the scalar-base form and a step costs no vector
  // address arithmetic.
  gbytes base[TM + TN];
  uint32_t off[TM + TN];
#pragma unroll
  for (int b = 0; b < TM + TN; ++b) {
    const bool rows_i = b < TM;
    const int64_t n = rows_i ? a.n_a : a.n_b, ld = rows_i ? a.lda : a.ldb;
    const int64_t r0 = rows_i ? I0 + 16 * b : J0 + 16 * (b - TM);
    const int64_t rf = r0 < n ? r0 : n - 1, r = r0 + rl < n ? r0 + rl : n - 1;
    const uint64_t bp = (uint64_t)((rows_i ? a.va : a.vb) + rf * ld);
    base[b] = (gbytes)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bp >> 32)) << 32) |
                       (uint32_t)__builtin_amdgcn_readfirstlane((int)bp));
    off[b] = (uint32_t)((r - rf) * ld + 16 * g);
  }
  using Acc = std::conditional_t<F4, v4f, v4i>;
  Acc acc[TM][TN];
#pragma unroll
  for (int m = 0; m < TM; ++m)
#pragma unroll
    for (int n = 0; n < TN; ++n) acc[m][n] = Acc{0, 0, 0, 0};

  // `complete`: every field of the step is inside n_f (no padding code)
  auto body = [&](const u4 (&xa)[TM], const u4 (&xb)[TN], auto complete) {
    if constexpr (F4) {
      // rho(1) nibbles of two words: the short form on whole steps of
      // complete data, the padding-aware one on the last step
      auto rho1_pair = [&](unsigned w0, unsigned w1) {
        if constexpr (complete.value)
          return rho1_nibbles_complete(w0, w1);
        else
          return nibbles32(rho1_16_f4<false>(w0), rho1_16_f4<false>(w1));
      };
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        v8i b1[TN];
#pragma unroll
        for (int n = 0; n < TN; ++n) b1[n] = rho1_pair(word_of(xb[n], 2 * h), word_of(xb[n], 2 * h + 1));
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          const v8i a1 = rho1_pair(word_of(xa[m], 2 * h), word_of(xa[m], 2 * h + 1));
#pragma unroll
          for (int n = 0; n < TN; ++n) acc[m][n] = mfma_f4(a1, b1[n], acc[m][n]);
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        v4i b1[TN];
#pragma unroll
        for (int n = 0; n < TN; ++n) b1[n] = unpack16_rho1(word_of(xb[n], s));
#pragma unroll
        for (int m = 0; m < TM; ++m) {
          const v4i a1 = unpack16_rho1(word_of(xa[m], s));
#pragma unroll
          for (int n = 0; n < TN; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, b1[n], acc[m][n], 0, 0, 0);
        }
      }
    }
  };
  // This wave's super-steps [s_begin, s_end): the whole ones with plain
  // loads, then the partial one (holding field n_f - 1) if it is in range.
  const int64_t steps = (a.n_f + 255) / 256, nfull = a.n_f / 256;
  const int64_t s_begin = steps * wave / 4, s_end = steps * (wave + 1) / 4;
  const int64_t e_full = s_end < nfull ? s_end : nfull;
  for (int64_t st = s_begin; st < e_full; ++st) {
    u4 xa[TM], xb[TN];
    // 32-bit lane offsets: the bytes read lie below 16 ld <= 2^32
    const uint32_t so = (uint32_t)st * 64u;
#pragma unroll
    for (int m = 0; m < TM; ++m)
      xa[m] = *reinterpret_cast<const __attribute__((address_space(1))) u4*>(base[m] +
                                                                           (off[m] + so));
#pragma unroll
    for (int n = 0; n < TN; ++n)
      xb[n] = *reinterpret_cast<const __attribute__((address_space(1))) u4*>(base[TM + n] +
                                                                           (off[TM + n] + so));
    body(xa, xb, std::true_type{});
  }
  if (nfull >= s_begin && nfull < s_end) {
    const int64_t kb = nfull * 64 + 16 * g;
    u4 xa[TM], xb[TN];
#pragma unroll
    for (int m = 0; m < TM; ++m)
      xa[m] = load_fields64((const uint8_t*)(base[m] + off[m] - 16 * g), kb, a.n_f);
#pragma unroll
    for (int n = 0; n < TN; ++n)
      xb[n] = load_fields64((const uint8_t*)(base[TM + n] + off[TM + n] - 16 * g), kb, a.n_f);
    body(xa, xb, std::false_type{});
  }

  // Sum the four partial tiles: half h holds block rows 4h..4h+3, owned by
  // waves 2h and 2h+1 (two block rows each).
  v4i own[2][TN];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int n = 0; n < TN; ++n) {
        if constexpr (F4) {
          const v4f x = acc[4 * h + m][n];
          part[wave][m * TN + n][lane] =
              v4i{f4_count(x[0]), f4_count(x[1]), f4_count(x[2]), f4_count(x[3])};
        } else {
          part[wave][m * TN + n][lane] = acc[4 * h + m][n];
        }
      }
    __syncthreads();
    if ((wave >> 1) == h) {
#pragma unroll
      for (int r = 0; r < 2; ++r) {
        const int ml = 2 * (wave & 1) + r;  // block row within the half
#pragma unroll
        for (int n = 0; n < TN; ++n)
          own[r][n] = part[0][ml * TN + n][lane] + part[1][ml * TN + n][lane] +
                      part[2][ml * TN + n][lane] + part[3][ml * TN + n][lane];
      }
    }
    __syncthreads();
  }

  // Epilogue over block rows 2w, 2w+1: C10 = 2 n_i(1) - C11, C01 = 2 n_j(1) - C11,
  // C00 = 4 n_f - 2 n_i(1) - 2 n_j(1) + C11.
  const int nf4 = (int)(4 * a.n_f);
#pragma unroll
  for (int n = 0; n < TN; ++n) {
    const int64_t j = J0 + 16 * n + rl;
    double wj[2];
    side_factors(a, 1, j, wj);
    const int n1j = reinterpret_cast<const v4i*>(a.counts_b)[j < a.n_b ? j : a.n_b - 1].y;
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = I0 + 16 * (2 * wave + r) + 4 * g + e;
        const int n1i = reinterpret_cast<const v4i*>(a.counts_a)[i < a.n_a ? i : a.n_a - 1].y;
        double wi[2];
        side_factors(a, 0, i, wi);
        const int c11 = own[r][n][e];
        const bool valid = i < a.n_a && j < a.n_b && !(a.tri && i >= j);
        const v4i t{nf4 - 2 * n1i - 2 * n1j + c11, 2 * n1j - c11, 2 * n1i - c11, c11};
        if constexpr (F4)  // `part` is free after the reduction: stage the CCC stores
          emit_pair_staged(a, valid, i, j, t, wi, wj, reinterpret_cast<u4*>(&part[wave][0][0]));
        else
          emit_pair(a, valid, i, j, t, wi, wj);
      }
  }
}

// Workgroup vote for mfma2_coop_complete: every row of the (32 WM) x (32 WN)
// tile at (I0, J0) complete (rows past the end repeat the last row), in a
// call that does not accumulate (whose counts are this call's own).  Every
// thread of the workgroup must call it.
template <int WM, int WN>
__device__ __forceinline__ bool workgroup_complete(const Pair2Args& a, int64_t I0, int64_t J0) {
  if (a.accumulate || a.n_f <= 0) return false;  // uniform: no vote needed
  const int t = threadIdx.x;
  bool ok = true;
  if (t < 32 * WM) {
    int64_t r = I0 + t;
    r = r < a.n_a ? r : a.n_a - 1;
    ok = reinterpret_cast<const v4i*>(a.counts_a)[r].z == a.n_f;
  } else if (t < 32 * WM + 32 * WN) {
    int64_t r = J0 + (t - 32 * WM);
    r = r < a.n_b ? r : a.n_b - 1;
    ok = reinterpret_cast<const v4i*>(a.counts_b)[r].z == a.n_f;
  }
  return __syncthreads_and(ok ? 1 : 0) != 0;
}

// ---------------------------------------------------------------------------
// popcount path
//
// The paper's tally form (Sec. 3.1): per pair of packed words, build one word
// per tally target with shifts/AND/OR, then count its set bits.  Here each
// vector's 32 fields become three bit-planes
//   P = present (code != 10),  O = rho(1) >= 1 (codes 01, 11),  H = rho(1) = 2 (11),
// so rho(1) = O + H and rho(0) = 2P - rho(1).  Four sums per pair,
//   c11 = sum rho_i(1) rho_j(1) = pop(Oi&Oj) + pop(Oi&Hj) + pop(Hi&Oj) + pop(Hi&Hj)
//   s1p = sum rho_i(1) P_j      = pop(Oi&Pj) + pop(Hi&Pj)
//   sp1 = sum P_i rho_j(1)      = pop(Pi&Oj) + pop(Pi&Hj)
//   spp = sum P_i P_j           = pop(Pi&Pj)
// (9 AND + 9 bit-count-and-add per 32 fields), give the table exactly:
//   C11 = c11, C10 = 2 s1p - c11, C01 = 2 sp1 - c11,
//   C00 = 4 spp - 2 sp1 - 2 s1p + c11.
//
// Workgroup: 256 threads, a 64 x 64 tile of pairs, 4 x 4 pairs per thread.
// Each stage stages 256 fields of the 128 tile rows as bit-planes in LDS.
// Planes interleave the fields of two packed words (any order works as long
// as both vectors of a pair use the same one).
// ---------------------------------------------------------------------------

constexpr int kTile = 64;
constexpr int kStageWords = 8;  // 32-field plane words per stage (= 64 bytes per row)

struct Planes {
  unsigned p, o, h;
};

// Bit-planes of 32 fields held in two packed words (missing/padding already
// turned into code 10).
__device__ __forceinline__ Planes make_planes(unsigned w0, unsigned w1) {
  unsigned b0 = (w0 & kEven) | ((w1 & kEven) << 1);
  unsigned b1 = ((w0 >> 1) & kEven) | (((w1 >> 1) & kEven) << 1);
  Planes r;
  r.o = b0;
  r.h = b0 & b1;
  r.p = ~(b1 & ~b0);
  return r;
}

// LDS staging for one 64 x 64 tile (2 sides x 8 plane words x 64 rows).
struct Pop2Smem {
  unsigned P[2][kStageWords][kTile];
  unsigned O[2][kStageWords][kTile];
  unsigned H[2][kStageWords][kTile];
};

// The 64 x 64 tile (I, J) of pairs for the whole workgroup (256 threads; every
// thread must call it, it uses workgroup barriers).  COMPLETE: every row of
// the tile has all n_f fields present, so P = 1 and only c11 is counted
// (4 AND + bit counts per 32 fields); s1p = n_i(1), sp1 = n_j(1), spp = n_f.
template <bool COMPLETE>
__device__ __forceinline__ void pop2_tile_body(const Pair2Args& a, int64_t I, int64_t J,
                                               Pop2Smem& sm) {
  const int64_t I0 = I * kTile, J0 = J * kTile;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;

  // loader role: side 0 = A rows, side 1 = B rows; 32 bytes per thread
  const int side = tid >> 7, lrow = (tid >> 1) & 63, half = tid & 1;
  const uint8_t* lptr;
  if (side == 0) {
    int64_t r = I0 + lrow < a.n_a ? I0 + lrow : a.n_a - 1;
    lptr = a.va + r * a.lda;
  } else {
    int64_t r = J0 + lrow < a.n_b ? J0 + lrow : a.n_b - 1;
    lptr = a.vb + r * a.ldb;
  }

  unsigned c11[4][4], s1p[4][4], sp1[4][4], spp[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) c11[r][c] = s1p[r][c] = sp1[r][c] = spp[r][c] = 0;

  const int64_t nbytes = (a.n_f + 3) / 4;
  for (int64_t kb = 0; kb < nbytes; kb += 4 * kStageWords * 2) {
    u4 x0 = load_fields64(lptr, kb + 32 * half, a.n_f);
    u4 x1 = load_fields64(lptr, kb + 32 * half + 16, a.n_f);
    Planes pl[4] = {make_planes(x0.x, x0.y), make_planes(x0.z, x0.w), make_planes(x1.x, x1.y),
                    make_planes(x1.z, x1.w)};
    __syncthreads();  // the previous stage has been consumed
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sm.P[side][half * 4 + k][lrow] = pl[k].p;
      sm.O[side][half * 4 + k][lrow] = pl[k].o;
      sm.H[side][half * 4 + k][lrow] = pl[k].h;
    }
    __syncthreads();
#pragma unroll 2
    for (int kw = 0; kw < kStageWords; ++kw) {
      unsigned aP[4], aO[4], aH[4], bP[4], bO[4], bH[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        aP[r] = sm.P[0][kw][ty + 16 * r];
        aO[r] = sm.O[0][kw][ty + 16 * r];
        aH[r] = sm.H[0][kw][ty + 16 * r];
        bP[r] = sm.P[1][kw][tx + 16 * r];
        bO[r] = sm.O[1][kw][tx + 16 * r];
        bH[r] = sm.H[1][kw][tx + 16 * r];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          unsigned x = c11[r][c];
          x += __popc(aO[r] & bO[c]);
          x += __popc(aO[r] & bH[c]);
          x += __popc(aH[r] & bO[c]);
          x += __popc(aH[r] & bH[c]);
          c11[r][c] = x;
          if (!COMPLETE) {
            s1p[r][c] += __popc(aO[r] & bP[c]) + __popc(aH[r] & bP[c]);
            sp1[r][c] += __popc(aP[r] & bO[c]) + __popc(aP[r] & bH[c]);
            spp[r][c] += __popc(aP[r] & bP[c]);
          }
        }
    }
  }

  double wj[4][2];
#pragma unroll
  for (int c = 0; c < 4; ++c) side_factors(a, 1, J0 + tx + 16 * c, wj[c]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = I0 + ty + 16 * r;
    double wi[2];
    side_factors(a, 0, i, wi);
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t j = J0 + tx + 16 * c;
      const bool valid = i < a.n_a && j < a.n_b && !(a.tri && i >= j);
      int x11 = (int)c11[r][c], x1p = (int)s1p[r][c], xp1 = (int)sp1[r][c],
          xpp = (int)spp[r][c];
      if (COMPLETE) {
        x1p = reinterpret_cast<const v4i*>(a.counts_a)[i < a.n_a ? i : a.n_a - 1].y;
        xp1 = reinterpret_cast<const v4i*>(a.counts_b)[j < a.n_b ? j : a.n_b - 1].y;
        xpp = (int)a.n_f;
      }
      emit_pair(a, valid, i, j,
                v4i{4 * xpp - 2 * xp1 - 2 * x1p + x11, 2 * xp1 - x11, 2 * x1p - x11, x11}, wi,
                wj[c]);
    }
  }
}


__device__ __forceinline__ void pop2_block_tile(const Pair2Args& a, int64_t I, int64_t J,
                                                Pop2Smem& sm) {
  // workgroup-uniform vote: each thread checks the row it stages
  const int tid = threadIdx.x;
  const int side = tid >> 7, lrow = (tid >> 1) & 63;
  int mine = !a.accumulate && a.n_f > 0;
  if (side == 0) {
    int64_t r = I * kTile + lrow;
    r = r < a.n_a ? r : a.n_a - 1;
    mine = mine && reinterpret_cast<const v4i*>(a.counts_a)[r].z == a.n_f;
  } else {
    int64_t r = J * kTile + lrow;
    r = r < a.n_b ? r : a.n_b - 1;
    mine = mine && reinterpret_cast<const v4i*>(a.counts_b)[r].z == a.n_f;
  }
  if (__syncthreads_and(mine))
    pop2_tile_body<true>(a, I, J, sm);
  else
    pop2_tile_body<false>(a, I, J, sm);
}

}  // namespace tile2
}  // namespace ccc
