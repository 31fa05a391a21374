// pop3.hip -- 3-way tallies by bitwise AND + population count (reference path).
//
// Bit-planes per 32 fields as in pop2: P (present), O (rho(1) >= 1),
// H (rho(1) = 2), with rho(1) = O + H and rho(0) = 2P - rho(1).  For each
// triple the kernel accumulates the eight sums
//   T[x][y][z] = sum_q x_i y_j z_k,   x, y, z in {P, R},  R = rho(1),
// each R expanding into its O and H planes (27 three-way AND + bit counts per
// 32 fields), and rebuilds the table from them:
//   C(a,b,c) = sum_{x,y,z} w_a(x) w_b(y) w_c(z) T[x][y][z],
//   w_0 = (2, -1) and w_1 = (0, 1) over (P, R).
// Same tetrahedral work units as the MFMA kernel, with 64 x 64 (i, k) tiles
// and 4 x 4 triples per thread; the 129 tile rows (64 i, 64 k and j) are
// staged as planes in LDS, 256 fields at a time.
#include "tile3.h"

namespace ccc {

namespace {

constexpr int kTile = 64;
static_assert(kTile == kUnitTile, "work units are kUnitTile-row tile pairs");
constexpr int kStageWords = 8;

__device__ __forceinline__ void make_planes(unsigned w0, unsigned w1, unsigned& p, unsigned& o,
                                            unsigned& h) {
  unsigned b0 = (w0 & kEven) | ((w1 & kEven) << 1);
  unsigned b1 = ((w0 >> 1) & kEven) | (((w1 >> 1) & kEven) << 1);
  o = b0;
  h = b0 & b1;
  p = ~(b1 & ~b0);
}

__global__ __launch_bounds__(256) void pop3_kernel(Triple3Args a, UnitGrid ug,
                                                   const int64_t* __restrict__ offs,
                                                   int64_t unit_base, int64_t count) {
#pragma clang fp contract(off)
  __shared__ unsigned sP[2][kStageWords][kTile], sO[2][kStageWords][kTile],
      sH[2][kStageWords][kTile];
  __shared__ unsigned jP[kStageWords], jO[kStageWords], jH[kStageWords];

  const int64_t n = a.n;
  int64_t j, it, kt;
  unit_coords(unit_base + xcd_unit(blockIdx.x, count), ug, offs, j, it, kt);
  const int64_t I0 = it * kTile, K0 = kt * kTile;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;

  const int side = tid >> 7, lrow = (tid >> 1) & 63, half = tid & 1;
  int64_t lr = (side == 0 ? I0 : K0) + lrow;
  if (lr >= n) lr = n - 1;
  const uint8_t* lptr = a.v + lr * a.ld;
  const uint8_t* jptr = a.v + j * a.ld;

  // T[x][y][z] with x,y,z in {P=0, R=1}: index 4x + 2y + z
  unsigned T[4][4][8];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int e = 0; e < 8; ++e) T[r][c][e] = 0;

  const int64_t nbytes = (a.n_f + 3) / 4;
  for (int64_t kb = 0; kb < nbytes; kb += 64) {
    u4 x0 = load_fields64(lptr, kb + 32 * half, a.n_f);
    u4 x1 = load_fields64(lptr, kb + 32 * half + 16, a.n_f);
    unsigned pp[4], oo[4], hh[4];
    make_planes(x0.x, x0.y, pp[0], oo[0], hh[0]);
    make_planes(x0.z, x0.w, pp[1], oo[1], hh[1]);
    make_planes(x1.x, x1.y, pp[2], oo[2], hh[2]);
    make_planes(x1.z, x1.w, pp[3], oo[3], hh[3]);
    unsigned jp = 0, jo = 0, jh = 0, jp2 = 0, jo2 = 0, jh2 = 0;
    if (tid < 4) {
      u4 y = load_fields64(jptr, kb + 16 * tid, a.n_f);
      make_planes(y.x, y.y, jp, jo, jh);
      make_planes(y.z, y.w, jp2, jo2, jh2);
    }
    __syncthreads();  // the previous stage has been consumed
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sP[side][half * 4 + k][lrow] = pp[k];
      sO[side][half * 4 + k][lrow] = oo[k];
      sH[side][half * 4 + k][lrow] = hh[k];
    }
    if (tid < 4) {
      jP[2 * tid] = jp; jO[2 * tid] = jo; jH[2 * tid] = jh;
      jP[2 * tid + 1] = jp2; jO[2 * tid + 1] = jo2; jH[2 * tid + 1] = jh2;
    }
    __syncthreads();
    for (int kw = 0; kw < kStageWords; ++kw) {
      const unsigned Pj = jP[kw], Oj = jO[kw], Hj = jH[kw];
      unsigned kP[4], kO[4], kH[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        kP[c] = sP[1][kw][tx + 16 * c];
        kO[c] = sO[1][kw][tx + 16 * c];
        kH[c] = sH[1][kw][tx + 16 * c];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const unsigned Pi = sP[0][kw][ty + 16 * r], Oi = sO[0][kw][ty + 16 * r],
                       Hi = sH[0][kw][ty + 16 * r];
        // i-j plane products: x in {P, O, H} for i, y in {P, O, H} for j
        const unsigned PP = Pi & Pj, PO = Pi & Oj, PH = Pi & Hj;
        const unsigned OP = Oi & Pj, OO = Oi & Oj, OH = Oi & Hj;
        const unsigned HP = Hi & Pj, HO = Hi & Oj, HH = Hi & Hj;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const unsigned zp = kP[c], zo = kO[c], zh = kH[c];
          unsigned* t = T[r][c];
          t[0] += __popc(PP & zp);                                            // P P P
          t[1] += __popc(PP & zo) + __popc(PP & zh);                          // P P R
          t[2] += __popc(PO & zp) + __popc(PH & zp);                          // P R P
          t[3] += __popc(PO & zo) + __popc(PO & zh) + __popc(PH & zo) + __popc(PH & zh);
          t[4] += __popc(OP & zp) + __popc(HP & zp);                          // R P P
          t[5] += __popc(OP & zo) + __popc(OP & zh) + __popc(HP & zo) + __popc(HP & zh);
          t[6] += __popc(OO & zp) + __popc(OH & zp) + __popc(HO & zp) + __popc(HH & zp);
          t[7] += __popc(OO & zo) + __popc(OO & zh) + __popc(OH & zo) + __popc(OH & zh) +
                  __popc(HO & zo) + __popc(HO & zh) + __popc(HH & zo) + __popc(HH & zh);
        }
      }
    }
  }

  double wj[2], wi[4][2];
  triple_factors(a, j, wj);
#pragma unroll
  for (int r = 0; r < 4; ++r) triple_factors(a, I0 + ty + 16 * r, wi[r]);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t k = K0 + tx + 16 * c;
    const bool kvalid = k > j && k < n;
    double wk[2];
    triple_factors(a, k, wk);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i = I0 + ty + 16 * r;
      // w_0 = (2, -1), w_1 = (0, 1) over (P, R); unsigned: partial sums may
      // leave the int32 range, the total fits
      int tab[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int aa = e >> 2, bb = (e >> 1) & 1, cc = e & 1;
        unsigned s = 0;
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int z = 0; z < 2; ++z) {
              const unsigned wx = aa ? (x ? 1u : 0u) : (x ? ~0u : 2u);
              const unsigned wy = bb ? (y ? 1u : 0u) : (y ? ~0u : 2u);
              const unsigned wz = cc ? (z ? 1u : 0u) : (z ? ~0u : 2u);
              s += wx * wy * wz * T[r][c][4 * x + 2 * y + z];
            }
        tab[e] = (int)s;
      }
      emit_triple(a, kvalid && i < j, i, j, k, tab, wi[r], wj, wk);
    }
  }
}

}  // namespace

hipError_t launch_pop3(const Triple3Args& a, hipStream_t stream) {
  return launch_units(pop3_kernel, a, kTile, "pop3", stream);
}

}  // namespace ccc
