// pop2.hip -- 2-way tallies by bitwise AND + population count.
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
#include "common.h"
#include "kernels.h"

namespace ccc {

namespace {

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

__global__ __launch_bounds__(256) void pop2_kernel(Pair2Args a, int64_t tiles_side,
                                                   int64_t tiles_n) {
  __shared__ unsigned sP[2][kStageWords][kTile];
  __shared__ unsigned sO[2][kStageWords][kTile];
  __shared__ unsigned sH[2][kStageWords][kTile];

  int64_t I, J;
  if (a.tri) {
    tri_tile(blockIdx.x, tiles_side, I, J);
  } else {
    I = blockIdx.x / tiles_n;
    J = blockIdx.x % tiles_n;
  }
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
      sP[side][half * 4 + k][lrow] = pl[k].p;
      sO[side][half * 4 + k][lrow] = pl[k].o;
      sH[side][half * 4 + k][lrow] = pl[k].h;
    }
    __syncthreads();
#pragma unroll 2
    for (int kw = 0; kw < kStageWords; ++kw) {
      unsigned aP[4], aO[4], aH[4], bP[4], bO[4], bH[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        aP[r] = sP[0][kw][ty + 16 * r];
        aO[r] = sO[0][kw][ty + 16 * r];
        aH[r] = sH[0][kw][ty + 16 * r];
        bP[r] = sP[1][kw][tx + 16 * r];
        bO[r] = sO[1][kw][tx + 16 * r];
        bH[r] = sH[1][kw][tx + 16 * r];
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
          s1p[r][c] += __popc(aO[r] & bP[c]) + __popc(aH[r] & bP[c]);
          sp1[r][c] += __popc(aP[r] & bO[c]) + __popc(aP[r] & bH[c]);
          spp[r][c] += __popc(aP[r] & bP[c]);
        }
    }
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t i = I0 + ty + 16 * r;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t j = J0 + tx + 16 * c;
      if (i >= a.n_a || j >= a.n_b || (a.tri && i >= j)) continue;
      int x11 = (int)c11[r][c], x1p = (int)s1p[r][c], xp1 = (int)sp1[r][c],
          xpp = (int)spp[r][c];
      v4i t = v4i{4 * xpp - 2 * xp1 - 2 * x1p + x11, 2 * xp1 - x11, 2 * x1p - x11, x11};
      int64_t p = a.tri ? pair_index(a.n_a, i, j) : i * a.n_b + j;
      if (a.accumulate) {
        v4i o = *reinterpret_cast<const v4i*>(a.tables + 4 * p);
        t = t + o;
      }
      v4i ci = reinterpret_cast<const v4i*>(a.counts_a)[i];
      v4i cj = reinterpret_cast<const v4i*>(a.counts_b)[j];
      store_pair(p, t, ci, cj, a.gamma, a.tables, a.ccc);
    }
  }
}

}  // namespace

hipError_t launch_pop2(const Pair2Args& a, hipStream_t stream) {
  int64_t tm = (a.n_a + kTile - 1) / kTile, tn = (a.n_b + kTile - 1) / kTile;
  int64_t ntiles = a.tri ? tm * (tm + 1) / 2 : tm * tn;
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  timing_begin("pop2", stream);
  hipLaunchKernelGGL(pop2_kernel, dim3((unsigned)ntiles), dim3(256), 0, stream, a, tm, tn);
  timing_end(stream);
  return hipGetLastError();
}

}  // namespace ccc
