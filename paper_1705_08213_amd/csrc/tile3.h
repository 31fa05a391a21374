// tile3.h -- output of one 3-way triple (Sec. 2.2, Eqs. (4)-(5)), shared by
// the MFMA and popcount 3-way kernels.
#pragma once

#include "common.h"
#include "kernels.h"

namespace ccc {

// CCC of one triple from its table t (entry 4a+2b+c) and the per-vector
// factors w_x[a] = 1 - gamma f_x(a); all zero when m_ijk = 0.
__device__ __forceinline__ void triple_ccc(const int (&t)[8], const double (&wi)[2],
                                           const double (&wj)[2], const double (&wk)[2],
                                           double (&r)[8]) {
#pragma clang fp contract(off)
  int sum = 0;
#pragma unroll
  for (int x = 0; x < 8; ++x) sum += t[x];
  const int m_ijk = sum >> 3;  // fields where all three are present
  if (m_ijk > 0) {
    const double den = 8.0 * (double)m_ijk, y = 1.0 / den;
#pragma unroll
    for (int x = 0; x < 8; ++x)
      r[x] = quot_rn((double)t[x], den, y) * wi[x >> 2] * wj[(x >> 1) & 1] * wk[x & 1];
  } else {
#pragma unroll
    for (int x = 0; x < 8; ++x) r[x] = 0.0;
  }
}

// Factors of vector x (clamped into range); only computed when some CCC value
// is produced.
__device__ __forceinline__ void triple_factors(const Triple3Args& a, int64_t x, double (&w)[2]) {
  if (a.ccc || a.sel.count) {
    vector_factors(a.counts, x < a.n ? x : a.n - 1, a.gamma, w);
  } else {
    w[0] = w[1] = 0.0;
  }
}

// Dense mode: table and/or CCC at entry T(i,j,k) - t_base.  Selection mode:
// keep the triple if one of its CCC values reaches the threshold; then every
// lane of the wave must call (one atomic per wave) and `valid` marks lanes
// that hold a triple.  wi / wj / wk are the factors of i, j and k (read on
// valid lanes only).
__device__ __forceinline__ void emit_triple(const Triple3Args& a, bool valid, int64_t i,
                                            int64_t j, int64_t k, const int (&t)[8],
                                            const double (&wi)[2], const double (&wj)[2],
                                            const double (&wk)[2]) {
  valid = valid && i >= a.i_begin && i < a.i_end;
  if (a.sel.count) {
    double r[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool keep = false;
    int64_t p = 0;
    if (valid) {
      p = triple_index(a.n, i, j, k);
      triple_ccc(t, wi, wj, wk, r);
#pragma unroll
      for (int x = 0; x < 8; ++x) keep = keep || r[x] >= a.sel.threshold;
    }
    const int64_t slot = select_slot(keep, a.sel.count);
    if (slot >= 0 && slot < a.sel.cap) {
      a.sel.index[slot] = p;
      double2* c = reinterpret_cast<double2*>(a.sel.ccc + 8 * slot);
#pragma unroll
      for (int x = 0; x < 4; ++x) c[x] = double2{r[2 * x], r[2 * x + 1]};
      if (a.sel.tables) {
        v4i* o = reinterpret_cast<v4i*>(a.sel.tables + 8 * slot);
        o[0] = v4i{t[0], t[1], t[2], t[3]};
        o[1] = v4i{t[4], t[5], t[6], t[7]};
      }
    }
    return;
  }
  if (!valid) return;
  const int64_t p = triple_index(a.n, i, j, k) - a.t_base;
  if (a.tables) {
    v4i* o = reinterpret_cast<v4i*>(a.tables + 8 * p);
    o[0] = v4i{t[0], t[1], t[2], t[3]};
    o[1] = v4i{t[4], t[5], t[6], t[7]};
  }
  if (a.ccc) {
    double r[8];
    triple_ccc(t, wi, wj, wk, r);
    double2* c = reinterpret_cast<double2*>(a.ccc + 8 * p);
#pragma unroll
    for (int x = 0; x < 4; ++x) c[x] = double2{r[2 * x], r[2 * x + 1]};
  }
}

// emit_triple with the dense output written through LDS so that every store
// instruction covers whole stretches of memory.  Every lane of the wave must
// call it; lane (g, rl) holds triple (i, j, k) with k = k_base + rl for one i
// per 16-lane group g (consecutive triples when valid, since T(i,j,k) grows by
// one with k).  Each group writes its 16 tables (32 B each) and CCC rows
// (64 B each) into `scratch` (wave-private, 384 x 16 B) in output order, then
// lane rl stores 16-byte piece rl of each 256-byte stretch, skipping pieces of
// invalid triples.  Selection mode falls back to emit_triple.
__device__ __forceinline__ void emit_triple_staged(const Triple3Args& a, bool valid, int64_t i,
                                                   int64_t j, int64_t k, const int (&t)[8],
                                                   const double (&wi)[2], const double (&wj)[2],
                                                   const double (&wk)[2], u4* scratch) {
  if (a.sel.count) {
    emit_triple(a, valid, i, j, k, t, wi, wj, wk);
    return;
  }
  valid = valid && i >= a.i_begin && i < a.i_end;
  const int lane = threadIdx.x & 63, g = lane >> 4, rl = lane & 15;
  const unsigned gm = (unsigned)(__ballot(valid ? 1 : 0) >> (16 * g)) & 0xFFFFu;
  // entry of the group's lane 0 (unused when no triple of the group is
  // valid): T(i, j, k) is affine in k, so it follows from that lane's k
  // whether or not its own triple is valid
  const int64_t p0 = triple_index(a.n, i, j, k - rl) - a.t_base;
  u4* T = scratch + 32 * g;        // 16 tables of the group: 32 x 16 B
  u4* C = scratch + 128 + 64 * g;  // 16 CCC rows: 64 x 16 B
  if (a.tables) {
    T[2 * rl] = u4{(unsigned)t[0], (unsigned)t[1], (unsigned)t[2], (unsigned)t[3]};
    T[2 * rl + 1] = u4{(unsigned)t[4], (unsigned)t[5], (unsigned)t[6], (unsigned)t[7]};
  }
  if (a.ccc) {
    double r[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (valid) triple_ccc(t, wi, wj, wk, r);
    double2* Cd = reinterpret_cast<double2*>(C + 4 * rl);
#pragma unroll
    for (int x = 0; x < 4; ++x) Cd[x] = double2{r[2 * x], r[2 * x + 1]};
  }
  // the wave's LDS accesses run in program order; keep the compiler to it
  asm volatile("" ::: "memory");
  // streaming stores: each instruction writes whole lines of output that is
  // written once and not read back here
  if (a.tables) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int piece = 16 * q + rl;
      const u4 d = T[piece];
      if ((gm >> (piece >> 1)) & 1u)
        __builtin_nontemporal_store(d, reinterpret_cast<u4*>(a.tables + 8 * p0) + piece);
    }
  }
  if (a.ccc) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int piece = 16 * q + rl;
      const u4 d = C[piece];
      if ((gm >> (piece >> 2)) & 1u)
        __builtin_nontemporal_store(d, reinterpret_cast<u4*>(a.ccc + 8 * p0) + piece);
    }
  }
  asm volatile("" ::: "memory");  // the scratch is reused by the next call
}

}  // namespace ccc
