// common.h -- device helpers shared by the CCC kernels (gfx950).
//
// Packed input: field q of a row sits at bits 2(q%4), 2(q%4)+1 of byte q/4;
// code = allele pair (high, low); 0b10 marks a missing entry.  Every helper
// that reads the input turns fields past n_f into the missing code, so the
// padding bits never reach a tally.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace ccc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Byte pointer into global memory.  A pointer rebuilt from integers (a
// wave-uniform row base read from lane 0) or loaded from a table is generic
// to the compiler, and loads through it take the flat form (no scalar base,
// counted against the LDS counter too); through this type they take the
// global form.
typedef const __attribute__((address_space(1))) uint8_t* gbytes;

// 16 fields of the missing code (0b10 each).
constexpr unsigned kAllMissing = 0xAAAAAAAAu;
constexpr unsigned kEven = 0x55555555u;

// Keep the first `valid` (clamped to [0,16]) fields of a 16-field word and
// turn the rest into missing entries.
__device__ __forceinline__ unsigned mask_fields(unsigned w, int valid) {
  if (valid >= 16) return w;
  if (valid <= 0) return kAllMissing;
  unsigned keep = (1u << (2 * valid)) - 1u;
  return (w & keep) | (kAllMissing & ~keep);
}

// Load 16 bytes (64 fields) of a row at byte offset `ob` (a multiple of 16).
// Only pieces holding at least one of the first n_f fields are read, so a
// row is never read past ceil(n_f/4) rounded up to 16 bytes (which the row
// stride always covers); other pieces come back as missing entries.  Fields
// at or past n_f are masked to missing.
__device__ __forceinline__ u4 load_fields64(const uint8_t* __restrict__ row, int64_t ob,
                                            int64_t n_f) {
  u4 w;
  if (ob * 4 < n_f) {
    w = *reinterpret_cast<const u4*>(row + ob);
  } else {
    w = u4{kAllMissing, kAllMissing, kAllMissing, kAllMissing};
  }
  int64_t q0 = ob * 4;  // first field of the 16 bytes
  if (q0 + 64 > n_f) {
    int64_t rem = n_f - q0;
    w.x = mask_fields(w.x, (int)(rem < 0 ? 0 : (rem > 16 ? 16 : rem)));
    rem -= 16;
    w.y = mask_fields(w.y, (int)(rem < 0 ? 0 : (rem > 16 ? 16 : rem)));
    rem -= 16;
    w.z = mask_fields(w.z, (int)(rem < 0 ? 0 : (rem > 16 ? 16 : rem)));
    rem -= 16;
    w.w = mask_fields(w.w, (int)(rem < 0 ? 0 : (rem > 16 ? 16 : rem)));
  }
  return w;
}

// Lexicographic index of pair (i, j), i < j, among n vectors.
__device__ __forceinline__ int64_t pair_index(int64_t n, int64_t i, int64_t j) {
  return i * n - i * (i + 1) / 2 + (j - i - 1);
}

__device__ __forceinline__ int64_t choose2(int64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }
__device__ __forceinline__ int64_t choose3(int64_t n) {
  return n < 3 ? 0 : n * (n - 1) / 2 * (n - 2) / 3;
}

// Lexicographic rank of triple (i, j, k), i < j < k, among n vectors.
__device__ __forceinline__ int64_t triple_index(int64_t n, int64_t i, int64_t j, int64_t k) {
  return choose3(n) - choose3(n - i) + choose2(n - i - 1) - choose2(n - j) + (k - j - 1);
}

// 1 - gamma f_i(a) with f_i(a) = n_i(a) / (2 m_i)  (Eq. (1)); f = 0 when m_i = 0.
// Contraction into fma is disabled in the epilogue so that it rounds exactly
// as the plain formula written left to right.
__device__ __forceinline__ double one_minus_gf(int n_a, int m, double gamma) {
#pragma clang fp contract(off)
  double f = m > 0 ? (double)n_a / (2.0 * (double)m) : 0.0;
  return 1.0 - gamma * f;
}

// Per-vector factors w(a) = 1 - gamma f(a), a = 0, 1, from the counts
// (n(0), n(1), m, 0) of one vector.
__device__ __forceinline__ void vector_factors(const int32_t* __restrict__ counts, int64_t x,
                                               double gamma, double (&w)[2]) {
  const v4i c = reinterpret_cast<const v4i*>(counts)[x];
  w[0] = one_minus_gf(c.x, c.z, gamma);
  w[1] = one_minus_gf(c.y, c.z, gamma);
}

// t / den rounded to nearest, for integers 0 <= t <= den < 2^34, given
// y = 1/den from one IEEE division shared by all t over the same den.
// q0 = t y lies within 2 ulp of x = t/den; the residual t - q0 den is then a
// multiple of ulp(q0) smaller than 2^36 ulp(q0), so one fma gets it exactly; and
// q0 + residual * y is within 2^-52 ulp of x.  A quotient of such integers is
// either representable (its reduced denominator is a power of two and its
// numerator has at most 34 bits) or at least 2^-35 ulp away from every
// rounding midpoint, so the final rounding gives exactly RN(t/den): the same
// double as the division itself.
__device__ __forceinline__ double quot_rn(double t, double den, double y) {
#pragma clang fp contract(off)
  const double q0 = t * y;
  const double r = __builtin_fma(-q0, den, t);
  return __builtin_fma(r, y, q0);
}

// CCC of one pair (Eqs. (2)-(3)) from its table t = (C00, C01, C10, C11) and
// the factors w_i, w_j of its two vectors; all zero when m_ij = 0.
__device__ __forceinline__ void pair_ccc(v4i t, const double (&wi)[2], const double (&wj)[2],
                                         double (&r)[4]) {
#pragma clang fp contract(off)
  int sum = t.x + t.y + t.z + t.w;
  int m_ij = sum >> 2;  // fields where both are present
  if (m_ij > 0) {
    const double den = 4.0 * (double)m_ij, y = 1.0 / den;
    r[0] = quot_rn((double)t.x, den, y) * wi[0] * wj[0];
    r[1] = quot_rn((double)t.y, den, y) * wi[0] * wj[1];
    r[2] = quot_rn((double)t.z, den, y) * wi[1] * wj[0];
    r[3] = quot_rn((double)t.w, den, y) * wi[1] * wj[1];
  } else {
    r[0] = r[1] = r[2] = r[3] = 0.0;
  }
}

// Dense 2-way store of entry p: the table (if `tables`) and CCC (if `ccc`).
__device__ __forceinline__ void store_pair(int64_t p, v4i t, const double (&wi)[2],
                                           const double (&wj)[2], int32_t* __restrict__ tables,
                                           double* __restrict__ ccc) {
  // streaming stores: the dense output is written once and not read back here
  if (tables) __builtin_nontemporal_store(t, reinterpret_cast<v4i*>(tables + 4 * p));
  if (ccc) {
    double r[4];
    pair_ccc(t, wi, wj, r);
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2* out = reinterpret_cast<d2*>(ccc + 4 * p);
    __builtin_nontemporal_store(d2{r[0], r[1]}, out);
    __builtin_nontemporal_store(d2{r[2], r[3]}, out + 1);
  }
}

// Slot for this lane's record in a selection buffer: one atomic per wave
// (ballot of the lanes that keep a record); every lane of the wave must call
// it.  Returns -1 for lanes that keep nothing.
__device__ __forceinline__ int64_t select_slot(bool keep, unsigned long long* count) {
  const unsigned long long mask = __ballot(keep ? 1 : 0);
  if (mask == 0ull) return -1;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(count, (unsigned long long)__popcll(mask));
  base = __shfl(base, leader);
  if (!keep) return -1;
  return (int64_t)(base + (unsigned long long)__popcll(mask & ((1ull << lane) - 1ull)));
}

}  // namespace ccc

namespace ccc {

// 1-way counts of one packed row by one wave (64 lanes): writes or adds
// (n(0), n(1), m, 0) at out[0..3] from lane 0.  Popcounts on the bit planes:
// b0 = low bits (01, 11), b1 = high bits (11, 10); n(1) = pop(b0) +
// pop(b0 & b1), missing = pop(b1 & ~b0), n(0) = 2m - n(1).
__device__ __forceinline__ void count_row_wave(const uint8_t* __restrict__ r, int64_t n_f,
                                               int32_t* __restrict__ out, int accumulate) {
  const int lane = threadIdx.x & 63;
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
    v4i* o4 = reinterpret_cast<v4i*>(out);
    if (accumulate) {
      v4i o = *o4;
      c = v4i{o.x + c.x, o.y + c.y, o.z + c.z, 0};
    }
    *o4 = c;
  }
}

}  // namespace ccc

namespace ccc {

// Tile (I, J), I <= J, of the t-th entry of the row-major upper triangle
// (diagonal included) of a T x T tile grid.
__device__ __forceinline__ void tri_tile(int64_t t, int64_t T, int64_t& I, int64_t& J) {
  double b = 2.0 * (double)T + 1.0;
  int64_t i = (int64_t)((b - sqrt(b * b - 8.0 * (double)t)) * 0.5);
  if (i < 0) i = 0;
  if (i > T - 1) i = T - 1;
  while (i > 0 && i * T - i * (i - 1) / 2 > t) --i;
  while (i + 1 < T && (i + 1) * T - (i + 1) * i / 2 <= t) ++i;
  I = i;
  J = i + (t - (i * T - i * (i - 1) / 2));
}

}  // namespace ccc

namespace ccc {

void timing_begin(const char* name, hipStream_t stream);
void timing_end(hipStream_t stream);

namespace {

// offs[p] = number of units of all tile pairs before p, for p = 0..pairs
// (one workgroup; thread t walks a contiguous run of pairs).
__global__ void unit_offsets_kernel(UnitGrid g, int64_t* __restrict__ offs) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t P = grid_pairs(g);
  const int64_t per = (P + 1023) / 1024;
  const int64_t lo = t * per, hi = lo + per < P ? lo + per : P;
  int64_t s = 0, it = 0, kt = 0;
  if (lo < hi) pair_tiles(g, lo, it, kt);
  for (int64_t p = lo; p < hi; ++p) {
    s += pair_units(g, it, kt);
    if (++kt == g.nt) kt = ++it;
  }
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int x = 0; x < 1024; ++x) {
      int64_t v = part[x];
      part[x] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = part[t];
  if (lo < hi) pair_tiles(g, lo, it, kt);
  for (int64_t p = lo; p < hi; ++p) {
    offs[p] = run;
    run += pair_units(g, it, kt);
    if (++kt == g.nt) kt = ++it;
  }
  if (t == 1023) offs[P] = run;
}

// Units of a whole grid (host side).
inline int64_t grid_units(const UnitGrid& g) {
  int64_t total = 0;
  for (int64_t it = g.it0; it < g.it1; ++it)
    for (int64_t kt = it; kt < g.nt; ++kt) total += pair_units(g, it, kt);
  return total;
}

// Launch a 3-way kernel over all its tetrahedral units of b x b tiles and
// `run` middle vectors (256 threads each), in slices of at most 2^30
// workgroups.  offs must hold grid_pairs + 1 int64; `name` (if any) opens a
// timing mark around the launches.
template <typename Kernel, typename Args>
hipError_t launch_units(Kernel kernel, const Args& a, int64_t b, const char* name,
                        hipStream_t stream, int64_t run = 1, int64_t* offs = nullptr) {
  if (!offs) offs = a.offs;
  const UnitGrid g = unit_grid(a.n, b, a.i_begin, a.i_end, run);
  const int64_t total = grid_units(g);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(unit_offsets_kernel, dim3(1), dim3(1024), 0, stream, g, offs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t kMaxGrid = 0x40000000;
  if (name) timing_begin(name, stream);
  for (int64_t base = 0; base < total; base += kMaxGrid) {
    int64_t cnt = total - base < kMaxGrid ? total - base : kMaxGrid;
    hipLaunchKernelGGL(kernel, dim3((unsigned)cnt), dim3(256), 0, stream, a, g,
                       (const int64_t*)offs, base, cnt);
    if ((e = hipGetLastError()) != hipSuccess) break;
  }
  if (name) timing_end(stream);
  return e;
}

}  // namespace
}  // namespace ccc
