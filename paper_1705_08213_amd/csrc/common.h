// common.h -- device helpers shared by the CCC kernels (gfx950).
//
// Packed input: field q of a row sits at bits 2(q%4), 2(q%4)+1 of byte q/4;
// code = allele pair (high, low); 0b10 marks a missing entry.  Every helper
// that reads the input turns fields past n_f into the missing code, so the
// padding bits never reach a tally.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ccc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef unsigned u4 __attribute__((ext_vector_type(4)));

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

// CCC of one pair (Eqs. (2)-(3)) from its table t = (C00, C01, C10, C11) and
// the counts (n(0), n(1), m, 0) of the two vectors; all zero when m_ij = 0.
__device__ __forceinline__ void pair_ccc(v4i t, v4i ci, v4i cj, double gamma, double (&r)[4]) {
#pragma clang fp contract(off)
  int sum = t.x + t.y + t.z + t.w;
  int m_ij = sum >> 2;  // fields where both are present
  if (m_ij > 0) {
    double den = 4.0 * (double)m_ij;
    double wi0 = one_minus_gf(ci.x, ci.z, gamma), wi1 = one_minus_gf(ci.y, ci.z, gamma);
    double wj0 = one_minus_gf(cj.x, cj.z, gamma), wj1 = one_minus_gf(cj.y, cj.z, gamma);
    r[0] = ((double)t.x / den) * wi0 * wj0;
    r[1] = ((double)t.y / den) * wi0 * wj1;
    r[2] = ((double)t.z / den) * wi1 * wj0;
    r[3] = ((double)t.w / den) * wi1 * wj1;
  } else {
    r[0] = r[1] = r[2] = r[3] = 0.0;
  }
}

// Dense 2-way store of entry p: the table (if `tables`) and CCC (if `ccc`).
__device__ __forceinline__ void store_pair(int64_t p, v4i t, v4i ci, v4i cj, double gamma,
                                           int32_t* __restrict__ tables,
                                           double* __restrict__ ccc) {
  if (tables) *reinterpret_cast<v4i*>(tables + 4 * p) = t;
  if (ccc) {
    double r[4];
    pair_ccc(t, ci, cj, gamma, r);
    double2* out = reinterpret_cast<double2*>(ccc + 4 * p);
    out[0] = double2{r[0], r[1]};
    out[1] = double2{r[2], r[3]};
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

// ---------------------------------------------------------------------------
// Tetrahedral work units for the 3-way kernels: for middle vector j, the
// I tiles [0, ceil(j/bi)) (rows below j) times the K tiles
// [floor((j+1)/bk), ceil(n/bk)) (columns above j).
// ---------------------------------------------------------------------------
// Only I tiles meeting rows [i_begin, min(j, i_end)) are kept (a staged
// range of first indices).
__host__ __device__ __forceinline__ int64_t units_for_j(int64_t j, int64_t n, int64_t bi,
                                                        int64_t bk, int64_t i_begin,
                                                        int64_t i_end) {
  if (j < 1 || j > n - 2 || j <= i_begin) return 0;
  const int64_t hi = j < i_end ? j : i_end;
  if (hi <= i_begin) return 0;
  int64_t ni = (hi + bi - 1) / bi - i_begin / bi;
  int64_t nk = (n + bk - 1) / bk - (j + 1) / bk;
  return ni * nk;
}

// Unit u -> (j, I tile, K tile), given offs[j] = units of all j' < j (j = 0..n).
__device__ __forceinline__ void unit_coords(int64_t u, int64_t n, int64_t bi, int64_t bk,
                                            int64_t i_begin, int64_t i_end,
                                            const int64_t* __restrict__ offs, int64_t& j,
                                            int64_t& it, int64_t& kt) {
  int64_t lo = 0, hi = n;  // offs[lo] <= u < offs[hi]
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) >> 1;
    if (offs[mid] <= u) lo = mid; else hi = mid;
  }
  j = lo;
  const int64_t r = u - offs[j];
  const int64_t top = j < i_end ? j : i_end;
  const int64_t ni = (top + bi - 1) / bi - i_begin / bi;
  it = i_begin / bi + r % ni;
  kt = (j + 1) / bk + r / ni;
}

}  // namespace ccc

namespace ccc {

void timing_begin(const char* name, hipStream_t stream);
void timing_end(hipStream_t stream);

namespace {

// offs[j] = number of units of all j' < j, for j = 0..n (one workgroup).
__global__ void unit_offsets_kernel(int64_t n, int64_t bi, int64_t bk, int64_t i_begin,
                                    int64_t i_end, int64_t* __restrict__ offs) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1 + 1023) / 1024;
  const int64_t lo = t * per, hi = lo + per < n + 1 ? lo + per : n + 1;
  int64_t s = 0;
  for (int64_t j = lo; j < hi; ++j) s += units_for_j(j, n, bi, bk, i_begin, i_end);
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
  for (int64_t j = lo; j < hi; ++j) {
    offs[j] = run;
    run += units_for_j(j, n, bi, bk, i_begin, i_end);
  }
}

// Launch a 3-way kernel over all its tetrahedral units (256 threads each),
// in slices of at most 2^30 workgroups.  a.offs must hold n+1 int64.
template <typename Kernel, typename Args>
hipError_t launch_units(Kernel kernel, const Args& a, int64_t bi, int64_t bk, const char* name,
                        hipStream_t stream) {
  int64_t total = 0;
  for (int64_t j = 0; j < a.n; ++j) total += units_for_j(j, a.n, bi, bk, a.i_begin, a.i_end);
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(unit_offsets_kernel, dim3(1), dim3(1024), 0, stream, a.n, bi, bk, a.i_begin,
                     a.i_end, a.offs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t kMaxGrid = 0x40000000;
  timing_begin(name, stream);
  for (int64_t base = 0; base < total; base += kMaxGrid) {
    int64_t cnt = total - base < kMaxGrid ? total - base : kMaxGrid;
    hipLaunchKernelGGL(kernel, dim3((unsigned)cnt), dim3(256), 0, stream, a,
                       (const int64_t*)a.offs, base);
    if ((e = hipGetLastError()) != hipSuccess) break;
  }
  timing_end(stream);
  return e;
}

}  // namespace
}  // namespace ccc
