// multi2.hip -- multi-allelic 2-way tallies and CCC on the matrix cores
// (markers with s = 2..4 states: the s x s table of relationships of the
// paper's stated extension, Sec. 7 item 2, with the Sec. 2.1 definitions
// taken over the state set {0, .., s-1}).
//
// Input layout: one byte per field, `ld` bytes per row; bits 2a and 2a+1 of
// the byte hold rho(a), the copies of state a among the entry's two alleles.
// A genotype's counts sum to 2; the byte 0 is a missing entry, which gives
// rho = 0 in every state and so drops out of every tally.  Bytes past n_f
// are padding and are turned into 0 before use.
//
// The tally is s^2 GEMMs C(a,b) = R_a R_b^T over one int8 plane per state,
// R_a[i][q] = rho_{i,q}(a).  A lane of the 16x16x64 operand holds 16 k-values
// of one row; here they are the row's 16 bytes at 16 g of each 64-field
// step, and state a's plane of 4 fields is (w >> 2a) & 0x03030303: one or
// two VALU ops, no table lookup.  A wave owns (16 WM) x (16 WN) pairs with
// s^2 accumulator sets; WM, WN are chosen per s to keep the accumulators at
// 128-144 registers (s = 2: 4 x 2, s = 3: 2 x 2, s = 4: 2 x 1), two waves per
// SIMD.  Workgroups of 2 x 2 waves cover (32 WM) x (32 WN); the triangle is
// walked in (32 WM)-square tiles split into WM / WN column parts.
//
// Epilogue: m_ij = sum_ab C(a,b) / 4; CCC(a,b) = C/(4 m_ij) * w_i(a) * w_j(b)
// with the per-vector factors w(a) = 1 - gamma n(a)/(2m) computed once per
// row and column, and the quotient corrected to the rounded C/(4 m_ij).
//
// fp4 form (n_f <= kF4MaxFields): the 16x16x128 scaled MFMA with e2m1 operands
// rho(a)/2 (values 0, 1/2, 1; sums of quarter-multiples at most n_f, exact in
// fp32).  A lane holds 32 fields of a row per MFMA step: the 32 bytes at 32 g
// of each 128-field step, as two 16-byte pieces; operand register r takes
// state a of piece 0's word r (4 fields) in its low nibbles and of piece 1's
// word r in its high nibbles, 3-4 VALU ops per 8 fields.  The next step's
// pieces travel from memory into the wave's LDS stage while the current step
// is multiplied.
#include <type_traits>

#include "tile2.h"

namespace ccc {

namespace {

constexpr unsigned kLow2 = 0x03030303u;

// Counts row of the multi-allelic layout: (n(0), n(1), n(2), n(3), m, 0, 0, 0).
constexpr int kMultiCountStride = 8;

// 16 bytes (16 fields) of a row at byte offset ob (a multiple of 16); bytes
// at or past n_f come back as 0 (missing), and a piece wholly past n_f is
// not read, so a row is never read past n_f rounded up to 16 bytes.
__device__ __forceinline__ u4 load_bytes16(const uint8_t* __restrict__ row, int64_t ob,
                                           int64_t n_f) {
  u4 w = u4{0u, 0u, 0u, 0u};
  if (ob >= n_f) return w;
  w = *reinterpret_cast<const u4*>(row + ob);
  if (ob + 16 > n_f) {
    const int64_t valid = n_f - ob;  // 1..15 bytes
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t vb = valid - 4 * t;
      const unsigned keep = vb >= 4 ? 0xFFFFFFFFu : (vb <= 0 ? 0u : (1u << (8 * vb)) - 1u);
      w[t] &= keep;
    }
  }
  return w;
}

// State a's int8 plane of 16 fields.
__device__ __forceinline__ v4i state_plane(const u4& w, int a) {
  return v4i{(int)((w.x >> (2 * a)) & kLow2), (int)((w.y >> (2 * a)) & kLow2),
             (int)((w.z >> (2 * a)) & kLow2), (int)((w.w >> (2 * a)) & kLow2)};
}

// State a of 8 fields (word r of two pieces) as 8 e2m1 nibbles.
template <int A>
__device__ __forceinline__ unsigned state_nibbles(unsigned lo, unsigned hi) {
  constexpr unsigned kLo = 0x03030303u, kHi = 0x30303030u;
  const unsigned l = (lo >> (2 * A)) & kLo;
  const unsigned h = (4 - 2 * A >= 0) ? (hi << (4 - 2 * A)) : (hi >> (2 * A - 4));
  return (h & kHi) | l;
}

template <int A>
__device__ __forceinline__ v8i state_operand_f4(const u4& p0, const u4& p1) {
  return v8i{(int)state_nibbles<A>(p0.x, p1.x), (int)state_nibbles<A>(p0.y, p1.y),
             (int)state_nibbles<A>(p0.z, p1.z), (int)state_nibbles<A>(p0.w, p1.w), 0, 0, 0, 0};
}

template <int S>
__device__ __forceinline__ void state_operands_f4(const u4& p0, const u4& p1, v8i (&o)[S]) {
  o[0] = state_operand_f4<0>(p0, p1);
  o[1] = state_operand_f4<1>(p0, p1);
  if constexpr (S > 2) o[2] = state_operand_f4<2>(p0, p1);
  if constexpr (S > 3) o[3] = state_operand_f4<3>(p0, p1);
}

// Sum of the 4 bytes of x when each is at most 63.
__device__ __forceinline__ unsigned byte_sum(unsigned x) { return (x * 0x01010101u) >> 24; }

// 1-way counts: one wave per row, 16-byte pieces with a 1 KiB lane stride.
// m = (sum of the state counts) / 2, the present fields of a valid row.
__global__ __launch_bounds__(256) void multi_count_kernel(const uint8_t* __restrict__ v,
                                                          int64_t ld, int64_t n, int64_t n_f,
                                                          int s, int32_t* __restrict__ counts) {
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int lane = threadIdx.x & 63;
  const uint8_t* r = v + row * ld;
  unsigned c[4] = {0u, 0u, 0u, 0u};
  for (int64_t ob = (int64_t)lane * 16; ob < n_f; ob += 64 * 16) {
    const u4 w = load_bytes16(r, ob, n_f);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      if (a < s) {
        c[a] += byte_sum((w.x >> (2 * a)) & kLow2) + byte_sum((w.y >> (2 * a)) & kLow2) +
                byte_sum((w.z >> (2 * a)) & kLow2) + byte_sum((w.w >> (2 * a)) & kLow2);
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int a = 0; a < 4; ++a) c[a] += __shfl_xor(c[a], off);
  if (lane == 0) {
    v4i* o = reinterpret_cast<v4i*>(counts + kMultiCountStride * row);
    o[0] = v4i{(int)c[0], (int)c[1], (int)c[2], (int)c[3]};
    o[1] = v4i{(int)((c[0] + c[1] + c[2] + c[3]) >> 1), 0, 0, 0};
  }
}

struct Multi2Args {
  const uint8_t* v;
  int64_t ld, n, n_f;
  int32_t* tables;  // [pairs][S*S] or null
  double* ccc;      // [pairs][S*S] or null
  const int32_t* counts;
  double gamma;
};

// Factors w(a) = 1 - gamma n(a)/(2m) of row x (clamped into range).
template <int S>
__device__ __forceinline__ void multi_factors(const Multi2Args& a, int64_t x, double (&w)[S]) {
  const int32_t* c = a.counts + kMultiCountStride * (x < a.n ? x : a.n - 1);
#pragma unroll
  for (int s = 0; s < S; ++s) w[s] = one_minus_gf(c[s], c[4], a.gamma);
}

// Store the table t and its CCC at pair p.
template <int S>
__device__ __forceinline__ void multi_store(const Multi2Args& a, int64_t p,
                                            const int (&t)[S * S], const double (&wi)[S],
                                            const double (&wj)[S]) {
#pragma clang fp contract(off)
  constexpr int SS = S * S;
  if (a.tables) {
    int32_t* o = a.tables + SS * p;
    if constexpr (SS % 4 == 0) {
#pragma unroll
      for (int x = 0; x < SS; x += 4)
        *reinterpret_cast<v4i*>(o + x) = v4i{t[x], t[x + 1], t[x + 2], t[x + 3]};
    } else {
#pragma unroll
      for (int x = 0; x < SS; ++x) o[x] = t[x];
    }
  }
  if (a.ccc) {
    int sum = 0;
#pragma unroll
    for (int x = 0; x < SS; ++x) sum += t[x];
    const int m_ij = sum >> 2;  // fields where both are present
    double r[SS];
    if (m_ij > 0) {
      const double den = 4.0 * (double)m_ij, y = 1.0 / den;
#pragma unroll
      for (int x = 0; x < SS; ++x)
        r[x] = quot_rn((double)t[x], den, y) * wi[x / S] * wj[x % S];
    } else {
#pragma unroll
      for (int x = 0; x < SS; ++x) r[x] = 0.0;
    }
    double* o = a.ccc + SS * p;
    if constexpr (SS % 2 == 0) {
#pragma unroll
      for (int x = 0; x < SS; x += 2)
        *reinterpret_cast<double2*>(o + x) = double2{r[x], r[x + 1]};
    } else {
#pragma unroll
      for (int x = 0; x < SS; ++x) o[x] = r[x];
    }
  }
}

template <int S, bool F4 = false>
struct MultiShape;
template <>
struct MultiShape<2, false> {
  static constexpr int WM = 4, WN = 2, U = 1;
};
// fp4, s = 2: the 4 x 2 tile needs more than the 256 registers of two waves
// per SIMD once its operands are nibbles, so it takes the s = 3 shape
template <>
struct MultiShape<2, true> {
  static constexpr int WM = 2, WN = 2;
};
template <int S>
struct MultiShape<S, true> : MultiShape<S, false> {};
template <>
struct MultiShape<3, false> {
  static constexpr int WM = 2, WN = 2, U = 1;
};
template <>
struct MultiShape<4, false> {
  static constexpr int WM = 2, WN = 1, U = 2;
};

template <int S, bool F4>
__global__ __launch_bounds__(256, 2) void multi2_kernel(Multi2Args a, int64_t tiles_side) {
  constexpr int WM = MultiShape<S, F4>::WM, WN = MultiShape<S, F4>::WN;
  constexpr int BM = 32 * WM, BN = 32 * WN, PARTS = BM / BN;
  static_assert(BM % BN == 0, "square tiles split into whole column parts");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, rl = lane & 15;
  // XCD-contiguous runs of squares in strip order: a run shares row and
  // column blocks in one L2
  const int64_t b = xcd_unit(blockIdx.x, gridDim.x);
  int64_t sq_i, sq_j;
  strip_square(b / PARTS, tiles_side, 0, tiles_side, sq_i, sq_j);
  const int64_t row0 = sq_i * BM + (wave & 1) * 16 * WM;
  const int64_t col0 = (sq_j * PARTS + b % PARTS) * BN + (wave >> 1) * 16 * WN;
  // a wave with no pair i < j does no MFMA work (in the fp4 form it still
  // shares the workgroup's loads and barriers)
  const bool active = !(row0 >= a.n || col0 >= a.n || row0 >= col0 + 16 * WN - 1);
  if (!F4 && !active) return;

  const uint8_t* pa[WM];
  const uint8_t* pb[WN];
#pragma unroll
  for (int m = 0; m < WM; ++m) {
    const int64_t r = row0 + 16 * m + rl;
    pa[m] = a.v + (r < a.n ? r : a.n - 1) * a.ld + 16 * g;
  }
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    const int64_t r = col0 + 16 * n + rl;
    pb[n] = a.v + (r < a.n ? r : a.n - 1) * a.ld + 16 * g;
  }

  using Acc = std::conditional_t<F4, v4f, v4i>;
  Acc acc[WM][WN][S * S];
#pragma unroll
  for (int m = 0; m < WM; ++m)
#pragma unroll
    for (int n = 0; n < WN; ++n)
#pragma unroll
      for (int x = 0; x < S * S; ++x) acc[m][n][x] = Acc{0, 0, 0, 0};

  if constexpr (F4) {
    // fp4: 128-field steps; lane group g holds bytes [32 g, 32 g + 32) of each
    // row's step as two 16-byte pieces.  The workgroup's 2 WM + 2 WN row
    // blocks are copied into LDS once per step (the four waves share the
    // 2 (2 WM + 2 WN) piece copies), double-buffered, one barrier per step;
    // each wave then reads its own WM + WN blocks from there.
    constexpr int NB = 2 * WM + 2 * WN, ND = 2 * NB, DPW = ND / 4;
    static_assert(ND % 4 == 0, "the piece copies split evenly over the waves");
    __shared__ u4 stage[2][ND][64];  // piece 2 blk + h; A blocks first, then B
    const int64_t I0 = sq_i * BM, J0 = (sq_j * PARTS + b % PARTS) * BN;
    // each copy: a wave-uniform base (the block's first row, clamped; read
    // from lane 0 so the compiler knows it is uniform) plus a fixed 32-bit
    // lane offset
    const int wu = __builtin_amdgcn_readfirstlane(wave);
    const uint8_t* base[DPW];
    uint32_t off[DPW];
#pragma unroll
    for (int q = 0; q < DPW; ++q) {
      const int d = wu + 4 * q, blk = d >> 1, h = d & 1;
      const int64_t r0 = blk < 2 * WM ? I0 + 16 * blk : J0 + 16 * (blk - 2 * WM);
      const int64_t rf = r0 < a.n ? r0 : a.n - 1, r = r0 + rl < a.n ? r0 + rl : a.n - 1;
      const uint64_t bp = (uint64_t)(a.v + rf * a.ld);
      base[q] = (const uint8_t*)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(bp >> 32))
                                  << 32) |
                                 (uint32_t)__builtin_amdgcn_readfirstlane((int)bp));
      off[q] = (uint32_t)((r - rf) * a.ld + 32 * g + 16 * h);
    }
    const int ablk = (wave & 1) * WM, bblk = 2 * WM + (wave >> 1) * WN;
    // row(side, r, h) gives piece h of this wave's row block r of side 0 (A) or 1 (B)
    auto step = [&](auto row) {
      v8i B[WN][S];
#pragma unroll
      for (int n = 0; n < WN; ++n) state_operands_f4<S>(row(1, n, 0), row(1, n, 1), B[n]);
#pragma unroll
      for (int m = 0; m < WM; ++m) {
        v8i A[S];
        state_operands_f4<S>(row(0, m, 0), row(0, m, 1), A);
#pragma unroll
        for (int n = 0; n < WN; ++n)
#pragma unroll
          for (int x = 0; x < S * S; ++x)
            acc[m][n][x] = tile2::mfma_f4(A[x / S], B[n][x % S], acc[m][n][x]);
      }
    };
    const int64_t nfull = a.n_f / 128;
    auto issue = [&](int64_t st, int buf) {
#pragma unroll
      for (int q = 0; q < DPW; ++q)
        tile2::stage_row(base[q] + st * 128 + off[q], &stage[buf][wu + 4 * q][0]);
    };
    if (nfull > 0) issue(0, 0);
    for (int64_t st = 0; st < nfull; ++st) {
      const int buf = (int)(st & 1);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // this wave's copies landed
      __syncthreads();  // every wave's copies landed; the other buffer is no longer read
      if (st + 1 < nfull) issue(st + 1, buf ^ 1);
      if (active)
        step([&](int side, int r, int h) -> u4 {
          return stage[buf][2 * (side ? bblk + r : ablk + r) + h][lane];
        });
    }
    if (!active) return;
    if (nfull * 128 < a.n_f) {
      const int64_t kb = nfull * 128 + 32 * g;
      u4 xa[WM][2], xb[WN][2];
#pragma unroll
      for (int m = 0; m < WM; ++m)
#pragma unroll
        for (int h = 0; h < 2; ++h) xa[m][h] = load_bytes16(pa[m] - 16 * g, kb + 16 * h, a.n_f);
#pragma unroll
      for (int n = 0; n < WN; ++n)
#pragma unroll
        for (int h = 0; h < 2; ++h) xb[n][h] = load_bytes16(pb[n] - 16 * g, kb + 16 * h, a.n_f);
      step([&](int side, int r, int h) -> u4 { return side ? xb[r][h] : xa[r][h]; });
    }
  } else {

  auto step = [&](const u4 (&xa)[WM], const u4 (&xb)[WN]) {
    v4i A[WM][S], B[WN][S];
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int s = 0; s < S; ++s) A[m][s] = state_plane(xa[m], s);
#pragma unroll
    for (int n = 0; n < WN; ++n)
#pragma unroll
      for (int s = 0; s < S; ++s) B[n][s] = state_plane(xb[n], s);
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int n = 0; n < WN; ++n)
#pragma unroll
        for (int x = 0; x < S * S; ++x)
          acc[m][n][x] = __builtin_amdgcn_mfma_i32_16x16x64_i8(A[m][x / S], B[n][x % S],
                                                               acc[m][n][x], 0, 0, 0);
  };

  // 64-field steps in groups of U: plain 16-byte loads of the next group are
  // issued before the current group's MFMAs while the steps are whole; then
  // the whole steps left over, and one masked step for the tail.
  constexpr int U = MultiShape<S, F4>::U;
  const int64_t nfull = a.n_f / 64, ngroups = nfull / U;
  u4 ca[U][WM], cb[U][WN];
  auto load_group = [&](int64_t st0, u4 (&xa)[U][WM], u4 (&xb)[U][WN]) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int m = 0; m < WM; ++m) xa[u][m] = *reinterpret_cast<const u4*>(pa[m] + (st0 + u) * 64);
#pragma unroll
      for (int n = 0; n < WN; ++n) xb[u][n] = *reinterpret_cast<const u4*>(pb[n] + (st0 + u) * 64);
    }
  };
  if (ngroups > 0) load_group(0, ca, cb);
  for (int64_t gr = 0; gr < ngroups; ++gr) {
    u4 na[U][WM], nb[U][WN];
    if (gr + 1 < ngroups) load_group((gr + 1) * U, na, nb);
#pragma unroll
    for (int u = 0; u < U; ++u) step(ca[u], cb[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
#pragma unroll
      for (int m = 0; m < WM; ++m) ca[u][m] = na[u][m];
#pragma unroll
      for (int n = 0; n < WN; ++n) cb[u][n] = nb[u][n];
    }
  }
  for (int64_t st = ngroups * U; st < nfull; ++st) {
#pragma unroll
    for (int m = 0; m < WM; ++m) ca[0][m] = *reinterpret_cast<const u4*>(pa[m] + st * 64);
#pragma unroll
    for (int n = 0; n < WN; ++n) cb[0][n] = *reinterpret_cast<const u4*>(pb[n] + st * 64);
    step(ca[0], cb[0]);
  }
  if (nfull * 64 < a.n_f) {
    const int64_t kb = nfull * 64 + 16 * g;
#pragma unroll
    for (int m = 0; m < WM; ++m) ca[0][m] = load_bytes16(pa[m] - 16 * g, kb, a.n_f);
#pragma unroll
    for (int n = 0; n < WN; ++n) cb[0][n] = load_bytes16(pb[n] - 16 * g, kb, a.n_f);
    step(ca[0], cb[0]);
  }

  }

  // Epilogue: lane holds rows 4g + e of column rl of each 16x16 block.
  const bool want_w = a.ccc != nullptr;
#pragma unroll
  for (int n = 0; n < WN; ++n) {
    const int64_t j = col0 + 16 * n + rl;
    double wj[S];
    if (want_w) multi_factors<S>(a, j, wj);
#pragma unroll
    for (int m = 0; m < WM; ++m)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t i = row0 + 16 * m + 4 * g + e;
        if (!(i < j && j < a.n)) continue;
        double wi[S];
        if (want_w) multi_factors<S>(a, i, wi);
        int t[S * S];
#pragma unroll
        for (int x = 0; x < S * S; ++x) {
          if constexpr (F4)
            t[x] = tile2::f4_count(acc[m][n][x][e]);
          else
            t[x] = acc[m][n][x][e];
        }
        multi_store<S>(a, pair_index(a.n, i, j), t, wi, wj);
      }
  }
}

template <int S, bool F4>
hipError_t launch_multi2_shape(const Multi2Args& a, hipStream_t stream) {
  constexpr int BM = 32 * MultiShape<S, F4>::WM, BN = 32 * MultiShape<S, F4>::WN;
  const int64_t T = (a.n + BM - 1) / BM;
  const int64_t ntiles = (BM / BN) * (T * (T + 1) / 2);
  if (ntiles <= 0) return hipSuccess;
  if (ntiles > 0x7FFFFFFF) return hipErrorInvalidValue;
  timing_begin("multi2", stream);
  hipLaunchKernelGGL((multi2_kernel<S, F4>), dim3((unsigned)ntiles), dim3(256), 0, stream, a, T);
  timing_end(stream);
  return hipGetLastError();
}

template <int S>
hipError_t launch_multi2_s(const Multi2Args& a, int f4, hipStream_t stream) {
  return f4 ? launch_multi2_shape<S, true>(a, stream) : launch_multi2_shape<S, false>(a, stream);
}

}  // namespace

hipError_t launch_multi_count(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int s,
                              int32_t* counts, hipStream_t stream) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(multi_count_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, v,
                     ld, n, n_f, s, counts);
  return hipGetLastError();
}

hipError_t launch_multi2(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int s,
                         int32_t* tables, double* ccc, const int32_t* counts, double gamma,
                         int f4, hipStream_t stream) {
  Multi2Args a{v, ld, n, n_f, tables, ccc, counts, gamma};
  switch (s) {
    case 2: return launch_multi2_s<2>(a, f4, stream);
    case 3: return launch_multi2_s<3>(a, f4, stream);
    case 4: return launch_multi2_s<4>(a, f4, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ccc
