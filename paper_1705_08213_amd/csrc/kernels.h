// kernels.h -- host-side launchers of the CCC kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace ccc {

// Threshold selection: instead of dense tables, keep every pair (triple)
// with a CCC value >= threshold as (index, CCC values[, table]) records at
// slots taken from a device counter; slots past `cap` are counted, not stored.
struct Select {
  unsigned long long* count;  // device counter (zeroed before the tally kernel)
  int64_t cap;
  double threshold;
  int64_t* index;             // [cap] pair (triple) index
  double* ccc;                // [cap][4] or [cap][8]
  int32_t* tables;            // [cap][4] or [cap][8], may be null
};

// Arguments of one 2-way tally launch: either the upper triangle (i < j) of
// one vector set (tri = 1, va == vb) or the full rectangle A x B (tri = 0).
struct Pair2Args {
  const uint8_t* va;
  int64_t lda, n_a;
  const uint8_t* vb;
  int64_t ldb, n_b;
  int64_t n_f;
  int f4;                     // MFMA operands: fp4 (1, needs n_f <= kF4MaxFields) or int8 (0)
  int tri;
  int accumulate;             // tables += result (rectangle only)
  int32_t* tables;            // may be null when ccc is set
  double* ccc;                // may be null
  const int32_t* counts_a;    // [n_a][4]
  const int32_t* counts_b;    // [n_b][4]
  // this call's own 1-way counts of its n_f fields (the same arrays as
  // counts_a / counts_b unless accumulating, where those are running totals)
  const int32_t* chunk_a;
  const int32_t* chunk_b;
  double gamma;
  // rows of A whose pairs are produced; pair (i, j) goes to entry p(i,j) - p_base
  int64_t row_begin, row_end;
  int64_t p_base;
  int64_t sq_offset;          // first square tile of the row range (triangle)
  Select sel;                 // threshold selection (sel.count != null) instead of dense output
  // Device flag (one int) that launch_mfma2 sets to 1 when every row of A and
  // B has all n_f fields present, 0 otherwise; null: no such check (each
  // workgroup tile votes for itself).  Only for calls that do not accumulate.
  int* complete;
};

// Largest n_f for which the MFMA kernels may take fp4 operands (their fp32
// sums of quarter-multiples, at most n_f, stay exact); int8 beyond.
constexpr int64_t kF4MaxFields = int64_t(1) << 22;

// Row tile of the 3-way work units (one-j units and the complete-data
// kernel's runs), and of the fp4 general kernel's runs of middle vectors.
constexpr int64_t kUnitTile = 64;
constexpr int64_t kRunTile = 32;

// Tetrahedral work units of the 3-way kernels.  Rows are cut into b-row
// tiles; a unit is (I tile it, K tile kt, middle vectors j .. j + run - 1)
// with it <= kt and covers every triple i < j < k with i in tile it (and in
// the staged range [i_begin, i_end)) and k in tile kt, for its run of
// consecutive middle vectors (cut from the pair's j range; the last run of
// a pair may be shorter).  Units are ordered by tile pair (it major, then
// kt) and, within a pair, by j: consecutive units share both row tiles, so
// a run of them on one XCD reads the tiles from its L2 once.
struct UnitGrid {
  int64_t n, b, i_begin, i_end;
  int64_t it0, it1;  // I tiles [it0, it1)
  int64_t nt;        // tiles of all n rows
  int64_t run;       // middle vectors per unit
};

__host__ __device__ __forceinline__ UnitGrid unit_grid(int64_t n, int64_t b, int64_t i_begin,
                                                       int64_t i_end, int64_t run = 1) {
  UnitGrid g;
  g.n = n;
  g.b = b;
  g.run = run;
  g.i_begin = i_begin;
  g.i_end = i_end;
  g.it0 = i_begin / b;
  g.it1 = i_end > i_begin ? (i_end + b - 1) / b : g.it0;
  g.nt = (n + b - 1) / b;
  return g;
}

// Number of tile pairs (it, kt), it0 <= it < it1, it <= kt < nt.
__host__ __device__ __forceinline__ int64_t grid_pairs(const UnitGrid& g) {
  int64_t p = 0;
  if (g.it1 > g.it0) {
    const int64_t rows = g.it1 - g.it0;  // sum of (nt - it) over the I tiles
    p = rows * g.nt - (g.it1 * (g.it1 - 1) / 2 - g.it0 * (g.it0 - 1) / 2);
  }
  return p;
}

// First pair index of I tile it.
__host__ __device__ __forceinline__ int64_t grid_row_start(const UnitGrid& g, int64_t it) {
  return (it - g.it0) * g.nt - (it * (it - 1) / 2 - g.it0 * (g.it0 - 1) / 2);
}

// Middle vectors [jlo, jhi) of tile pair (it, kt): j above the first row of
// tile it in the range, and below the last row of tile kt.
__host__ __device__ __forceinline__ void pair_j_range(const UnitGrid& g, int64_t it, int64_t kt,
                                                      int64_t& jlo, int64_t& jhi) {
  jlo = (it * g.b > g.i_begin ? it * g.b : g.i_begin) + 1;
  jhi = (kt + 1) * g.b - 1;
  if (jhi > g.n - 1) jhi = g.n - 1;
  if (jhi < jlo) jhi = jlo;
}

// Units of tile pair (it, kt): its j range in runs of g.run.
__host__ __device__ __forceinline__ int64_t pair_units(const UnitGrid& g, int64_t it,
                                                       int64_t kt) {
  int64_t jlo, jhi;
  pair_j_range(g, it, kt, jlo, jhi);
  return (jhi - jlo + g.run - 1) / g.run;
}

// Tile pair of pair index p.
__host__ __device__ __forceinline__ void pair_tiles(const UnitGrid& g, int64_t p, int64_t& it,
                                                    int64_t& kt) {
  int64_t lo = g.it0, hi = g.it1;  // row_start(lo) <= p < row_start(hi)
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (grid_row_start(g, mid) <= p) lo = mid; else hi = mid;
  }
  it = lo;
  kt = it + (p - grid_row_start(g, it));
}

// Unit u -> (first middle vector j of its run, I tile, K tile), given
// offs[p] = units of all pairs before p (p = 0..pairs).
__host__ __device__ __forceinline__ void unit_coords(int64_t u, const UnitGrid& g,
                                                     const int64_t* __restrict__ offs,
                                                     int64_t& j, int64_t& it, int64_t& kt) {
  int64_t lo = 0, hi = grid_pairs(g);  // offs[lo] <= u < offs[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (offs[mid] <= u) lo = mid; else hi = mid;
  }
  pair_tiles(g, lo, it, kt);
  int64_t jlo, jhi;
  pair_j_range(g, it, kt, jlo, jhi);
  j = jlo + g.run * (u - offs[lo]);
}

// Workgroup b of a grid of `count` -> unit index, so that the workgroups the
// dispatcher sends to one of the 8 XCDs (b mod 8) take one contiguous run of
// units, in order.
__host__ __device__ __forceinline__ int64_t xcd_unit(int64_t b, int64_t count) {
  const int64_t q = count >> 3, r = count & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}

// Strip order of the squares of a 2-way triangle launch, so that the
// consecutive squares an XCD has in flight (xcd_unit hands each XCD a
// contiguous run) share both their row and their column blocks: strips of
// kStripRows square rows, walked column by column, rows ascending within a
// column.  (A rectangle keeps the row-major order, which measured faster.)
constexpr int64_t kStripRows = 8;

// Triangle: square t of the squares (I, J), s0 <= I < s1, I <= J < T, in
// strips of H square rows.  A strip of h rows r0 .. r1 - 1 holds
// h (h - 1) / 2 squares in its first h - 1 columns (column r0 + c has c + 1)
// and h in each of the T - r1 + 1 columns after them; the strips before the
// last are full, so the squares before strip k number
// k A - H^2 k (k + 1) / 2 with A = H (H - 1) / 2 + H (T - s0 + 1).
__host__ __device__ inline void strip_square(int64_t t, int64_t T, int64_t s0, int64_t s1,
                                             int64_t& I, int64_t& J,
                                             int64_t H = kStripRows) {
  const int64_t nstrips = (s1 - s0 + H - 1) / H;
  const int64_t A = H * (H - 1) / 2 + H * (T - s0 + 1);
  auto before = [&](int64_t k) { return k * A - H * H * k * (k + 1) / 2; };
  const double bq = (double)A - 0.5 * (double)(H * H);
  const double disc = bq * bq - 2.0 * (double)(H * H) * (double)t;
  int64_t k = (int64_t)((bq - sqrt(disc > 0.0 ? disc : 0.0)) / (double)(H * H));
  if (k < 0) k = 0;
  if (k > nstrips - 1) k = nstrips - 1;
  while (k > 0 && before(k) > t) --k;
  while (k + 1 < nstrips && before(k + 1) <= t) ++k;
  const int64_t r0 = s0 + k * H, r1 = r0 + H < s1 ? r0 + H : s1, h = r1 - r0;
  const int64_t u = t - before(k), diag = h * (h - 1) / 2;
  if (u < diag) {  // column r0 + c holds rows r0 .. r0 + c
    int64_t c = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
    while (c > 0 && c * (c + 1) / 2 > u) --c;
    while ((c + 1) * (c + 2) / 2 <= u) ++c;
    J = r0 + c;
    I = r0 + (u - c * (c + 1) / 2);
  } else {
    J = r1 - 1 + (u - diag) / h;
    I = r0 + (u - diag) % h;
  }
}

// Arguments of one 3-way tally launch over all triples i < j < k.
struct Triple3Args {
  const uint8_t* v;
  int64_t ld, n, n_f;
  int f4;         // MFMA operands: fp4 (1, needs n_f <= kF4MaxFields) or int8 (0)
  int32_t* tables;
  double* ccc;
  const int32_t* counts;
  double gamma;
  int64_t* offs;  // workspace: tile pairs + 1 int64 (work-unit offsets per tile pair)
  // triples whose first index lies in [i_begin, i_end); triple t goes to entry t - t_base
  int64_t i_begin, i_end;
  int64_t t_base;
  Select sel;
  // Dense rho(1) Gram matrix of rows [g0, g0 + ng) (workspace), filled by the
  // MFMA launcher; null turns the complete-data path off.
  int32_t* gram;
  int64_t g0, ng;
  // Complete-data flag and the unit offsets of the run grid its kernel walks
  // (fp4 MFMA with a Gram matrix only; null: every unit votes for itself).
  // launch_mfma3 sets *complete to 1 when every row of [g0, n) has all n_f
  // fields present.
  int* complete;
  int64_t* offs_run;
  // Unit offsets of the fp4 general kernel's grid (32-row tiles, runs of
  // four middle vectors).
  int64_t* offs_gen;
};

enum Path { kPathPopcount = 1, kPathMfma = 2 };

// Kernel-shape table (tune.hip): kinds of launch, and the variant the table
// picks for a problem of n_v vectors over n_f fields (0 .. n_variants - 1).
enum TuneKind { kTuneManyMfma = 0, kTuneManyPopcount = 1, kTuneOneShot = 2 };
struct TuneChoice {
  int variant;    // tile variant, in [0, n_variants)
  int wg_per_cu;  // persistent workgroups per compute unit; 0: the launcher's default
};
TuneChoice tune_pick(int kind, int64_t n_v, int64_t n_f, int n_variants);

// Optional event timing around the main kernel of a launcher (no-ops unless
// enabled through ccc_timing_enable).
void timing_begin(const char* name, hipStream_t stream);
void timing_end(hipStream_t stream);
// A host-side duration under `name` (recorded only while timing is enabled).
void timing_host(const char* name, double ms);

hipError_t launch_count1(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int32_t* counts,
                         int accumulate, hipStream_t stream);
// count1 that also zeroes a selection counter (a kernel store, graph safe)
hipError_t launch_count1_zero(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f,
                              int32_t* counts, int accumulate, unsigned long long* zero,
                              hipStream_t stream);
hipError_t launch_pop2(const Pair2Args& a, hipStream_t stream);
hipError_t launch_mfma2(const Pair2Args& a, hipStream_t stream);
hipError_t launch_mfma3(const Triple3Args& a, hipStream_t stream);
hipError_t launch_pop3(const Triple3Args& a, hipStream_t stream);
// Multi-allelic 2-way (one byte per field, s = 2..4 states): counts are
// [n][8] = (n(0), n(1), n(2), n(3), m, 0, 0, 0); tables / ccc [pairs][s*s].
hipError_t launch_multi_count(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int s,
                              int32_t* counts, hipStream_t stream);
hipError_t launch_multi2(const uint8_t* v, int64_t ld, int64_t n, int64_t n_f, int s,
                         int32_t* tables, double* ccc, const int32_t* counts, double gamma,
                         int f4, hipStream_t stream);

}  // namespace ccc
