// Host-side check of the 3-way work-unit enumeration (UnitGrid helpers of
// the library's kernels.h, compiled for the host): for each case, tile (64,
// 32, 16 rows) and run length (1 middle vector per unit, and the runs of 4
// of the complete-data and fp4 general kernels), the units cover every triple i < j < k with i in
// [i_begin, min(i_end, n-2)) exactly once, every unit lies inside its tile
// pair, and the XCD remap of a grid is a permutation.  Also the 2-way strip order of squares (strip_square) is a
// one-to-one map onto each row range's squares.  Prints "ok <cases>" and
// exits 0, or names the first failure.
#include <stdio.h>
#include <stdlib.h>

#include <vector>

#include "../../paper_1705_08213_amd/csrc/kernels.h"

using namespace ccc;

static int fail(const char* what, long n, long ib, long ie) {
  printf("FAIL %s n=%ld i_begin=%ld i_end=%ld\n", what, n, ib, ie);
  return 1;
}

static int check(int64_t n, int64_t ib, int64_t ie, int64_t b, int64_t run) {
  const int64_t row_end = ie < n - 2 ? ie : n - 2;
  if (row_end <= ib) return 0;
  const UnitGrid g = unit_grid(n, b, ib, row_end, run);
  const int64_t P = grid_pairs(g);
  std::vector<int64_t> offs(P + 1, 0);
  for (int64_t p = 0; p < P; ++p) {
    int64_t it, kt, jlo, jhi;
    pair_tiles(g, p, it, kt);
    if (it < g.it0 || it >= g.it1 || kt < it || kt >= g.nt) return fail("pair_tiles", n, ib, ie);
    pair_j_range(g, it, kt, jlo, jhi);
    offs[p + 1] = offs[p] + (jhi - jlo + run - 1) / run;
    if (pair_units(g, it, kt) != offs[p + 1] - offs[p]) return fail("pair_units", n, ib, ie);
  }
  const int64_t U = offs[P];
  std::vector<unsigned char> seen(U, 0);
  for (int64_t w = 0; w < U; ++w) {
    const int64_t u = xcd_unit(w, U);
    if (u < 0 || u >= U || seen[u]) return fail("xcd_unit", n, ib, ie);
    seen[u] = 1;
  }
  // cover[i][j][k] as a flat count over the staged triples
  std::vector<unsigned char> cover((size_t)n * n * n, 0);
  for (int64_t u = 0; u < U; ++u) {
    int64_t j0, it, kt, jlo, jhi;
    unit_coords(u, g, offs.data(), j0, it, kt);
    pair_j_range(g, it, kt, jlo, jhi);
    if (j0 < jlo || j0 >= jhi || j0 < 1 || j0 > n - 2 || (j0 - jlo) % run)
      return fail("unit_coords", n, ib, ie);
    for (int64_t j = j0; j < j0 + run && j < jhi; ++j)
      for (int64_t i = it * b; i < (it + 1) * b && i < j; ++i) {
        if (i < ib || i >= row_end) continue;
        for (int64_t k = kt * b; k < (kt + 1) * b && k < n; ++k)
          if (k > j) ++cover[((size_t)i * n + j) * n + k];
      }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j)
      for (int64_t k = j + 1; k < n; ++k) {
        const int want = (i >= ib && i < row_end) ? 1 : 0;
        if (cover[((size_t)i * n + j) * n + k] != want) return fail("coverage", n, ib, ie);
      }
  return 0;
}

// The 2-way strip order of squares (strip_square): for a triangle of T
// square rows and a row range [s0, s1), squares 0 .. count - 1 map one to
// one onto the squares (I, J) with s0 <= I < s1 and I <= J < T.
static int check_strips(int64_t T, int64_t s0, int64_t s1) {
  const int64_t cnt = s1 * T - s1 * (s1 - 1) / 2 - (s0 * T - s0 * (s0 - 1) / 2);
  std::vector<unsigned char> seen(T * T, 0);
  for (int64_t t = 0; t < cnt; ++t) {
    int64_t I, J;
    strip_square(t, T, s0, s1, I, J);
    if (I < s0 || I >= s1 || J < I || J >= T || seen[I * T + J]) {
      printf("FAIL strip_square T=%ld s0=%ld s1=%ld t=%ld\n", (long)T, (long)s0, (long)s1, (long)t);
      return 1;
    }
    seen[I * T + J] = 1;
  }
  return 0;
}

int main() {
  const long cases[][3] = {{3, 0, 3},      {4, 0, 4},      {5, 0, 5},     {64, 0, 64},
                           {65, 0, 65},    {66, 0, 66},    {130, 0, 130}, {150, 5, 64},
                           {150, 64, 70},  {150, 70, 129}, {150, 129, 150}, {90, 0, 5},
                           {90, 88, 90},   {200, 63, 65},  {200, 127, 128}, {197, 0, 197}};
  int count = 0;
  for (int64_t run : {1, 4})
    for (const auto& c : cases) {
      if (check(c[0], c[1], c[2], 64, run) || check(c[0], c[1], c[2], 32, run)) return 1;
      count += 2;
    }
  srand(7);
  for (int r = 0; r < 40; ++r) {
    const long n = 3 + rand() % 180, ib = rand() % (n + 1), ie = ib + rand() % (n + 1 - ib);
    const long b = (r % 3 == 0) ? 64 : (r % 3 == 1 ? 32 : 16);
    if (check(n, ib, ie, b, (r & 2) ? 4 : 1)) return 1;
    ++count;
  }
  for (int64_t T = 1; T <= 40; ++T)  // every row range of small triangles
    for (int64_t s0 = 0; s0 < T; ++s0)
      for (int64_t s1 = s0 + 1; s1 <= T; ++s1) {
        if (check_strips(T, s0, s1)) return 1;
        ++count;
      }
  if (check_strips(256, 0, 256) || check_strips(700, 93, 611)) return 1;  // the c2 shape, a ragged range
  count += 2;
  printf("ok %d\n", count);
  return 0;
}
