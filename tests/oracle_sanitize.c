/* Drives every oracle entry point on small ragged inputs (garbage padding,
 * missing codes) under AddressSanitizer and UndefinedBehaviorSanitizer.  Built
 * and run by test_oracle_sanitizers.py; includes the oracle source directly.
 * Exit status 0 when every internal consistency check holds. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/ccc_oracle.c"

static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) {
  st ^= st << 13;
  st ^= st >> 7;
  st ^= st << 17;
  return st;
}

#define CHECK(c)                                                       \
  do {                                                                 \
    if (!(c)) {                                                        \
      fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c);     \
      return 1;                                                        \
    }                                                                  \
  } while (0)

static int run(int64_t n, int64_t n_f, int64_t ld) {
  uint8_t* v = malloc((size_t)(n * ld));
  for (int64_t i = 0; i < n * ld; ++i) v[i] = (uint8_t)next();
  int64_t* cnt = malloc(sizeof(int64_t) * 3 * n);
  oracle_counts1(v, n, n_f, ld, cnt);
  int64_t np = n * (n - 1) / 2;
  int64_t* t2 = malloc(sizeof(int64_t) * 4 * (np ? np : 1));
  double* c2 = malloc(sizeof(double) * 4 * (np ? np : 1));
  if (n >= 2) oracle_2way_rows(v, n, n_f, ld, 0, n - 1, cnt, 2.0 / 3.0, t2, c2);
  for (int64_t p = 0; p < np; ++p) {
    int64_t s = t2[4 * p] + t2[4 * p + 1] + t2[4 * p + 2] + t2[4 * p + 3];
    CHECK(s % 4 == 0 && s <= 4 * n_f);
    for (int e = 0; e < 4; ++e) CHECK(c2[4 * p + e] >= 0.0 && c2[4 * p + e] <= 1.0);
  }
  /* the block of the set with itself contains the triangle */
  int64_t* tb = malloc(sizeof(int64_t) * 4 * n * n);
  double* cb = malloc(sizeof(double) * 4 * n * n);
  oracle_block_rows(v, ld, v, n, ld, n_f, 0, n, cnt, cnt, 2.0 / 3.0, tb, cb);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = i + 1; j < n; ++j) {
      int64_t p = oracle_pair_index(n, i, j);
      for (int e = 0; e < 4; ++e) CHECK(tb[(i * n + j) * 4 + e] == t2[4 * p + e]);
    }
  /* explicit lists */
  int64_t ia[8], jb[8];
  for (int k = 0; k < 8; ++k) {
    ia[k] = (int64_t)(next() % (uint64_t)n);
    jb[k] = (int64_t)(next() % (uint64_t)n);
  }
  int64_t tl[32];
  double cl[32];
  oracle_2way_list(v, ld, v, ld, n_f, ia, jb, 8, cnt, cnt, 2.0 / 3.0, tl, cl);
  for (int k = 0; k < 8; ++k)
    for (int e = 0; e < 4; ++e) CHECK(tl[4 * k + e] == tb[(ia[k] * n + jb[k]) * 4 + e]);
  /* 3-way */
  int64_t nt = n >= 3 ? n * (n - 1) * (n - 2) / 6 : 0;
  int64_t* t3 = malloc(sizeof(int64_t) * 8 * (nt ? nt : 1));
  double* c3 = malloc(sizeof(double) * 8 * (nt ? nt : 1));
  if (n >= 3) oracle_3way_rows(v, n, n_f, ld, 0, n - 2, cnt, 2.0 / 3.0, t3, c3);
  if (n >= 3) {
    int64_t ii[4], jj[4], kk[4];
    for (int k = 0; k < 4; ++k) { /* random distinct sorted triples */
      int64_t x = (int64_t)(next() % (uint64_t)(n - 2));
      int64_t y = x + 1 + (int64_t)(next() % (uint64_t)(n - 2 - x));
      int64_t z = y + 1 + (int64_t)(next() % (uint64_t)(n - 1 - y));
      ii[k] = x; jj[k] = y; kk[k] = z;
    }
    int64_t t3l[32];
    double c3l[32];
    oracle_3way_list(v, ld, n_f, ii, jj, kk, 4, cnt, 2.0 / 3.0, t3l, c3l);
    for (int k = 0; k < 4; ++k) {
      int64_t p = oracle_triple_index(n, ii[k], jj[k], kk[k]);
      for (int e = 0; e < 8; ++e) CHECK(t3l[8 * k + e] == t3[8 * p + e]);
    }
  }
  /* checksums */
  uint64_t* w = malloc(sizeof(uint64_t) * 3 * n);
  for (int64_t i = 0; i < 3 * n; ++i) w[i] = next() % ((1ull << 61) - 1);
  int32_t* t2i = malloc(sizeof(int32_t) * 4 * (np ? np : 1));
  for (int64_t i = 0; i < 4 * np; ++i) t2i[i] = (int32_t)t2[i];
  uint64_t fa[4], fb[4];
  oracle_fp2_from_input(v, n, n_f, ld, w, w + n, fa);
  oracle_fp2_from_tables(t2i, n, w, w + n, fb);
  for (int e = 0; e < 4; ++e) CHECK(fa[e] == fb[e]);
  int32_t* tbi = malloc(sizeof(int32_t) * 4 * n * n);
  for (int64_t i = 0; i < 4 * n * n; ++i) tbi[i] = (int32_t)tb[i];
  oracle_fpb_from_input(v, n, ld, v, n, ld, n_f, w, w + n, fa);
  oracle_fpb_from_tables(tbi, n, n, w, w + n, fb);
  for (int e = 0; e < 4; ++e) CHECK(fa[e] == fb[e]);
  if (n >= 3) {
    int32_t* t3i = malloc(sizeof(int32_t) * 8 * nt);
    for (int64_t i = 0; i < 8 * nt; ++i) t3i[i] = (int32_t)t3[i];
    uint64_t ga[8], gb[8];
    oracle_fp3_from_input(v, n, n_f, ld, w, w + n, w + 2 * n, ga);
    oracle_fp3_from_tables(t3i, n, 0, nt, w, w + n, w + 2 * n, gb);
    for (int e = 0; e < 8; ++e) CHECK(ga[e] == gb[e]);
    free(t3i);
  }
  free(v); free(cnt); free(t2); free(c2); free(tb); free(cb); free(t3); free(c3); free(w);
  free(t2i); free(tbi);
  return 0;
}

/* Multi-allelic entry points on random bytes (valid genotypes, missing bytes
   and arbitrary bytes alike) with s = 2..4 states. */
static int run_multi(int64_t n, int64_t n_f, int64_t ld, int s) {
  uint8_t* v = malloc((size_t)(n * ld));
  for (int64_t i = 0; i < n * ld; ++i) v[i] = (uint8_t)next();
  (void)oracle_multi_invalid(v, n, n_f, ld, s);
  int64_t* cnt = malloc(sizeof(int64_t) * 5 * n);
  oracle_multi_counts1(v, n, n_f, ld, s, cnt);
  const int ss = s * s;
  int64_t np = n * (n - 1) / 2;
  int64_t* t = malloc(sizeof(int64_t) * ss * (np ? np : 1));
  double* c = malloc(sizeof(double) * ss * (np ? np : 1));
  int32_t* ti = malloc(sizeof(int32_t) * ss * (np ? np : 1));
  if (n >= 2) oracle_multi_2way_rows(v, n, n_f, ld, s, 0, n - 1, cnt, 2.0 / 3.0, t, c);
  for (int64_t p = 0; p < np; ++p) {
    int64_t sum = 0;
    for (int e = 0; e < ss; ++e) {
      sum += t[p * ss + e];
      CHECK(c[p * ss + e] >= 0.0 && c[p * ss + e] <= 1.0);
      ti[p * ss + e] = (int32_t)t[p * ss + e];
    }
    CHECK(sum % 4 == 0 && sum <= 4 * n_f);
  }
  int64_t ia[4] = {0, 0, n - 1, n / 2}, jb[4] = {n - 1, 0, 0, n / 2};
  int64_t tl[4 * 16];
  double cl[4 * 16];
  oracle_multi_2way_list(v, ld, n_f, s, ia, jb, 4, cnt, 2.0 / 3.0, tl, cl);
  uint64_t* w = malloc(sizeof(uint64_t) * 2 * n);
  for (int64_t i = 0; i < 2 * n; ++i) w[i] = next() % P61;
  uint64_t fa[16], fb[16];
  oracle_multi_fp2_from_input(v, n, n_f, ld, s, w, w + n, fa);
  oracle_multi_fp2_from_tables(ti, n, s, w, w + n, fb);
  for (int e = 0; e < ss; ++e) CHECK(fa[e] == fb[e]);
  free(v); free(cnt); free(t); free(c); free(ti); free(w);
  return 0;
}

int main(void) {
  const int64_t mshapes[][3] = {{2, 1, 16}, {3, 17, 32}, {8, 100, 112}, {11, 0, 16}};
  for (size_t k = 0; k < sizeof(mshapes) / sizeof(mshapes[0]); ++k)
    for (int s = 2; s <= 4; ++s)
      if (run_multi(mshapes[k][0], mshapes[k][1], mshapes[k][2], s)) {
        fprintf(stderr, "multi shape %zu s %d failed\n", k, s);
        return 1;
      }
  const int64_t shapes[][3] = {{2, 1, 16}, {3, 5, 16}, {7, 65, 32}, {12, 257, 80}, {5, 0, 16},
                               {9, 300, 96}};
  for (size_t s = 0; s < sizeof(shapes) / sizeof(shapes[0]); ++s) {
    if (run(shapes[s][0], shapes[s][1], shapes[s][2])) {
      fprintf(stderr, "shape %zu failed\n", s);
      return 1;
    }
  }
  printf("oracle sanitizer run ok\n");
  return 0;
}
