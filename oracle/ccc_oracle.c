/*
 * ccc_oracle.c -- plain CPU oracle for the Custom Correlation Coefficient
 * tallies (Joubert et al., "Parallel Accelerated Custom Correlation
 * Coefficient Calculations for Genomics Applications").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is used by the tests, by the smoke
 * check and by the benchmark's CPU-baseline leg; the GPU library neither links
 * nor calls it, and it shares no code with the GPU library.
 *
 * Everything here is the definition written out as direct loops over vectors
 * and fields, with int64 tallies and double arithmetic:
 *
 *   rho_{i,q}(a)  = number of the two alleles of entry v_{i,q} equal to a
 *                                                  (Sec. 2.1, before Eq. (1))
 *   f_i(a)        = sum_q rho_{i,q}(a) / (2 m_i)            (Sec. 2.1, Eq. (1))
 *   C_ij(a,b)     = sum_q rho_{i,q}(a) rho_{j,q}(b)         (Sec. 2.1, Eq. (2))
 *   f_ij(a,b)     = C_ij(a,b) / (4 m_ij)
 *   CCC_ij(a,b)   = f_ij(a,b) (1 - g f_i(a)) (1 - g f_j(b))  (Sec. 2.1, Eq. (3))
 *   C_ijk(a,b,c)  = sum_q rho_i(a) rho_j(b) rho_k(c)         (Sec. 2.2, Eq. (5))
 *   CCC_ijk       = f_ijk (1-g f_i(a))(1-g f_j(b))(1-g f_k(c)) (Sec. 2.2, Eq. (4))
 *
 * Readings taken where the paper is silent (missing data is only sketched in
 * its future-work section, which reserves the allele pair (1,0) as the
 * missing marker):
 *   - a missing entry contributes to no tally (rho = 0 for both alleles);
 *   - m_i is the number of present fields of vector i, m_ij (m_ijk) the number
 *     of fields where all vectors of the pair (triple) are present, so that
 *     f_i(0)+f_i(1) = 1 and the joint frequencies sum to 1 as the paper notes;
 *     with no missing data m_i = m_ij = m_ijk = n_f, the paper's normaliser;
 *   - a zero denominator gives f = 0 (m_i = 0) or CCC = 0 (m_ij = 0);
 *   - table entry order is 2a+b (2-way) and 4a+2b+c (3-way), a belonging to
 *     the smallest vector index; pairs i<j and triples i<j<k are stored in
 *     lexicographic order.
 *
 * Packed input: uint8 v[n][ld]; field q at bits 2(q%4) and 2(q%4)+1 of byte
 * q/4; the 2-bit code is the allele pair (high bit, low bit).
 *
 * Loops run over the first index serially and over the second in parallel
 * (OpenMP), so a single sampled row uses every core.
 *
 * Whole-output checksums (the paper's exact checksum idea, Sec. 5) are
 * weighted sums mod the prime 2^61-1; the *_from_input forms evaluate the same
 * sum through a reordering that needs only O(n_v n_f) work.
 */
#include <stdint.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* Entry decoding (Sec. 2.1).                                                 */
/* ------------------------------------------------------------------------- */

/* The 2-bit code of field q of a packed row. */
static inline unsigned code_at(const uint8_t* row, int64_t q) {
  return (row[q >> 2] >> (2 * (q & 3))) & 3u;
}

/* Allele pair (v)_1 = high bit, (v)_2 = low bit; (1,0) marks a missing entry. */
static inline int is_missing(unsigned code) { return code == 2u; }

/* rho(a): how many of the two alleles equal a; 0 for a missing entry. */
static inline int rho(unsigned code, int a) {
  if (is_missing(code)) return 0;
  int r1 = (int)((code >> 1) & 1u), r2 = (int)(code & 1u);
  return (r1 == a) + (r2 == a);
}

static inline int present(unsigned code) { return !is_missing(code); }

/* ------------------------------------------------------------------------- */
/* 1-way: n_i(a) and m_i.                                                     */
/* ------------------------------------------------------------------------- */

/* out[i*3 + 0] = n_i(0), out[i*3 + 1] = n_i(1), out[i*3 + 2] = m_i. */
void oracle_counts1(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_v; ++i) {
    const uint8_t* row = v + i * ld;
    int64_t n0 = 0, n1 = 0, m = 0;
    for (int64_t q = 0; q < n_f; ++q) {
      unsigned c = code_at(row, q);
      n0 += rho(c, 0);
      n1 += rho(c, 1);
      m += present(c);
    }
    out[i * 3 + 0] = n0;
    out[i * 3 + 1] = n1;
    out[i * 3 + 2] = m;
  }
}

/* f_i(a) = n_i(a) / (2 m_i), 0 when nothing is present (Eq. (1)). */
static inline double freq1(int64_t n_a, int64_t m) {
  return m > 0 ? (double)n_a / (2.0 * (double)m) : 0.0;
}

/* ------------------------------------------------------------------------- */
/* Packed pair / triple indices.                                              */
/* ------------------------------------------------------------------------- */

/* Index of pair (i, j), i < j, in lexicographic order over n vectors. */
int64_t oracle_pair_index(int64_t n, int64_t i, int64_t j) {
  return i * n - i * (i + 1) / 2 + (j - i - 1);
}

static inline int64_t choose3(int64_t n) { return n < 3 ? 0 : n * (n - 1) * (n - 2) / 6; }
static inline int64_t choose2(int64_t n) { return n < 2 ? 0 : n * (n - 1) / 2; }

/* Index of triple (i, j, k), i < j < k, in lexicographic order over n vectors. */
int64_t oracle_triple_index(int64_t n, int64_t i, int64_t j, int64_t k) {
  /* triples whose first index is below i, then pairs (j', k') of the rest
     with j' < j, then k's offset */
  int64_t before_i = choose3(n) - choose3(n - i);
  int64_t before_j = choose2(n - i - 1) - choose2(n - j);
  return before_i + before_j + (k - j - 1);
}

/* ------------------------------------------------------------------------- */
/* 2-way tallies and CCC (Sec. 2.1, Eqs. (2)-(3)).                            */
/* ------------------------------------------------------------------------- */

static void ccc_pair(const int64_t t[4], const int64_t* ci, const int64_t* cj, double gamma,
                     double out[4]) {
  int64_t sum = t[0] + t[1] + t[2] + t[3];
  int64_t m_ij = sum / 4; /* fields where both are present */
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      double val = 0.0;
      if (m_ij > 0) {
        double f_ij = (double)t[2 * a + b] / (4.0 * (double)m_ij);
        double fi = freq1(ci[a], ci[2]);
        double fj = freq1(cj[b], cj[2]);
        val = f_ij * (1.0 - gamma * fi) * (1.0 - gamma * fj);
      }
      out[2 * a + b] = val;
    }
}

/*
 * All pairs (i, j) with i0 <= i < i1 and i < j < n_v.  tables (int64 [.][4])
 * and ccc (double [.][4], may be NULL) are indexed from the first pair of row
 * i0, i.e. entry p(i,j) - p(i0, i0+1).  counts is [n_v][3] from
 * oracle_counts1 (needed only when ccc is not NULL).
 */
void oracle_2way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i0,
                      int64_t i1, const int64_t* counts, double gamma, int64_t* tables,
                      double* ccc) {
  if (i0 >= i1) return;
  int64_t base = oracle_pair_index(n_v, i0, i0 + 1);
  for (int64_t i = i0; i < i1; ++i) {
    const uint8_t* ri = v + i * ld;
#pragma omp parallel for schedule(static)
    for (int64_t j = i + 1; j < n_v; ++j) {
      const uint8_t* rj = v + j * ld;
      int64_t t[4] = {0, 0, 0, 0};
      for (int64_t q = 0; q < n_f; ++q) {
        unsigned ci = code_at(ri, q), cj = code_at(rj, q);
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) t[2 * a + b] += (int64_t)rho(ci, a) * rho(cj, b);
      }
      int64_t p = oracle_pair_index(n_v, i, j) - base;
      for (int e = 0; e < 4; ++e) tables[p * 4 + e] = t[e];
      if (ccc) ccc_pair(t, counts + i * 3, counts + j * 3, gamma, ccc + p * 4);
    }
  }
}

/*
 * Off-diagonal block: every (i in A, j in B) for rows a0 <= i < a1 of A.
 * tables/ccc are row-major [a1-a0][n_b][4].  counts_a / counts_b are the
 * [n][3] 1-way counts of A and B (needed only for ccc).
 */
void oracle_block_rows(const uint8_t* va, int64_t lda, const uint8_t* vb, int64_t n_b,
                       int64_t ldb, int64_t n_f, int64_t a0, int64_t a1,
                       const int64_t* counts_a, const int64_t* counts_b, double gamma,
                       int64_t* tables, double* ccc) {
  for (int64_t i = a0; i < a1; ++i) {
    const uint8_t* ri = va + i * lda;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_b; ++j) {
      const uint8_t* rj = vb + j * ldb;
      int64_t t[4] = {0, 0, 0, 0};
      for (int64_t q = 0; q < n_f; ++q) {
        unsigned ci = code_at(ri, q), cj = code_at(rj, q);
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) t[2 * a + b] += (int64_t)rho(ci, a) * rho(cj, b);
      }
      int64_t p = (i - a0) * n_b + j;
      for (int e = 0; e < 4; ++e) tables[p * 4 + e] = t[e];
      if (ccc) ccc_pair(t, counts_a + i * 3, counts_b + j * 3, gamma, ccc + p * 4);
    }
  }
}

/* ------------------------------------------------------------------------- */
/* 3-way tallies and CCC (Sec. 2.2, Eqs. (4)-(5)).                            */
/* ------------------------------------------------------------------------- */

static void ccc_triple(const int64_t t[8], const int64_t* ci, const int64_t* cj,
                       const int64_t* ck, double gamma, double out[8]) {
  int64_t sum = 0;
  for (int e = 0; e < 8; ++e) sum += t[e];
  int64_t m_ijk = sum / 8; /* fields where all three are present */
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int c = 0; c < 2; ++c) {
        double val = 0.0;
        if (m_ijk > 0) {
          double f = (double)t[4 * a + 2 * b + c] / (8.0 * (double)m_ijk);
          val = f * (1.0 - gamma * freq1(ci[a], ci[2])) * (1.0 - gamma * freq1(cj[b], cj[2])) *
                (1.0 - gamma * freq1(ck[c], ck[2]));
        }
        out[4 * a + 2 * b + c] = val;
      }
}

/*
 * All triples (i, j, k), i0 <= i < i1, i < j < k < n_v; tables int64 [.][8]
 * and ccc double [.][8] (may be NULL) indexed from the first triple of row
 * i0.
 */
void oracle_3way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i0,
                      int64_t i1, const int64_t* counts, double gamma, int64_t* tables,
                      double* ccc) {
  if (i0 >= i1 || n_v < 3) return;
  int64_t base = oracle_triple_index(n_v, i0, i0 + 1, i0 + 2);
  for (int64_t i = i0; i < i1; ++i) {
#pragma omp parallel for schedule(dynamic)
    for (int64_t j = i + 1; j < n_v; ++j) {
      const uint8_t* ri = v + i * ld;
      const uint8_t* rj = v + j * ld;
      for (int64_t k = j + 1; k < n_v; ++k) {
        const uint8_t* rk = v + k * ld;
        int64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t q = 0; q < n_f; ++q) {
          unsigned ci = code_at(ri, q), cj = code_at(rj, q), ck = code_at(rk, q);
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
              for (int c = 0; c < 2; ++c)
                t[4 * a + 2 * b + c] += (int64_t)rho(ci, a) * rho(cj, b) * rho(ck, c);
        }
        int64_t p = oracle_triple_index(n_v, i, j, k) - base;
        for (int e = 0; e < 8; ++e) tables[p * 8 + e] = t[e];
        if (ccc) ccc_triple(t, counts + i * 3, counts + j * 3, counts + k * 3, gamma, ccc + p * 8);
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Explicit lists of pairs / triples (sampled checks at full size).           */
/* ------------------------------------------------------------------------- */

/* 2-way tables and CCC for the pairs (ia[p] in A, jb[p] in B), p < np; for a
   triangle pass the same set as A and B.  counts_a/counts_b are [n][3]. */
void oracle_2way_list(const uint8_t* va, int64_t lda, const uint8_t* vb, int64_t ldb,
                      int64_t n_f, const int64_t* ia, const int64_t* jb, int64_t np,
                      const int64_t* counts_a, const int64_t* counts_b, double gamma,
                      int64_t* tables, double* ccc) {
#pragma omp parallel for schedule(dynamic)
  for (int64_t p = 0; p < np; ++p) {
    const uint8_t* ri = va + ia[p] * lda;
    const uint8_t* rj = vb + jb[p] * ldb;
    int64_t t[4] = {0, 0, 0, 0};
    for (int64_t q = 0; q < n_f; ++q) {
      unsigned ci = code_at(ri, q), cj = code_at(rj, q);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) t[2 * a + b] += (int64_t)rho(ci, a) * rho(cj, b);
    }
    for (int e = 0; e < 4; ++e) tables[p * 4 + e] = t[e];
    if (ccc) ccc_pair(t, counts_a + ia[p] * 3, counts_b + jb[p] * 3, gamma, ccc + p * 4);
  }
}

/* 3-way tables and CCC for the triples (ii[p], jj[p], kk[p]), p < np. */
void oracle_3way_list(const uint8_t* v, int64_t ld, int64_t n_f, const int64_t* ii,
                      const int64_t* jj, const int64_t* kk, int64_t np, const int64_t* counts,
                      double gamma, int64_t* tables, double* ccc) {
#pragma omp parallel for schedule(dynamic)
  for (int64_t p = 0; p < np; ++p) {
    const uint8_t* ri = v + ii[p] * ld;
    const uint8_t* rj = v + jj[p] * ld;
    const uint8_t* rk = v + kk[p] * ld;
    int64_t t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t q = 0; q < n_f; ++q) {
      unsigned ci = code_at(ri, q), cj = code_at(rj, q), ck = code_at(rk, q);
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int c = 0; c < 2; ++c)
            t[4 * a + 2 * b + c] += (int64_t)rho(ci, a) * rho(cj, b) * rho(ck, c);
    }
    for (int e = 0; e < 8; ++e) tables[p * 8 + e] = t[e];
    if (ccc)
      ccc_triple(t, counts + ii[p] * 3, counts + jj[p] * 3, counts + kk[p] * 3, gamma,
                 ccc + p * 8);
  }
}

/* ------------------------------------------------------------------------- */
/* Whole-output checksums mod 2^61 - 1.                                       */
/* ------------------------------------------------------------------------- */

static const uint64_t P61 = (1ull << 61) - 1;

static inline uint64_t mod61(unsigned __int128 x) {
  uint64_t lo = (uint64_t)(x & P61);
  uint64_t hi = (uint64_t)(x >> 61);
  uint64_t r = lo + (hi & P61) + (uint64_t)(hi >> 61);
  while (r >= P61) r -= P61;
  return r;
}
static inline uint64_t mulmod(uint64_t a, uint64_t b) { return mod61((unsigned __int128)a * b); }
static inline uint64_t addmod(uint64_t a, uint64_t b) {
  uint64_t r = a + b;
  return r >= P61 ? r - P61 : r;
}

/*
 * F2(a,b) = sum_{i<j} w_i u_j C_ij(a,b) mod P, evaluated from the input as
 * sum_q sum_j u_j rho_{j,q}(b) (sum_{i<j} w_i rho_{i,q}(a)).  out[2a+b].
 */
void oracle_fp2_from_input(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld,
                           const uint64_t* w, const uint64_t* u, uint64_t out[4]) {
  enum { QB = 256 };
  uint64_t total[4] = {0, 0, 0, 0};
  int64_t nblk = (n_f + QB - 1) / QB;
#pragma omp parallel
  {
    uint64_t acc[4] = {0, 0, 0, 0};
    uint64_t pre[2][QB];
#pragma omp for schedule(dynamic)
    for (int64_t blk = 0; blk < nblk; ++blk) {
      int64_t q0 = blk * QB, q1 = q0 + QB < n_f ? q0 + QB : n_f;
      memset(pre, 0, sizeof(pre));
      for (int64_t j = 0; j < n_v; ++j) {
        const uint8_t* row = v + j * ld;
        for (int64_t q = q0; q < q1; ++q) {
          unsigned c = code_at(row, q);
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              uint64_t ub = mulmod(u[j], (uint64_t)rho(c, b));
              acc[2 * a + b] = addmod(acc[2 * a + b], mulmod(ub, pre[a][q - q0]));
            }
          for (int a = 0; a < 2; ++a)
            pre[a][q - q0] = addmod(pre[a][q - q0], mulmod(w[j], (uint64_t)rho(c, a)));
        }
      }
    }
#pragma omp critical
    for (int e = 0; e < 4; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < 4; ++e) out[e] = total[e];
}

/* The same checksum evaluated directly over given int32 tables [pairs][4]. */
void oracle_fp2_from_tables(const int32_t* tables, int64_t n_v, const uint64_t* w,
                            const uint64_t* u, uint64_t out[4]) {
  uint64_t total[4] = {0, 0, 0, 0};
#pragma omp parallel
  {
    uint64_t acc[4] = {0, 0, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_v; ++i) {
      int64_t p = oracle_pair_index(n_v, i, i + 1);
      for (int64_t j = i + 1; j < n_v; ++j, ++p) {
        uint64_t wu = mulmod(w[i], u[j]);
        for (int e = 0; e < 4; ++e) {
          int64_t t = tables[p * 4 + e];
          uint64_t tv = t >= 0 ? (uint64_t)t : P61 - (uint64_t)(-t);
          acc[e] = addmod(acc[e], mulmod(wu, tv));
        }
      }
    }
#pragma omp critical
    for (int e = 0; e < 4; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < 4; ++e) out[e] = total[e];
}

/*
 * Fb(a,b) = sum_{i in A, j in B} w_i u_j C_ij(a,b)
 *         = sum_q (sum_i w_i rho_{i,q}(a)) (sum_j u_j rho_{j,q}(b)).
 */
void oracle_fpb_from_input(const uint8_t* va, int64_t n_a, int64_t lda, const uint8_t* vb,
                           int64_t n_b, int64_t ldb, int64_t n_f, const uint64_t* w,
                           const uint64_t* u, uint64_t out[4]) {
  enum { QB = 256 };
  uint64_t total[4] = {0, 0, 0, 0};
  int64_t nblk = (n_f + QB - 1) / QB;
#pragma omp parallel
  {
    uint64_t acc[4] = {0, 0, 0, 0};
    uint64_t sa[2][QB], sb[2][QB];
#pragma omp for schedule(dynamic)
    for (int64_t blk = 0; blk < nblk; ++blk) {
      int64_t q0 = blk * QB, q1 = q0 + QB < n_f ? q0 + QB : n_f;
      memset(sa, 0, sizeof(sa));
      memset(sb, 0, sizeof(sb));
      for (int64_t i = 0; i < n_a; ++i)
        for (int64_t q = q0; q < q1; ++q) {
          unsigned c = code_at(va + i * lda, q);
          for (int a = 0; a < 2; ++a)
            sa[a][q - q0] = addmod(sa[a][q - q0], mulmod(w[i], (uint64_t)rho(c, a)));
        }
      for (int64_t j = 0; j < n_b; ++j)
        for (int64_t q = q0; q < q1; ++q) {
          unsigned c = code_at(vb + j * ldb, q);
          for (int b = 0; b < 2; ++b)
            sb[b][q - q0] = addmod(sb[b][q - q0], mulmod(u[j], (uint64_t)rho(c, b)));
        }
      for (int64_t q = q0; q < q1; ++q)
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b)
            acc[2 * a + b] = addmod(acc[2 * a + b], mulmod(sa[a][q - q0], sb[b][q - q0]));
    }
#pragma omp critical
    for (int e = 0; e < 4; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < 4; ++e) out[e] = total[e];
}

/* Direct form over given int32 block tables [n_a][n_b][4]. */
void oracle_fpb_from_tables(const int32_t* tables, int64_t n_a, int64_t n_b, const uint64_t* w,
                            const uint64_t* u, uint64_t out[4]) {
  uint64_t total[4] = {0, 0, 0, 0};
#pragma omp parallel
  {
    uint64_t acc[4] = {0, 0, 0, 0};
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n_a; ++i)
      for (int64_t j = 0; j < n_b; ++j) {
        uint64_t wu = mulmod(w[i], u[j]);
        for (int e = 0; e < 4; ++e) {
          int64_t t = tables[(i * n_b + j) * 4 + e];
          uint64_t tv = t >= 0 ? (uint64_t)t : P61 - (uint64_t)(-t);
          acc[e] = addmod(acc[e], mulmod(wu, tv));
        }
      }
#pragma omp critical
    for (int e = 0; e < 4; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < 4; ++e) out[e] = total[e];
}

/*
 * F3(a,b,c) = sum_{i<j<k} w_i u_j z_k C_ijk(a,b,c)
 *           = sum_q sum_j u_j rho_j(b) (sum_{i<j} w_i rho_i(a)) (sum_{k>j} z_k rho_k(c)).
 * out[4a+2b+c].
 */
void oracle_fp3_from_input(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld,
                           const uint64_t* w, const uint64_t* u, const uint64_t* z,
                           uint64_t out[8]) {
  enum { QB = 128 };
  uint64_t total[8] = {0};
  int64_t nblk = (n_f + QB - 1) / QB;
#pragma omp parallel
  {
    uint64_t acc[8] = {0};
    uint64_t pre[2][QB], suf[2][QB];
#pragma omp for schedule(dynamic)
    for (int64_t blk = 0; blk < nblk; ++blk) {
      int64_t q0 = blk * QB, q1 = q0 + QB < n_f ? q0 + QB : n_f;
      memset(pre, 0, sizeof(pre));
      memset(suf, 0, sizeof(suf));
      /* suffix sums over all k first, then peel k = j off as j advances */
      for (int64_t k = 0; k < n_v; ++k)
        for (int64_t q = q0; q < q1; ++q) {
          unsigned c = code_at(v + k * ld, q);
          for (int cc = 0; cc < 2; ++cc)
            suf[cc][q - q0] = addmod(suf[cc][q - q0], mulmod(z[k], (uint64_t)rho(c, cc)));
        }
      for (int64_t j = 0; j < n_v; ++j) {
        const uint8_t* row = v + j * ld;
        for (int64_t q = q0; q < q1; ++q) {
          unsigned c = code_at(row, q);
          for (int cc = 0; cc < 2; ++cc) /* now suf holds k > j */
            suf[cc][q - q0] = addmod(suf[cc][q - q0],
                                     P61 - mulmod(z[j], (uint64_t)rho(c, cc)));
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              uint64_t ub = mulmod(u[j], (uint64_t)rho(c, b));
              uint64_t t = mulmod(ub, pre[a][q - q0]);
              for (int cc = 0; cc < 2; ++cc)
                acc[4 * a + 2 * b + cc] =
                    addmod(acc[4 * a + 2 * b + cc], mulmod(t, suf[cc][q - q0]));
            }
          for (int a = 0; a < 2; ++a)
            pre[a][q - q0] = addmod(pre[a][q - q0], mulmod(w[j], (uint64_t)rho(c, a)));
        }
      }
    }
#pragma omp critical
    for (int e = 0; e < 8; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < 8; ++e) out[e] = total[e];
}

/*
 * Direct form over a slice of given int32 triple tables: the tables hold the
 * consecutive triples starting at lexicographic index t_begin (count n_t).
 * Partial results from consecutive slices add up mod P.
 */
void oracle_fp3_from_tables(const int32_t* tables, int64_t n_v, int64_t t_begin, int64_t n_t,
                            const uint64_t* w, const uint64_t* u, const uint64_t* z,
                            uint64_t out[8]) {
  uint64_t total[8] = {0};
  if (n_t <= 0) {
    for (int e = 0; e < 8; ++e) out[e] = 0;
    return;
  }
  int64_t t_end = t_begin + n_t;
#pragma omp parallel
  {
    uint64_t acc[8] = {0};
#pragma omp for schedule(dynamic, 1)
    for (int64_t i = 0; i < n_v; ++i) {
      for (int64_t j = i + 1; j < n_v; ++j) {
        int64_t first = oracle_triple_index(n_v, i, j, j + 1);
        int64_t cnt = n_v - j - 1;
        if (cnt <= 0 || first + cnt <= t_begin || first >= t_end) continue;
        uint64_t wu = mulmod(w[i], u[j]);
        for (int64_t k = j + 1; k < n_v; ++k) {
          int64_t p = first + (k - j - 1);
          if (p < t_begin || p >= t_end) continue;
          uint64_t wuz = mulmod(wu, z[k]);
          const int32_t* t = tables + (p - t_begin) * 8;
          for (int e = 0; e < 8; ++e) {
            int64_t tv = t[e];
            uint64_t x = tv >= 0 ? (uint64_t)tv : P61 - (uint64_t)(-tv);
            acc[e] = addmod(acc[e], mulmod(wuz, x));
          }
        }
      }
    }
#pragma omp critical
    for (int e = 0; e < 8; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < 8; ++e) out[e] = total[e];
}

/* Threads an OpenMP region would use (1 without OpenMP). */
/* ========================================================================= */
/* Multi-allelic 2-way CCC: markers with s states (2 <= s <= 4).  The paper    */
/* states this extension (Sec. 7, item 2): a pair of markers with s1 and s2   */
/* states gets the s1 x s2 table of relationships.  The 2-way definitions of  */
/* Sec. 2.1 are taken over the state set {0, .., s-1} unchanged:              */
/*   rho_{i,q}(a) = copies of state a among the entry's two alleles,          */
/*   f_i(a) = n_i(a) / (2 m_i),  C_ij(a,b) = sum_q rho_i(a) rho_j(b),          */
/*   f_ij(a,b) = C_ij(a,b) / (4 m_ij),                                        */
/*   CCC_ij(a,b) = f_ij(a,b) (1 - g f_i(a)) (1 - g f_j(b)),                    */
/* with the same missing-data readings as above.  A marker with fewer than s  */
/* states simply never holds the others (zero rows / columns).                */
/*                                                                             */
/* Input: uint8 v[n][ld], one byte per field: bits 2a, 2a+1 hold rho(a) for    */
/* a < s.  A present entry has counts summing to 2; the byte 0 is a missing   */
/* entry.  Tables and CCC hold s*s entries per pair, entry a*s + b.           */
/* ========================================================================= */

static inline int mrho(uint8_t byte, int a) { return (byte >> (2 * a)) & 3; }

/* 1 when the entry holds two alleles among the first s states. */
static inline int mpresent(uint8_t byte, int s) {
  int total = 0;
  for (int a = 0; a < s; ++a) total += mrho(byte, a);
  return total == 2;
}

/* Number of bytes among the first n_f of every row that are neither a
   genotype (counts summing to 2 over the first s states, no other bits) nor
   the missing byte 0. */
int64_t oracle_multi_invalid(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s) {
  int64_t bad = 0;
  const unsigned high = s >= 4 ? 0u : (0xFFu << (2 * s)) & 0xFFu;
  for (int64_t i = 0; i < n_v; ++i)
    for (int64_t q = 0; q < n_f; ++q) {
      uint8_t b = v[i * ld + q];
      if (b != 0 && (!mpresent(b, s) || (b & high))) ++bad;
    }
  return bad;
}

/* out[i*5 + a] = n_i(a) for a < 4 (0 for a >= s), out[i*5 + 4] = m_i. */
void oracle_multi_counts1(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s,
                          int64_t* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n_v; ++i) {
    int64_t n[4] = {0, 0, 0, 0}, m = 0;
    for (int64_t q = 0; q < n_f; ++q) {
      uint8_t b = v[i * ld + q];
      if (!mpresent(b, s)) continue;
      ++m;
      for (int a = 0; a < s; ++a) n[a] += mrho(b, a);
    }
    for (int a = 0; a < 4; ++a) out[i * 5 + a] = n[a];
    out[i * 5 + 4] = m;
  }
}

static void multi_tally(const uint8_t* ri, const uint8_t* rj, int64_t n_f, int s,
                        int64_t* t) {
  for (int e = 0; e < s * s; ++e) t[e] = 0;
  for (int64_t q = 0; q < n_f; ++q) {
    uint8_t bi = ri[q], bj = rj[q];
    if (!mpresent(bi, s) || !mpresent(bj, s)) continue;
    for (int a = 0; a < s; ++a)
      for (int b = 0; b < s; ++b) t[a * s + b] += (int64_t)mrho(bi, a) * mrho(bj, b);
  }
}

static void multi_ccc(const int64_t* t, int s, const int64_t* ci, const int64_t* cj,
                      double gamma, double* out) {
  int64_t sum = 0;
  for (int e = 0; e < s * s; ++e) sum += t[e];
  int64_t m_ij = sum / 4; /* fields where both are present */
  for (int a = 0; a < s; ++a)
    for (int b = 0; b < s; ++b) {
      double val = 0.0;
      if (m_ij > 0) {
        double f_ij = (double)t[a * s + b] / (4.0 * (double)m_ij);
        double fi = freq1(ci[a], ci[4]);
        double fj = freq1(cj[b], cj[4]);
        val = f_ij * (1.0 - gamma * fi) * (1.0 - gamma * fj);
      }
      out[a * s + b] = val;
    }
}

/* All pairs i < j with i0 <= i < i1; tables int64 [.][s*s] and ccc (may be
   NULL) from the first pair of row i0; counts [n_v][5] from
   oracle_multi_counts1. */
void oracle_multi_2way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s,
                            int64_t i0, int64_t i1, const int64_t* counts, double gamma,
                            int64_t* tables, double* ccc) {
  if (i0 >= i1) return;
  const int ss = s * s;
  int64_t base = oracle_pair_index(n_v, i0, i0 + 1);
  for (int64_t i = i0; i < i1; ++i) {
#pragma omp parallel for schedule(static)
    for (int64_t j = i + 1; j < n_v; ++j) {
      int64_t p = oracle_pair_index(n_v, i, j) - base;
      multi_tally(v + i * ld, v + j * ld, n_f, s, tables + p * ss);
      if (ccc) multi_ccc(tables + p * ss, s, counts + i * 5, counts + j * 5, gamma, ccc + p * ss);
    }
  }
}

/* Tables and CCC of the listed pairs (ia[p], jb[p]), p < np. */
void oracle_multi_2way_list(const uint8_t* v, int64_t ld, int64_t n_f, int s, const int64_t* ia,
                            const int64_t* jb, int64_t np, const int64_t* counts, double gamma,
                            int64_t* tables, double* ccc) {
  const int ss = s * s;
#pragma omp parallel for schedule(dynamic)
  for (int64_t p = 0; p < np; ++p) {
    multi_tally(v + ia[p] * ld, v + jb[p] * ld, n_f, s, tables + p * ss);
    if (ccc)
      multi_ccc(tables + p * ss, s, counts + ia[p] * 5, counts + jb[p] * 5, gamma, ccc + p * ss);
  }
}

/* F(a,b) = sum_{i<j} w_i u_j C_ij(a,b) mod 2^61-1 from the input in
   O(n_v n_f s^2) (as oracle_fp2_from_input); out[a*s + b]. */
void oracle_multi_fp2_from_input(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s,
                                 const uint64_t* w, const uint64_t* u, uint64_t* out) {
  enum { QB = 256 };
  const int ss = s * s;
  uint64_t total[16] = {0};
  int64_t nblk = (n_f + QB - 1) / QB;
#pragma omp parallel
  {
    uint64_t acc[16] = {0};
    uint64_t pre[4][QB];
#pragma omp for schedule(dynamic)
    for (int64_t blk = 0; blk < nblk; ++blk) {
      int64_t q0 = blk * QB, q1 = q0 + QB < n_f ? q0 + QB : n_f;
      memset(pre, 0, sizeof(pre));
      for (int64_t j = 0; j < n_v; ++j) {
        for (int64_t q = q0; q < q1; ++q) {
          uint8_t b = v[j * ld + q];
          if (!mpresent(b, s)) continue;
          for (int x = 0; x < s; ++x)
            for (int y = 0; y < s; ++y) {
              uint64_t uy = mulmod(u[j], (uint64_t)mrho(b, y));
              acc[x * s + y] = addmod(acc[x * s + y], mulmod(uy, pre[x][q - q0]));
            }
          for (int x = 0; x < s; ++x)
            pre[x][q - q0] = addmod(pre[x][q - q0], mulmod(w[j], (uint64_t)mrho(b, x)));
        }
      }
    }
#pragma omp critical
    for (int e = 0; e < ss; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < ss; ++e) out[e] = total[e];
}

/* The same checksum over given int32 tables [pairs][s*s]. */
void oracle_multi_fp2_from_tables(const int32_t* tables, int64_t n_v, int s, const uint64_t* w,
                                  const uint64_t* u, uint64_t* out) {
  const int ss = s * s;
  uint64_t total[16] = {0};
#pragma omp parallel
  {
    uint64_t acc[16] = {0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n_v; ++i) {
      int64_t p = oracle_pair_index(n_v, i, i + 1);
      for (int64_t j = i + 1; j < n_v; ++j, ++p) {
        uint64_t wu = mulmod(w[i], u[j]);
        for (int e = 0; e < ss; ++e) {
          int64_t t = tables[p * ss + e];
          uint64_t tv = t >= 0 ? (uint64_t)t : P61 - (uint64_t)(-t);
          acc[e] = addmod(acc[e], mulmod(wu, tv));
        }
      }
    }
#pragma omp critical
    for (int e = 0; e < ss; ++e) total[e] = addmod(total[e], acc[e]);
  }
  for (int e = 0; e < ss; ++e) out[e] = total[e];
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
