/*
 * ccc.h -- C ABI of the MI355X (gfx950) Custom Correlation Coefficient tally
 * library (Joubert et al., "Parallel Accelerated Custom Correlation
 * Coefficient Calculations for Genomics Applications").
 *
 * Problem statement (Sec. 2.1): n_v vectors of n_f entries; each entry is a
 * pair of alleles from {0,1}.  rho_{i,q}(a) is the number of alleles of entry
 * (i,q) equal to a.  The library computes, for every pair i<j (Sec. 2.1) or
 * triple i<j<k (Sec. 2.2), the allele co-occurrence tables
 *     C_ij(a,b)    = sum_q rho_{i,q}(a) rho_{j,q}(b)                 (Eq. (2))
 *     C_ijk(a,b,c) = sum_q rho_{i,q}(a) rho_{j,q}(b) rho_{k,q}(c)    (Eq. (5))
 * as exact integers, and the CCC values
 *     CCC_ij(a,b)    = f_ij(a,b) (1 - g f_i(a)) (1 - g f_j(b))       (Eq. (3))
 *     CCC_ijk(a,b,c) = f_ijk(a,b,c) (1-g f_i(a)) (1-g f_j(b)) (1-g f_k(c)) (Eq. (4))
 * in double precision, with f_i(a) = n_i(a) / (2 m_i) (Eq. (1)),
 * f_ij = C_ij / (4 m_ij), f_ijk = C_ijk / (8 m_ijk).
 *
 * Input layout (all entry points): packed rows, uint8 v[n][ld], ld % 16 == 0,
 * ld >= ceil(n_f/4).  Field q of vector i sits at bits 2(q%4) (low) and
 * 2(q%4)+1 (high) of byte i*ld + q/4; the 2-bit code is the allele pair, high
 * bit first: 00 = (0,0), 01 = (0,1), 11 = (1,1), and 10 = (1,0) marks a
 * missing entry (the marker the paper's future-work section sets aside).  Bits
 * past n_f are ignored whatever they hold.  Only the first ceil(n_f/4) bytes
 * of each row, rounded up to a multiple of 16, are ever read, so a row pointer
 * may point into a wider row (a field chunk) whose stride is ld.  The kernels
 * address a 16-row block of the input with 32-bit offsets, so ld (bytes) is
 * at most 2^28 (CCC_ERR_RANGE beyond; ccc_2way_multi likewise).
 *
 * Missing data: a missing entry contributes to no tally; m_i counts the
 * present fields of vector i, m_ij (m_ijk) the fields where every vector of
 * the pair (triple) is present -- so m_ij = sum C_ij / 4 and m_ijk = sum C_ijk
 * / 8.  With no missing data these all equal n_f, the paper's normaliser.  A
 * zero m_i gives f_i = 0; a zero m_ij (m_ijk) gives CCC = 0 for the pair
 * (triple).
 *
 * Output layouts: table entry order is 2a+b (2-way) and 4a+2b+c (3-way), a
 * belonging to the smallest vector index.  Pairs i<j are stored at
 *     p(i,j) = i*n_v - i(i+1)/2 + (j-i-1)                     (lexicographic),
 * triples i<j<k at their lexicographic rank
 *     C(n_v,3) - C(n_v-i,3) + C(n_v-i-1,2) - C(n_v-j,2) + (k-j-1).
 * Per-vector counts are int32 [n][4] = (n_i(0), n_i(1), m_i, 0).
 *
 * Conventions for every entry point:
 *  - All array arguments are DEVICE pointers owned by the caller, 16-byte
 *    aligned.  The library never frees them.
 *  - Work is enqueued on `stream` (NULL = the default stream) and returns
 *    without waiting for it.
 *  - A negative return code comes from argument validation done before any
 *    work is enqueued; outputs are then untouched.  CCC_ERR_HIP means a HIP
 *    call or launch failed after validation.
 *  - The library keeps a per-device workspace (allocated on first need,
 *    grown on demand, released by ccc_release_workspace).  Calls are
 *    reentrant per stream; calls on different streams of one device that
 *    need the workspace must be ordered by the caller.
 */
#ifndef CCC_H
#define CCC_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
enum {
  CCC_OK = 0,
  CCC_ERR_ARG = -1,         /* null pointer, negative size, bad option, ld < ceil(n_f/4) */
  CCC_ERR_RANGE = -2,       /* a table entry could exceed INT32_MAX (see each call) */
  CCC_ERR_ALIGN = -3,       /* pointer not 16-byte aligned or ld % 16 != 0 */
  CCC_ERR_HIP = -4,         /* a HIP call or kernel launch failed */
  CCC_ERR_NOMEM = -5,       /* workspace allocation failed */
  CCC_ERR_UNSUPPORTED = -6  /* no gfx950 device / feature not available */
};

/* Computation paths.  Both give bit-identical tables. */
enum {
  CCC_PATH_AUTO = 0,      /* MFMA */
  CCC_PATH_POPCOUNT = 1,  /* bitwise AND + population count (the paper's tally form, Sec. 3.1) */
  CCC_PATH_MFMA = 2       /* per-allele counts as matrix-core operands (formats below) */
};

/*
 * Operand formats of the MFMA path (ccc_opts.operands).  Both give the same
 * exact integer tables; they differ in speed and range.
 *  - CCC_OPERANDS_INT8: per-allele counts rho(a) in {0,1,2} (or planes built
 *    from them) as int8 operands with int32 accumulation -- the paper's
 *    modified-GEMM tally (Sec. 3.1) on the int8 matrix cores.  Valid for
 *    every n_f the call accepts.
 *  - CCC_OPERANDS_FP4: the same planes halved (rho(a)/2, P/2 with P = 1 for
 *    a present entry, and for the 3-way middle vector (rho(1) - P)/2), values
 *    0, +-1/2 and 1, each exact in e2m1, with fp32 accumulation at twice the
 *    int8 rate.  Every partial sum is a multiple of 1/4 of magnitude at most
 *    n_f, so fp32 holds it exactly while n_f <= 2^22 (a batch of
 *    ccc_2way_many: while every problem's n_f is; a chunk of ccc_2way_block:
 *    while the chunk's n_f is).  Beyond that the call returns CCC_ERR_RANGE.
 *  - CCC_OPERANDS_AUTO (0): fp4 while n_f <= 2^22, int8 beyond.
 * With CCC_PATH_POPCOUNT the field must be CCC_OPERANDS_AUTO (else
 * CCC_ERR_ARG).
 */
enum { CCC_OPERANDS_AUTO = 0, CCC_OPERANDS_FP4 = 4, CCC_OPERANDS_INT8 = 8 };

/* CCC_OPERANDS_FP4 or _INT8: the format an MFMA call over n_f fields takes
 * with CCC_OPERANDS_AUTO (host only, no device work); CCC_ERR_ARG for
 * n_f < 0. */
int ccc_mfma_operands(int64_t n_f);

/* Flags for ccc_2way_block (field-chunked use). */
enum {
  CCC_ACCUMULATE = 1u, /* add this chunk into tables and counts instead of overwriting */
  CCC_FINALIZE = 2u    /* this is the last chunk: write CCC values */
};

typedef struct {
  int path;       /* CCC_PATH_* */
  double gamma;   /* the constant of Eqs. (3)-(4); the paper uses 2/3 */
  unsigned flags; /* CCC_ACCUMULATE | CCC_FINALIZE (ccc_2way_block only) */
  int operands;   /* CCC_OPERANDS_* (MFMA path only; AUTO otherwise) */
} ccc_opts;

/* Options used when `opts` is NULL: CCC_PATH_AUTO, gamma = 2/3, flags 0,
 * CCC_OPERANDS_AUTO. */
ccc_opts ccc_default_opts(void);

/*
 * ccc_2way -- all pairs i<j of one vector set (Sec. 2.1, Eqs. (1)-(3)).
 *   v       [n_v][ld] packed input.
 *   tables  int32 [n_v(n_v-1)/2][4] or NULL; written.
 *   ccc     double [n_v(n_v-1)/2][4] or NULL; written.  At least one of
 *           tables / ccc must be non-NULL.
 *   counts  int32 [n_v][4] or NULL; if given, the 1-way counts are written.
 * n_v < 2 is valid and writes no tables (counts are written when n_v == 1).
 * n_f == 0 writes all-zero tables and CCC.  CCC_ERR_RANGE if 4*n_f >
 * INT32_MAX.  opts->flags must be 0.
 */
int ccc_2way(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int32_t* tables,
             double* ccc, int32_t* counts, const ccc_opts* opts, hipStream_t stream);

/*
 * ccc_3way -- all triples i<j<k of one vector set (Sec. 2.2, Eqs. (4)-(5)).
 *   tables  int32 [C(n_v,3)][8] or NULL;  ccc double [C(n_v,3)][8] or NULL
 *   (at least one non-NULL);  counts as for ccc_2way.
 * n_v < 3 writes no tables.  CCC_ERR_RANGE if 8*n_f > INT32_MAX.
 * The path option selects the MFMA or popcount kernel.  Workspace: 8 bytes
 * per pair of 64-row tiles (work-unit offsets), 16 bytes per vector when
 * counts is NULL, and on the MFMA path the rho(1) Gram matrix that
 * complete-data units read: 4 bytes per entry over the rows from the first
 * staged row (i_begin of ccc_3way_rows, else 0) rounded down to 64, so n_v^2
 * * 4 bytes for a whole call; beyond 32768 such rows it is not kept and every
 * unit takes the general form.
 */
int ccc_3way(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int32_t* tables,
             double* ccc, int32_t* counts, const ccc_opts* opts, hipStream_t stream);

/*
 * ccc_2way_block -- every pair (i in A, j in B) of two vector sets: one
 * off-diagonal block of the paper's block decomposition of the 2-way result
 * matrix (Sec. 4), over one chunk of fields (the field axis of Sec. 4, whose
 * partial tallies are reduced by summation).
 *   va [n_a][lda], vb [n_b][ldb]: packed fields of this chunk (n_f of them).
 *   tables   int32 [n_a][n_b][4], row-major, required.  Overwritten, or added
 *            to with CCC_ACCUMULATE.
 *   counts_a int32 [n_a][4], counts_b int32 [n_b][4], required; overwritten,
 *            or added to with CCC_ACCUMULATE.
 *   ccc      double [n_a][n_b][4]; written only with CCC_FINALIZE (then
 *            required), from the (accumulated) tables and counts.
 * A sequence of calls over consecutive field chunks, the first without
 * CCC_ACCUMULATE, the rest with it, and the last with CCC_FINALIZE, gives the
 * same tables, counts and CCC as one call over all fields.  CCC_ERR_RANGE if
 * 4*n_f > INT32_MAX for this chunk; keeping the accumulated total within
 * range is the caller's duty (the counts' m_i bound it).  n_a or n_b == 0 is
 * valid and writes nothing.  A CCC_ACCUMULATE call uses (n_a + n_b) * 16 bytes
 * of the library workspace for its chunk's own counts.
 */
int ccc_2way_block(const uint8_t* va, int64_t n_a, int64_t lda, const uint8_t* vb, int64_t n_b,
                   int64_t ldb, int64_t n_f, int32_t* tables, int32_t* counts_a,
                   int32_t* counts_b, double* ccc, const ccc_opts* opts, hipStream_t stream);

/*
 * ccc_2way_rows -- the pairs (i, j) with i_begin <= i < i_end, i < j: a
 * contiguous run of the lexicographic pair order, so a large result can be
 * produced in stages (the paper's 2-way "phases", Sec. 7 item 3).  tables /
 * ccc hold the run only: pair (i, j) goes to entry p(i,j) - p(i_begin,
 * i_begin+1); the run has p(i_end-1, n_v-1) + 1 - p(i_begin, i_begin+1)
 * entries (rows i >= n_v - 1 have none).  0 <= i_begin <= i_end <= n_v,
 * else CCC_ERR_ARG; the rest as ccc_2way (counts cover all n_v vectors).
 */
int ccc_2way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i_begin,
                  int64_t i_end, int32_t* tables, double* ccc, int32_t* counts,
                  const ccc_opts* opts, hipStream_t stream);

/*
 * ccc_3way_rows -- the triples (i, j, k) with i_begin <= i < i_end: a
 * contiguous run of the lexicographic triple order (the paper's 3-way
 * stages, Sec. 4).  Triple t goes to entry t - T(i_begin, i_begin+1,
 * i_begin+2); otherwise as ccc_3way.
 */
int ccc_3way_rows(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int64_t i_begin,
                  int64_t i_end, int32_t* tables, double* ccc, int32_t* counts,
                  const ccc_opts* opts, hipStream_t stream);

/*
 * Threshold-filtered output (the paper's production use keeps only values
 * above a threshold, Sec. 7 item 6).  A pair (triple) is kept when at least
 * one of its 4 (8) CCC values is >= threshold; each kept one takes a slot from
 * the device counter `count` and, if the slot is below `cap`, writes
 *   index[slot]  = its pair index p(i,j) (triple index T(i,j,k)),
 *   ccc[slot]    = its CCC values (4 or 8 doubles),
 *   tables[slot] = its table (4 or 8 int32; skipped when tables is NULL).
 * After the call *count holds the number of kept pairs (triples); when it
 * exceeds cap only cap records were written.  Slot order is unspecified (it
 * depends on scheduling); the set of records is deterministic.  All pointers
 * are device pointers, 16-byte aligned; the library clears *count itself.
 */
typedef struct {
  int64_t* index;
  double* ccc;
  int32_t* tables;
  int64_t cap;
  unsigned long long* count;
} ccc_selection;

int ccc_2way_select(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, double threshold,
                    const ccc_selection* out, int32_t* counts, const ccc_opts* opts,
                    hipStream_t stream);
int ccc_3way_select(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, double threshold,
                    const ccc_selection* out, int32_t* counts, const ccc_opts* opts,
                    hipStream_t stream);

/* One independent 2-way problem for ccc_2way_many (same meaning as ccc_2way). */
typedef struct {
  const uint8_t* v;
  int64_t n_v, n_f, ld;
  int32_t* tables;
  double* ccc;
  int32_t* counts;
} ccc_problem;

/*
 * ccc_2way_many -- many independent 2-way problems of uneven n_v and n_f in
 * one persistent launch.  `probs` is a HOST array of n_probs descriptors
 * (device pointers inside).  Each problem gives exactly what ccc_2way would.
 * The launch sequence is captured once into a HIP graph per distinct batch
 * (same descriptors) and replayed on later calls with that batch.
 * Validation covers every problem before anything is enqueued.
 */
int ccc_2way_many(const ccc_problem* probs, int n_probs, const ccc_opts* opts,
                  hipStream_t stream);

/*
 * ccc_2way_multi -- multi-allelic 2-way CCC: markers with s = 2..4 states,
 * an s x s table per pair (the extension announced in Sec. 7 item 2: for
 * markers with s1 and s2 states, the s1 x s2 table of relationships).  The
 * Sec. 2.1 definitions are taken over the states {0, .., s-1}:
 *   rho_{i,q}(a) = copies of state a among entry (i,q)'s two alleles,
 *   f_i(a) = n_i(a) / (2 m_i),  C_ij(a,b) = sum_q rho_i(a) rho_j(b),
 *   CCC_ij(a,b) = C_ij(a,b)/(4 m_ij) * (1 - gamma f_i(a)) (1 - gamma f_j(b)),
 * with the missing-data rules of ccc_2way.
 *   v       [n_v][ld] one byte per field (ld >= n_f, ld % 16 == 0): bits 2a
 *           and 2a+1 hold rho(a) for a < s.  A genotype's counts sum to 2; the
 *           byte 0 is a missing entry.  Other byte values are invalid input:
 *           the outputs for them are unspecified (nothing is read or written
 *           out of bounds).  Bytes past n_f are ignored.  A marker with fewer
 *           than s states leaves its other rows and columns zero.
 *   s       states, 2 <= s <= 4 (else CCC_ERR_ARG).
 *   tables  int32 [n_v(n_v-1)/2][s*s] or NULL, entry a*s + b; written.
 *   ccc     double [n_v(n_v-1)/2][s*s] or NULL; at least one of the two.
 *   counts  int32 [n_v][8] or NULL: (n(0), n(1), n(2), n(3), m, 0, 0, 0),
 *           n(a) = 0 for a >= s.
 * Pairs are in lexicographic order p(i,j).  opts: path AUTO or MFMA (there is
 * no popcount form: CCC_ERR_UNSUPPORTED), flags 0.  CCC_ERR_RANGE if
 * 4*n_f > INT32_MAX.  Pointers 16-byte aligned (CCC_ERR_ALIGN).
 */
int ccc_2way_multi(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int s,
                   int32_t* tables, double* ccc, int32_t* counts, const ccc_opts* opts,
                   hipStream_t stream);

/*
 * ccc_3way_noalloc -- ccc_3way for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, validation and results as ccc_3way; it calls
 * no hipMalloc, hipFree or other allocating routine (with kernel timing off).
 * Its scratch (work-unit offsets, the counts when `counts` is NULL, and the
 * complete-data Gram matrix) lives in a fixed device array of
 * CCC_NOALLOC_SCRATCH_BYTES per device, kept until the process ends, instead
 * of the library workspace.  CCC_ERR_RANGE when the unit offsets (8 bytes per
 * tile pair of each of three unit grids: two of 64-row tiles and one of
 * 32-row tiles, about 3 n_v^2 / 512 bytes in all) plus the counts (16 bytes
 * per vector when `counts` is NULL) exceed it, about n_v > 64,000.  The Gram
 * matrix (4 n_v^2 bytes) is used only when it also fits (n_v up to about
 * 2500); otherwise every unit takes the general form, with the same results.  Every call on a
 * device shares that device's array: calls whose work overlaps on one device
 * (two streams, or two host threads) race and give undefined results; the
 * caller must order them.  The first call on a device looks up the array's
 * address there (CCC_ERR_HIP if that fails).
 */
#define CCC_NOALLOC_SCRATCH_BYTES (24ull << 20)
int ccc_3way_noalloc(const uint8_t* v, int64_t n_v, int64_t n_f, int64_t ld, int32_t* tables,
                     double* ccc, int32_t* counts, const ccc_opts* opts, hipStream_t stream);

/* Static text for a status code. */
const char* ccc_status_string(int status);

/* Free the workspace and cached graphs of every device (waits for the device). */
void ccc_release_workspace(void);

/*
 * Kernel timing (profiling aid, off by default).  While enabled, the library
 * records a pair of HIP events on the launching stream around each tally
 * kernel launch; names are "count1", "pop2", "mfma2", "pop3", "mfma3",
 * "multi2", and "many" around a ccc_2way_many launch (its graph replay).
 * "many_setup" is a host-side duration: building a new batch's work list,
 * uploading it, and capturing and instantiating its graph.
 * Do not enable it while a stream is being captured into a graph.
 *   ccc_timing_query: total milliseconds and number of recorded launches of
 *   kernel `name` (NULL = all); waits for the recorded events.
 */
void ccc_timing_enable(int on);
void ccc_timing_reset(void);
double ccc_timing_query(const char* name, int* count);

/* Library version: major*10000 + minor*100 + patch. */
int ccc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CCC_H */
