// kernels.h -- host-side launchers of the CCC kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
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
  int tri;
  int accumulate;             // tables += result (rectangle only)
  int32_t* tables;            // may be null when ccc is set
  double* ccc;                // may be null
  const int32_t* counts_a;    // [n_a][4]
  const int32_t* counts_b;    // [n_b][4]
  double gamma;
  // rows of A whose pairs are produced; pair (i, j) goes to entry p(i,j) - p_base
  int64_t row_begin, row_end;
  int64_t p_base;
  int64_t sq_offset;          // first square tile of the row range (triangle)
  Select sel;                 // threshold selection (sel.count != null) instead of dense output
};

// Arguments of one 3-way tally launch over all triples i < j < k.
struct Triple3Args {
  const uint8_t* v;
  int64_t ld, n, n_f;
  int32_t* tables;
  double* ccc;
  const int32_t* counts;
  double gamma;
  int64_t* offs;  // workspace: n+1 int64 (work-unit offsets per middle vector)
  // triples whose first index lies in [i_begin, i_end); triple t goes to entry t - t_base
  int64_t i_begin, i_end;
  int64_t t_base;
  Select sel;
};

enum Path { kPathPopcount = 1, kPathMfma = 2 };

// Optional event timing around the main kernel of a launcher (no-ops unless
// enabled through ccc_timing_enable).
void timing_begin(const char* name, hipStream_t stream);
void timing_end(hipStream_t stream);

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

}  // namespace ccc
