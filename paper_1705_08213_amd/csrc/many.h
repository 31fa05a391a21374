// many.h -- batched 2-way problems (internal to the library).
#pragma once

#include "../../include/ccc.h"

namespace ccc {

int workspace(size_t bytes, void** out);
// f4: fp4 operands for the MFMA path (the caller checked that every n_f
// allows them), else int8.
int run_many(const ccc_problem* probs, int n_probs, const ccc_opts& opts, bool f4,
             hipStream_t stream);
void release_many_cache();

}  // namespace ccc
