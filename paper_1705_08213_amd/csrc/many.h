// many.h -- batched 2-way problems (internal to the library).
#pragma once

#include "../../include/ccc.h"

namespace ccc {

int workspace(size_t bytes, void** out);
int run_many(const ccc_problem* probs, int n_probs, const ccc_opts& opts, hipStream_t stream);
void release_many_cache();

}  // namespace ccc
