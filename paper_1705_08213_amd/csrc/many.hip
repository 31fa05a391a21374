// many.hip -- many independent 2-way problems.
#include "kernels.h"
#include "many.h"

namespace ccc {

int run_many(const ccc_problem* probs, int n_probs, const ccc_opts& opts, hipStream_t stream) {
  size_t need = 0;
  for (int p = 0; p < n_probs; ++p)
    if (!probs[p].counts && probs[p].n_v >= 2) need += (size_t)probs[p].n_v * 16;
  char* ws = nullptr;
  if (need) {
    void* w = nullptr;
    int st = workspace(need, &w);
    if (st) return st;
    ws = static_cast<char*>(w);
  }
  for (int p = 0; p < n_probs; ++p) {
    const ccc_problem& q = probs[p];
    if (q.n_v < 1) continue;
    int32_t* cnt = q.counts;
    if (!cnt) {
      if (q.n_v < 2) continue;
      cnt = reinterpret_cast<int32_t*>(ws);
      ws += (size_t)q.n_v * 16;
    }
    if (launch_count1(q.v, q.ld, q.n_v, q.n_f, cnt, 0, stream) != hipSuccess) return CCC_ERR_HIP;
    if (q.n_v < 2) continue;
    Pair2Args a{};
    a.va = q.v; a.lda = q.ld; a.n_a = q.n_v;
    a.vb = q.v; a.ldb = q.ld; a.n_b = q.n_v;
    a.n_f = q.n_f;
    a.tri = 1;
    a.tables = q.tables;
    a.ccc = q.ccc;
    a.counts_a = cnt;
    a.counts_b = cnt;
    a.gamma = opts.gamma;
    hipError_t e = opts.path == CCC_PATH_POPCOUNT ? launch_pop2(a, stream) : launch_mfma2(a, stream);
    if (e != hipSuccess) return CCC_ERR_HIP;
  }
  return CCC_OK;
}

void release_many_cache() {}

}  // namespace ccc
