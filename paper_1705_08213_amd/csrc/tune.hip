// tune.hip -- the kernel-shape table (host only).
//
// Lines "n_v_max n_f_max kind variant"; the first line of a kind whose
// bounds hold picks the variant (Sec. 6.3's point that the kernel shape
// should follow the problem size, made a measured table).  Kinds:
//   mfma, popcount  the batched 2-way launch (ccc_2way_many), per path.
// The table is read once from $CCC_TUNE_FILE, else from tune_gfx950.txt next
// to the library.  A missing table or line gives variant 0.  For the
// autotuner, $CCC_MANY_VARIANT forces a variant.
#include <dlfcn.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace ccc {

namespace {

struct TuneRule {
  int64_t nv_max, nf_max;
  int kind;
  int variant;
};

std::once_flag g_once;
std::vector<TuneRule> g_rules;

int kind_of(const char* name) {
  if (strcmp(name, "mfma") == 0) return kTuneManyMfma;
  if (strcmp(name, "popcount") == 0) return kTuneManyPopcount;
  return -1;
}

void load_table() {
  std::string path;
  if (const char* env = getenv("CCC_TUNE_FILE")) {
    path = env;
  } else {
    Dl_info info;
    if (dladdr(reinterpret_cast<void*>(&load_table), &info) && info.dli_fname) {
      path = info.dli_fname;
      const size_t slash = path.rfind('/');
      path = (slash == std::string::npos ? std::string(".") : path.substr(0, slash)) +
             "/tune_gfx950.txt";
    }
  }
  FILE* f = path.empty() ? nullptr : fopen(path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    long long nv, nf;
    char k[32];
    int var;
    if (sscanf(line, "%lld %lld %31s %d", &nv, &nf, k, &var) != 4) continue;
    const int kind = kind_of(k);
    if (kind >= 0 && var >= 0) g_rules.push_back(TuneRule{nv, nf, kind, var});
  }
  fclose(f);
}

}  // namespace

int tune_pick(int kind, int64_t n_v, int64_t n_f, int n_variants) {
  const char* env = getenv("CCC_MANY_VARIANT");
  if (env) {
    const int v = atoi(env);
    if (v >= 0 && v < n_variants) return v;
  }
  std::call_once(g_once, load_table);
  for (const TuneRule& r : g_rules)
    if (r.kind == kind && n_v <= r.nv_max && n_f <= r.nf_max)
      return r.variant < n_variants ? r.variant : 0;
  return 0;
}

}  // namespace ccc
