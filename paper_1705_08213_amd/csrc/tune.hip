// tune.hip -- the kernel-shape table (host only).
//
// Lines "n_v_max n_f_max kind variant [wg_per_cu]"; the first line of a kind
// whose bounds hold picks the tile variant and, for the persistent batched
// launches, the workgroups per compute unit (0 or absent: the launcher's
// default).  This is Sec. 6.3's point that the kernel shape should follow
// the problem size, made a measured table.  Kinds:
//   mfma, popcount  the batched 2-way launch (ccc_2way_many), per path;
//   oneshot         the one-shot 2-way MFMA kernel (ccc_2way, _rows, _select,
//                   _block), by the larger side of the call.
// The table is read once from $CCC_TUNE_FILE, else from tune_gfx950.txt next
// to the library.  A missing table or line gives variant 0.  For the
// autotuner, $CCC_MANY_VARIANT and $CCC_MANY_WG force the batched choice and
// $CCC_ONESHOT_VARIANT the one-shot one.
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
  int wg_per_cu;
};

std::once_flag g_once;
std::vector<TuneRule> g_rules;

int kind_of(const char* name) {
  if (strcmp(name, "mfma") == 0) return kTuneManyMfma;
  if (strcmp(name, "popcount") == 0) return kTuneManyPopcount;
  if (strcmp(name, "oneshot") == 0) return kTuneOneShot;
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
    int var, wg = 0;
    const int got = sscanf(line, "%lld %lld %31s %d %d", &nv, &nf, k, &var, &wg);
    if (got < 4) continue;
    if (got < 5 || wg < 0 || wg > 64) wg = 0;
    const int kind = kind_of(k);
    if (kind >= 0 && var >= 0) g_rules.push_back(TuneRule{nv, nf, kind, var, wg});
  }
  fclose(f);
}

}  // namespace

// An integer from the environment in [lo, hi], else -1.
static int env_int(const char* name, int lo, int hi) {
  const char* env = getenv(name);
  if (!env || !*env) return -1;
  char* end = nullptr;
  const long v = strtol(env, &end, 10);
  return (*end == 0 && v >= lo && v <= hi) ? (int)v : -1;
}

TuneChoice tune_pick(int kind, int64_t n_v, int64_t n_f, int n_variants) {
  TuneChoice c{0, 0};
  std::call_once(g_once, load_table);
  for (const TuneRule& r : g_rules)
    if (r.kind == kind && n_v <= r.nv_max && n_f <= r.nf_max) {
      c = TuneChoice{r.variant < n_variants ? r.variant : 0, r.wg_per_cu};
      break;
    }
  const bool many = kind == kTuneManyMfma || kind == kTuneManyPopcount;
  const int v = env_int(many ? "CCC_MANY_VARIANT" : "CCC_ONESHOT_VARIANT", 0, n_variants - 1);
  if (v >= 0) c.variant = v;
  if (many) {
    const int wg = env_int("CCC_MANY_WG", 1, 64);
    if (wg > 0) c.wg_per_cu = wg;
  }
  return c;
}

}  // namespace ccc
