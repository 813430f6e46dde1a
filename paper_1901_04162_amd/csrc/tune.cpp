// Tuning of the fill kernels: the cache of choices and the single-fill tuner.
//
// An EFIE fill (table or direct mode) can run on three kernels
// (fill_choice_name): the triangle-block tiling with 16 or 8 waves per
// workgroup, or the edge-block tiling.  mf_fill_tune times them on the caller's own fill and keeps the
// fastest, per (triangles, edges, rule, mode, output type, table placement);
// batched launches keep their workgroup size the same way.  Choices are kept
// for the process and, when MOMFILL_TUNE_CACHE names a file, in that file
// (one "key<TAB>value" line per choice, appended), so that later processes
// skip the timing.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "internal.hpp"

namespace mf {

static std::mutex g_tune_mu;
static std::map<std::string, int> g_tune;
static bool g_tune_loaded = false;

static const char *cache_file() {
  const char *f = std::getenv("MOMFILL_TUNE_CACHE");
  return f && *f ? f : nullptr;
}

static void load_locked() {
  if (g_tune_loaded) return;
  g_tune_loaded = true;
  const char *f = cache_file();
  if (!f) return;
  FILE *fp = std::fopen(f, "r");
  if (!fp) return;
  char line[512];
  while (std::fgets(line, sizeof line, fp)) {
    std::string s(line);
    const size_t tab = s.find('\t');
    if (tab == std::string::npos) continue;
    const int v = std::atoi(s.c_str() + tab + 1);
    g_tune[s.substr(0, tab)] = v;  // the last line of a key wins
  }
  std::fclose(fp);
}

bool tune_cache_get(const std::string &key, int *value) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_locked();
  auto it = g_tune.find(key);
  if (it == g_tune.end()) return false;
  *value = it->second;
  return true;
}

void tune_cache_put(const std::string &key, int value) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  load_locked();
  g_tune[key] = value;
  if (const char *f = cache_file()) {
    if (FILE *fp = std::fopen(f, "a")) {
      std::fprintf(fp, "%s\t%d\n", key.c_str(), value);
      std::fclose(fp);
    }
  }
}

std::string fill_tune_key(const mf_mesh *m, int nq, int mode, int z_dtype, const mf_tables *tab) {
  const bool lds = tab && tab->g.n - 1 <= 1899;
  return "fill nt=" + std::to_string(m->nt) + " ne=" + std::to_string(m->ne) +
         " q=" + std::to_string(nq) + " mode=" + std::to_string(mode) +
         " z=" + std::to_string(z_dtype) + " ldstable=" + std::to_string((int)lds);
}

int cached_fill_choice(const mf_mesh *m, int nq, int mode, int z_dtype, const mf_tables *tab) {
  int c = kFillTB1024;
  if (tune_cache_get(fill_tune_key(m, nq, mode, z_dtype, tab), &c) && c >= 0 && c < kFillChoices)
    return c;
  return kFillTB1024;
}

}  // namespace mf

using namespace mf;

extern "C" {

int mf_fill_tune(mf_mesh *m, const double *V, double k, int quad_order, int mode,
                 const mf_tables *tab, void *Z, int z_dtype, int64_t ldz, hipStream_t s,
                 int32_t *choice, float *ms) {
  Rule r;
  if (!m || !V || !Z || !choice) return (set_error("mf_fill_tune: NULL argument"), MF_EINVAL);
  if (!make_rule(quad_order, &r))
    return (set_error("mf_fill_tune: quad_order must be 3, 6 or 7"), MF_EINVAL);
  if (!(k > 0.0) || !std::isfinite(k)) return (set_error("mf_fill_tune: k must be > 0"), MF_EINVAL);
  if (mode != MF_MODE_TABLE && mode != MF_MODE_DIRECT)
    return (set_error("mf_fill_tune: mode must be MF_MODE_TABLE or MF_MODE_DIRECT"), MF_EINVAL);
  if (mode == MF_MODE_TABLE && (!tab || tab->g.n == 0 || std::fabs(tab->k - k) > 1e-12 * k))
    return (set_error("mf_fill_tune: tables missing, without a Green table or built for another k"),
            MF_EINVAL);
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return (set_error("mf_fill_tune: unknown z_dtype"), MF_EINVAL);
  if (ldz < m->ne) return (set_error("mf_fill_tune: ldz < number of edges"), MF_EINVAL);
  if (!m->ws)
    return (set_error("mf_fill_tune: mesh has no device workspace (mf_mesh_set_workspace)"),
            MF_EINVAL);
  if (ms)
    for (int c = 0; c < kFillChoices; ++c) ms[c] = 0.0f;
  // meshes without a triangle-block plan have one kernel
  if (!m->tb_ok) {
    *choice = kFillEB1024;
    return MF_OK;
  }
  const std::string key = fill_tune_key(m, r.nq, mode, z_dtype, tab);
  int c = -1;
  if (tune_cache_get(key, &c) && c >= 0 && c < kFillChoices) {
    m->fill_choice[mode] = c;
    *choice = c;
    return MF_OK;
  }
  int rc;
  if ((rc = launch_geometry(m, V, r, s)) || (rc = launch_singular(m, V, r, k, 0, s))) return rc;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  MF_HIP(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_fail(he, "tuner events");
  }
  int best = kFillTB1024;
  float best_ms = INFINITY;
  for (int cand = 0; cand < kFillChoices && !rc; ++cand) {
    m->fill_choice[mode] = cand;
    rc = launch_fill(m, r, k, mode, tab, Z, z_dtype, ldz, s);  // warm-up
    if (rc) break;
    he = hipEventRecord(e0, s);
    if (he == hipSuccess) rc = launch_fill(m, r, k, mode, tab, Z, z_dtype, ldz, s);
    if (!rc && he == hipSuccess) he = hipEventRecord(e1, s);
    if (!rc && he == hipSuccess) he = hipEventSynchronize(e1);
    float t = 0.0f;
    if (!rc && he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
    if (he != hipSuccess) rc = hip_fail(he, "tuner timing");
    if (ms) ms[cand] = t;
    if (!rc && t < best_ms) {
      best_ms = t;
      best = cand;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    m->fill_choice[mode] = -1;
    return rc;
  }
  m->fill_choice[mode] = best;
  *choice = best;
  tune_cache_put(key, best);
  // leave the output as the chosen kernel computes it
  return launch_fill(m, r, k, mode, tab, Z, z_dtype, ldz, s);
}

const char *mf_fill_choice_name(int32_t choice) { return fill_choice_name(choice); }

int mf_mesh_set_fill_choice(mf_mesh *m, int32_t choice) {
  if (!m) return (set_error("mf_mesh_set_fill_choice: null mesh"), MF_EINVAL);
  if (choice < -1 || choice >= kFillChoices)
    return (set_error("mf_mesh_set_fill_choice: choice must be -1, 0, 1 or 2"), MF_EINVAL);
  m->fill_choice[0] = m->fill_choice[1] = choice;
  return MF_OK;
}

}  // extern "C"
