// Autotuner of the launch configuration of a TJM run: the tile choices of
// the contractions (tile_mode) and the resident workgroups (workers).  Every
// choice computes the same trajectories (the tile shapes sum each output's
// terms in the same order, and each trajectory runs alone in its workgroup),
// so candidates are compared on identical work: separate runs of a copy of
// the model with the caller's seed.  See include/tjm.h for the contract.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "tjm_internal.h"

namespace {

struct Choice {
  int tile_mode = 0, workers = 0;
  double us = 0.0;
};

std::mutex g_mu;
std::map<std::string, Choice> g_cache;   // results of this process

int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// One trial run on a copy of src: step-kernel microseconds per
// trajectory-step over `timed` steps after `warm` untimed ones.
tjm_status trial(const tjm_model* src, int n, double dt, double T, int chi, int n_obs, const int* site,
                 const double* op, uint64_t seed, const tjm_options& o, int warm, int timed, double* us,
                 std::string* err) {
  tjm_model* c = tjm_model_copy(src);
  if (!c) { *err = "out of host memory"; return TJM_E_NOMEM; }
  tjm_status st = tjm_run_begin(c, n, dt, T, chi, n_obs, site, op, seed, &o);
  tjm_stats s0{}, s1{};
  if (st == TJM_OK && warm > 0) st = tjm_run_advance(c, warm);
  if (st == TJM_OK) st = tjm_get_stats(c, &s0);
  if (st == TJM_OK) st = tjm_run_advance(c, timed);
  if (st == TJM_OK) st = tjm_get_stats(c, &s1);
  if (st != TJM_OK) *err = tjm_last_error(c);
  if (st == TJM_OK && s1.failed_traj) { st = TJM_E_NUMERIC; *err = "non-finite norm in a trial run"; }
  tjm_destroy(c);                        // releases the unfinished run
  if (st == TJM_OK) *us = 1e3 * (s1.step_kernel_ms_total - s0.step_kernel_ms_total) / ((double)timed * n);
  return st;
}

// The cache file first (its last line for the key wins), then the results
// of this process.
bool cache_lookup(const char* path, const std::string& key, Choice* out) {
  if (path) {
    std::ifstream f(path);
    bool found = false;
    std::string line;
    while (f && std::getline(f, line)) {
      std::istringstream ls(line);
      std::string k;
      Choice c;
      if (ls >> k >> c.tile_mode >> c.workers >> c.us && k == key && c.tile_mode >= 0 && c.tile_mode <= 7 &&
          c.workers > 0) {
        *out = c;
        found = true;
      }
    }
    if (found) return true;
  }
  std::lock_guard<std::mutex> g(g_mu);
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *out = it->second;
  return true;
}

bool cache_store(const char* path, const std::string& key, const Choice& c) {
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key] = c;
  }
  if (!path) return false;
  std::FILE* f = std::fopen(path, "a");
  if (!f) return false;
  const bool ok = std::fprintf(f, "%s %d %d %.6g\n", key.c_str(), c.tile_mode, c.workers, c.us) > 0;
  return std::fclose(f) == 0 && ok;
}

}  // namespace

extern "C" tjm_status tjm_autotune(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                                   const int* obs_site, const double* obs_op, uint64_t seed,
                                   const tjm_options* base, int warm_steps, int timed_steps,
                                   const char* cache_path, tjm_tune_progress progress, void* progress_ctx,
                                   tjm_options* tuned, tjm_tune_report* rep) {
  if (!m || !tuned || !rep) return tjm_model_fail(m, TJM_E_INVAL, "NULL argument");
  if (tjm_model_busy(m)) return tjm_model_fail(m, TJM_E_BUSY, "a run is in progress on this model");
  tjm_options opt;
  tjm_default_options(&opt);
  if (base) opt = *base;
  opt.record_bonds = 0;
  opt.graph = 0;
  const int n_steps = dt > 0 && T > 0 ? (int)std::lround(T / dt) : 0;
  if (warm_steps < 0 || timed_steps < 1 || warm_steps + timed_steps > n_steps)
    return tjm_model_fail(m, TJM_E_INVAL, "warm_steps + timed_steps must be within the run's steps");
  // validation of the run as tjm_run_begin does it, and its automatic workers
  size_t bytes = 0;
  int w_auto = 0;
  tjm_options probe = opt;
  probe.workers = 0;
  tjm_status st = tjm_run_footprint(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, &probe, &bytes, &w_auto);
  if (st != TJM_OK) return st;
  int cus = 0;
  hipDeviceProp_t prop;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, opt.device) != hipSuccess ||
      hipGetDeviceProperties(&prop, opt.device) != hipSuccess)
    return tjm_model_fail(m, TJM_E_DEVICE, "device query failed");
  const int n_trial = w_auto;            // already capped by n_traj
  std::ostringstream ks;
  ks << prop.gcnArchName << "/" << cus << "cu/" << (opt.precision == TJM_PREC_MIXED ? "mixed" : "fp64") << "/L"
     << pow2_at_least(tjm_model_L(m)) << "/chi" << chi_max << "/D" << tjm_model_Dmax(m) << "/d" << tjm_model_d(m)
     << "/N" << n_trial << "/o" << opt.trotter_order;
  std::string key = ks.str();
  for (char& ch : key)
    if (ch == ' ' || ch == '\t' || ch == '\n') ch = '_';
  std::memset(rep, 0, sizeof *rep);
  std::snprintf(rep->key, sizeof rep->key, "%s", key.c_str());
  rep->trial_traj = n_trial;

  Choice best;
  if (cache_lookup(cache_path, key, &best)) {
    rep->cached = 1;
  } else {
    // tile modes that can change a product at this chi_max: the wide tiles
    // (bits 0 and 2) need 48 or more rows
    std::vector<int> modes = chi_max >= 48 ? std::vector<int>{0, 1, 2, 3, 4, 5, 6, 7} : std::vector<int>{0, 2};
    std::string err;
    best.us = -1.0;
    for (int tm : modes) {
      tjm_options o = opt;
      o.tile_mode = tm;
      o.workers = w_auto;
      double us = 0.0;
      if ((st = trial(m, n_trial, dt, T, chi_max, n_obs, obs_site, obs_op, seed, o, warm_steps, timed_steps, &us,
                      &err)) != TJM_OK)
        return tjm_model_fail(m, st, ("autotune trial: " + err).c_str());
      if (progress) progress(rep->trials, tm, w_auto, us, progress_ctx);
      ++rep->trials;
      if (tm == 0) rep->default_us_per_traj_step = us;
      if (best.us < 0 || us < best.us) { best.tile_mode = tm; best.workers = w_auto; best.us = us; }
    }
    if (cus > 0 && cus < w_auto) {       // one workgroup per compute unit
      tjm_options o = opt;
      o.tile_mode = best.tile_mode;
      o.workers = cus;
      double us = 0.0;
      if ((st = trial(m, n_trial, dt, T, chi_max, n_obs, obs_site, obs_op, seed, o, warm_steps, timed_steps, &us,
                      &err)) != TJM_OK)
        return tjm_model_fail(m, st, ("autotune trial: " + err).c_str());
      if (progress) progress(rep->trials, best.tile_mode, cus, us, progress_ctx);
      ++rep->trials;
      if (us < best.us) { best.workers = cus; best.us = us; }
    }
    rep->cache_written = cache_store(cache_path, key, best) ? 1 : 0;
  }
  *tuned = opt;
  if (base) {                            // the caller's record_bonds and graph stay
    tuned->record_bonds = base->record_bonds;
    tuned->graph = base->graph;
  }
  tuned->tile_mode = best.tile_mode;
  tuned->workers = best.workers;
  rep->tile_mode = best.tile_mode;
  rep->workers = best.workers;
  rep->us_per_traj_step = best.us;
  return TJM_OK;
}
