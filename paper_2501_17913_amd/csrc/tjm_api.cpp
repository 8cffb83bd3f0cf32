// C ABI of the TJM library: validation, host-side tables, device memory and
// launches.  See include/tjm.h for the contract of every entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tjm.h"
#include "tjm_internal.h"
#include "tjm_selftest.h"

typedef std::complex<double> cd;

namespace {

struct Run {
  int n_traj = 0, n_steps = 0, n_obs = 0, steps_done = 0, workers = 0;
  TjmParams P;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::vector<void*> allocs;
  size_t bytes = 0;
  double init_ms = 0, step_ms_total = 0, step_ms_last = 0;
  int step_launches = 0;
  int use_graph = 0;
  // device pointers needed at the end
  double* d_obs = nullptr;
  int* d_jlog = nullptr;
  int* d_blog = nullptr;
  unsigned long long* d_stats = nullptr;
  int* d_flags = nullptr;
  int record_bonds = 0;

  // server jobs: no fill kernels (the serve kernel clears what it needs),
  // and uploads from pinned staging buffers on the server's upload stream,
  // which the job borrows; both leave the device to the resident kernel
  bool no_fill = false;
  bool own_stream = true;                    // false: the server's upload stream, borrowed
  std::vector<void*> host_allocs;            // pinned staging, freed with the run
  // server jobs: the host-coherent buffers the serve kernel reduces the job into
  double* h_mean = nullptr;
  double* h_sem = nullptr;
  unsigned long long* h_stats = nullptr;     // [TJM_NSTAT + 1]: statistics, failed trajectories
};

std::string g_create_err;



}  // namespace

struct tjm_model {
  int L = 0, d = 0;
  std::vector<int> mpoD;
  std::vector<std::vector<cd>> W;     // per site [wl][wr][so][si]
  int n_jump = 0;
  std::vector<int> jsite;
  std::vector<cd> jop;                // [n_jump][d][d]
  std::vector<double> jrate;
  std::vector<cd> init;               // [L][d]
  std::vector<std::vector<int>> omD;  // MPO observables: bond dimensions
  std::vector<std::vector<std::vector<cd>>> oW;   //   and site tensors [wl][wr][so][si]
  std::vector<int> init_bond;         // non-empty: Psi(0) is the MPS init_mps
  std::vector<cd> init_mps;           // M_l[s][a][b] concatenated
  std::string err;
  Run* run = nullptr;
  tjm_stats last{};
};

static tjm_status fail(tjm_model* m, tjm_status st, const std::string& msg) {
  if (m) m->err = msg; else g_create_err = msg;
  return st;
}

tjm_status tjm_fail_global(tjm_status st, const char* msg) { return fail(nullptr, st, msg); }

static bool finite_arr(const double* p, long n) {
  for (long i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

#define HIPCHK(m, expr)                                                                     \
  do {                                                                                      \
    hipError_t e_ = (expr);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(m, e_ == hipErrorOutOfMemory ? TJM_E_NOMEM : TJM_E_DEVICE,               \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

extern "C" void tjm_default_options(tjm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = TJM_PREC_FP64;
  o->chi_cap = 0;
  o->svd_discard = 1e-12;
  o->krylov_max = 30;
  o->krylov_tol = 0.0;
  o->deg_tol = 1e-12;
  o->workers = 0;
  o->record_bonds = 0;
  o->traj_base = 0;
  o->device = 0;
  o->certify_sweeps = -1;
  o->sweep_jumps = 1;
  o->generic_heff = 0;
  o->graph = 0;
  o->trotter_order = 2;
  o->tile_mode = 0;
}

// Validates an MPO in the layout of tjm_create (bond dimensions mpo_bond[0..L],
// site tensors W[s_out][s_in][w_l][w_r] concatenated) and copies it into
// per-site arrays [w_l][w_r][s_out][s_in].  Returns an error message or "".
static std::string read_mpo(int L, int d, const int* mpo_bond, const double* mpo, std::vector<int>& D,
                            std::vector<std::vector<cd>>& W) {
  if (!mpo_bond || !mpo) return "mpo_bond / mpo is NULL";
  if (mpo_bond[0] != 1 || mpo_bond[L] != 1) return "MPO boundary bonds must be 1";
  for (int b = 0; b <= L; ++b)
    if (mpo_bond[b] < 1 || mpo_bond[b] > 8) return "MPO bond dimensions must be in 1..8";
  D.assign(mpo_bond, mpo_bond + L + 1);
  W.assign(L, {});
  long off = 0;
  for (int s = 0; s < L; ++s) {
    const int Dl = mpo_bond[s], Dr = mpo_bond[s + 1];
    const long n = (long)d * d * Dl * Dr;
    if (!finite_arr(mpo + 2 * off, 2 * n)) return "MPO has non-finite entries";
    W[s].assign((size_t)n, cd(0, 0));
    for (int so = 0; so < d; ++so)
      for (int si = 0; si < d; ++si)
        for (int wl = 0; wl < Dl; ++wl)
          for (int wr = 0; wr < Dr; ++wr) {
            long src = off + (((long)so * d + si) * Dl + wl) * Dr + wr;
            W[s][(((long)wl * Dr + wr) * d + so) * d + si] = cd(mpo[2 * src], mpo[2 * src + 1]);
          }
    off += n;
  }
  return "";
}

extern "C" tjm_status tjm_add_mpo_observable(tjm_model* m, const int* mpo_bond, const double* mpo, int* index) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  if (m->run) return fail(m, TJM_E_BUSY, "a run is active");
  if (m->oW.size() >= 64) return fail(m, TJM_E_INVAL, "at most 64 MPO observables");
  std::vector<int> D;
  std::vector<std::vector<cd>> W;
  const std::string e = read_mpo(m->L, m->d, mpo_bond, mpo, D, W);
  if (!e.empty()) return fail(m, TJM_E_INVAL, e);
  m->omD.push_back(D);
  m->oW.push_back(W);
  if (index) *index = (int)m->oW.size() - 1;
  return TJM_OK;
}

extern "C" tjm_status tjm_clear_mpo_observables(tjm_model* m) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  if (m->run) return fail(m, TJM_E_BUSY, "a run is active");
  m->omD.clear();
  m->oW.clear();
  return TJM_OK;
}

extern "C" tjm_status tjm_create(tjm_model** out, int L, int d, const int* mpo_bond, const double* mpo,
                                 int n_jump, const int* jump_site, const double* jump_op,
                                 const double* rate) {
  if (!out) return fail(nullptr, TJM_E_INVAL, "out is NULL");
  *out = nullptr;
  if (L < 1) return fail(nullptr, TJM_E_INVAL, "L must be >= 1");
  if (d != 2) return fail(nullptr, TJM_E_UNSUPPORTED, "only local dimension d = 2 is supported");
  if (n_jump < 0) return fail(nullptr, TJM_E_INVAL, "n_jump must be >= 0");
  if (n_jump > 0 && (!jump_site || !jump_op || !rate))
    return fail(nullptr, TJM_E_INVAL, "jump arrays are NULL");
  tjm_model* m = new tjm_model();
  m->L = L; m->d = d;
  const std::string e = read_mpo(L, d, mpo_bond, mpo, m->mpoD, m->W);
  if (!e.empty()) {
    delete m;
    return fail(nullptr, TJM_E_INVAL, e);
  }
  m->n_jump = n_jump;
  for (int j = 0; j < n_jump; ++j) {
    if (jump_site[j] < 0 || jump_site[j] >= L) {
      delete m;
      return fail(nullptr, TJM_E_INVAL, "jump site out of range");
    }
    if (!std::isfinite(rate[j]) || rate[j] < 0.0) {
      delete m;
      return fail(nullptr, TJM_E_INVAL, "jump rates must be finite and >= 0");
    }
    if (!finite_arr(jump_op + 8L * j, 8)) {
      delete m;
      return fail(nullptr, TJM_E_INVAL, "jump operator has non-finite entries");
    }
    m->jsite.push_back(jump_site[j]);
    m->jrate.push_back(rate[j]);
    for (int e = 0; e < 4; ++e) m->jop.push_back(cd(jump_op[8L * j + 2 * e], jump_op[8L * j + 2 * e + 1]));
  }
  m->init.assign((size_t)L * d, cd(0, 0));
  for (int s = 0; s < L; ++s) m->init[(size_t)s * d] = 1.0;
  *out = m;
  return TJM_OK;
}

extern "C" tjm_status tjm_set_initial_mps(tjm_model* m, const int* bond, const double* t) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  if (!bond || !t) return fail(m, TJM_E_INVAL, "bond / tensors is NULL");
  const int L = m->L, d = m->d;
  if (bond[0] != 1 || bond[L] != 1) return fail(m, TJM_E_INVAL, "boundary bonds of the initial MPS must be 1");
  long n = 0;
  for (int l = 0; l < L; ++l) {
    if (bond[l + 1] < 1 || bond[l + 1] > 64) return fail(m, TJM_E_INVAL, "initial MPS bonds must be in 1..64");
    n += (long)d * bond[l] * bond[l + 1];
  }
  if (!finite_arr(t, 2 * n)) return fail(m, TJM_E_INVAL, "initial MPS has non-finite entries");
  m->init_bond.assign(bond, bond + L + 1);
  m->init_mps.resize(n);
  for (long i = 0; i < n; ++i) m->init_mps[i] = cd(t[2 * i], t[2 * i + 1]);
  return TJM_OK;
}

extern "C" tjm_status tjm_set_initial_product(tjm_model* m, const double* v) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  if (!v) return fail(m, TJM_E_INVAL, "site_vec is NULL");
  if (!finite_arr(v, 2L * m->L * m->d)) return fail(m, TJM_E_INVAL, "site vectors must be finite");
  for (int s = 0; s < m->L; ++s) {
    double n2 = 0;
    for (int q = 0; q < m->d; ++q) n2 += v[2 * (s * m->d + q)] * v[2 * (s * m->d + q)] + v[2 * (s * m->d + q) + 1] * v[2 * (s * m->d + q) + 1];
    if (!(n2 > 0.0)) return fail(m, TJM_E_INVAL, "a site vector is zero");
    const double f = 1.0 / std::sqrt(n2);
    for (int q = 0; q < m->d; ++q)
      m->init[(size_t)s * m->d + q] = f * cd(v[2 * (s * m->d + q)], v[2 * (s * m->d + q) + 1]);
  }
  m->init_bond.clear();
  m->init_mps.clear();
  return TJM_OK;
}

// exp(-tau/2 G) for a 2x2 Hermitian G = [[a, b], [conj b, c]]:
// -tau/2 G = mu I + N with N traceless, N^2 = rho^2 I, so
// exp = e^mu (cosh(rho) I + sinh(rho)/rho N).
static void dissipator2(const cd G[4], double tau, cd out[4]) {
  const double a = G[0].real(), c = G[3].real();
  const double f = -0.5 * tau;
  const double mu = f * 0.5 * (a + c);
  const cd n00 = f * 0.5 * (a - c), n01 = f * G[1], n10 = f * G[2];
  const double rho = std::sqrt(std::norm(n00) + std::norm(n01));
  const double ch = std::cosh(rho);
  const double sr = rho > 1e-8 ? std::sinh(rho) / rho : 1.0 + rho * rho / 6.0;
  const double e = std::exp(mu);
  out[0] = e * (ch + sr * n00);
  out[1] = e * (sr * n01);
  out[2] = e * (sr * n10);
  out[3] = e * (ch - sr * n00);
}

static void free_run(Run* r) {
  if (!r) return;
  for (void* p : r->allocs) (void)hipFree(p);
  for (void* h : r->host_allocs) (void)hipHostFree(h);
  if (r->h_mean) (void)hipHostFree(r->h_mean);
  if (r->h_sem) (void)hipHostFree(r->h_sem);
  if (r->h_stats) (void)hipHostFree(r->h_stats);
  if (r->ev0) (void)hipEventDestroy(r->ev0);
  if (r->ev1) (void)hipEventDestroy(r->ev1);
  if (r->stream && r->own_stream) (void)hipStreamDestroy(r->stream);
  delete r;
}

template <typename T>
static hipError_t upload(Run* r, const std::vector<T>& h, T** dptr) {
  size_t n = std::max<size_t>(h.size(), 1) * sizeof(T);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, n);
  if (e != hipSuccess) return e;
  r->allocs.push_back(p);
  r->bytes += n;
  if (!h.empty()) {
    const void* src = h.data();
    if (r->no_fill) {
      void* pin = nullptr;
      e = hipHostMalloc(&pin, h.size() * sizeof(T), hipHostMallocDefault);
      if (e != hipSuccess) return e;
      r->host_allocs.push_back(pin);
      std::memcpy(pin, h.data(), h.size() * sizeof(T));
      src = pin;
    }
    e = hipMemcpyAsync(p, src, h.size() * sizeof(T), hipMemcpyHostToDevice, r->stream);
  }
  *dptr = (T*)p;
  return e;
}

static hipError_t dalloc(Run* r, size_t n, void** dptr) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(n, 16));
  if (e != hipSuccess) return e;
  r->allocs.push_back(p);
  r->bytes += n;
  if (!r->no_fill) e = hipMemsetAsync(p, 0, std::max<size_t>(n, 16), r->stream);
  *dptr = p;
  return e;
}

static long align256(long x) { return (x + 255) & ~255L; }

namespace {
// Everything a run needs that is computed on the host: validated sizes, the
// kernel parameters except device pointers, the tables to upload and the
// device-memory layout.  No HIP call is made while it is built.
struct Plan {
  TjmParams P;
  long n = 0;
  std::vector<MixEnt> ents;
  std::vector<int> mixL_ptr, mixR_ptr, mix2_ptr, jptr, jidx, optr, oidx, bcap;
  // structured effective Hamiltonians (see the structure section of plan_run)
  std::vector<int> sptr1, schan1, sn1, sptr2, schan2, sn2, env_st, env_en, lr_chan, lr_n;
  std::vector<double> sloc1, sloc2;
  std::vector<int> oD, omix_ptr;        // MPO observables
  std::vector<double> Dh, Df, jopd, initd, obsd, init_t;
  std::vector<long> soff;
  double per_traj = 0;       // device bytes per trajectory (MPS, logs, outputs)
};
}  // namespace

template <typename T>
static double vec_bytes(const std::vector<T>& v) { return (double)std::max<size_t>(v.size(), 1) * sizeof(T); }

static tjm_status plan_run(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                           const int* obs_site, const double* obs_op, uint64_t seed,
                           const tjm_options& opt, Plan& pl) {
  const int L = m->L, d = m->d;
  if (n_traj < 1) return fail(m, TJM_E_INVAL, "n_traj must be >= 1");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(m, TJM_E_INVAL, "dt must be > 0");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(m, TJM_E_INVAL, "T must be > 0");
  const double ratio = T / dt;
  const long n = std::lround(ratio);
  if (n < 1 || std::fabs(ratio - (double)n) > 1e-9 * std::max(1.0, ratio))
    return fail(m, TJM_E_INVAL, "T / dt must be a positive integer");
  if (n > 1000000) return fail(m, TJM_E_INVAL, "too many steps");
  if (chi_max < 1) return fail(m, TJM_E_INVAL, "chi_max must be >= 1");
  if (opt.precision != TJM_PREC_FP64 && opt.precision != TJM_PREC_MIXED)
    return fail(m, TJM_E_INVAL, "unknown precision");
  const int chi_cap = opt.chi_cap > 0 ? opt.chi_cap : chi_max;
  if (chi_cap > 64) return fail(m, TJM_E_UNSUPPORTED, "chi_cap above 64 is not supported");
  if (opt.krylov_max < 1 || opt.krylov_max > 32) return fail(m, TJM_E_INVAL, "krylov_max must be in 1..32");
  if (opt.trotter_order != 1 && opt.trotter_order != 2) return fail(m, TJM_E_INVAL, "trotter_order must be 1 or 2");
  if (opt.tile_mode < 0 || opt.tile_mode > 7) return fail(m, TJM_E_INVAL, "tile_mode must be in 0..7");
  if (opt.sweep_jumps != 1)
    return fail(m, TJM_E_UNSUPPORTED, "only the jump process with the printed sweeps (sweep_jumps = 1) is implemented");
  if (!std::isfinite(opt.svd_discard) || !std::isfinite(opt.deg_tol) || opt.deg_tol < 0)
    return fail(m, TJM_E_INVAL, "svd_discard / deg_tol must be finite");
  if (n_obs < 0 || (n_obs > 0 && (!obs_site || !obs_op))) return fail(m, TJM_E_INVAL, "bad observables");
  for (int i = 0; i < n_obs; ++i)
    if (obs_site[i] < 0 || obs_site[i] >= L) return fail(m, TJM_E_INVAL, "observable site out of range");
  if (n_obs > 0 && !finite_arr(obs_op, 2L * n_obs * d * d)) return fail(m, TJM_E_INVAL, "observable not finite");
  const int n_mobs = (int)m->oW.size();
  const int n_out = n_obs + n_mobs;          // output columns: site observables, then MPO observables
  if ((double)n_traj * (double)(n + 1) * std::max(n_out, 1) > 4e9)
    return fail(m, TJM_E_INVAL, "output too large");
  if ((double)(n + 1) * std::max(n_out, 1) > 2e9) return fail(m, TJM_E_INVAL, "too many output entries per trajectory");
  double tol = opt.krylov_tol;
  if (!(tol > 0.0)) tol = opt.precision == TJM_PREC_MIXED ? 1e-6 : 1e-12;   // mixed: at the FP32 contraction accuracy


  TjmParams& P = pl.P;
  std::memset(&P, 0, sizeof(P));
  pl.n = n;
  P.L = L; P.d = d;
  P.Dmax = *std::max_element(m->mpoD.begin(), m->mpoD.end());
  P.n_traj = n_traj; P.n_steps = (int)n;
  P.chi_max = chi_max; P.chi_cap = chi_cap; P.krylov_max = opt.krylov_max;
  P.n_jump = m->n_jump; P.n_obs = n_out; P.record_bonds = opt.record_bonds ? 1 : 0;
  P.n_site_obs = n_obs; P.n_mpo_obs = n_mobs;
  P.order = opt.trotter_order;
  P.tile_mode = opt.tile_mode;
  P.mixed = opt.precision == TJM_PREC_MIXED ? 1 : 0;
  P.certify = opt.certify_sweeps < 0 ? P.mixed : (opt.certify_sweeps ? 1 : 0);
  P.dt = dt; P.krylov_tol = tol; P.svd_discard = opt.svd_discard; P.deg_tol = opt.deg_tol;
  P.seed = seed; P.traj_base = opt.traj_base;

  // ---- MPO mixing tables -------------------------------------------------
  const int Dm = P.Dmax;
  auto& ents = pl.ents;
  auto& mixL_ptr = pl.mixL_ptr; auto& mixR_ptr = pl.mixR_ptr; auto& mix2_ptr = pl.mix2_ptr;
  mixL_ptr.assign((size_t)L * (Dm * d + 1), 0);
  mixR_ptr.assign((size_t)L * (Dm * d + 1), 0);
  mix2_ptr.assign((size_t)std::max(L - 1, 1) * (Dm * d * d + 1), 0);
  auto push = [&](int w, int s, cd v) {
    MixEnt e; e.w = w; e.s = s; e.re = v.real(); e.im = v.imag();
    ents.push_back(e);
  };
  for (int s = 0; s < L; ++s) {
    const int Dl = m->mpoD[s], Dr = m->mpoD[s + 1];
    const auto& W = m->W[s];
    auto at = [&](int wl, int wr, int so, int si) { return W[(((long)wl * Dr + wr) * d + so) * d + si]; };
    int* rp = &mixL_ptr[(size_t)s * (Dm * d + 1)];
    for (int row = 0; row <= Dm * d; ++row) {
      rp[row] = (int)ents.size();
      if (row == Dm * d || row >= Dr * d) continue;
      const int wr = row / d, so = row % d;
      for (int wl = 0; wl < Dl; ++wl)
        for (int si = 0; si < d; ++si)
          if (at(wl, wr, so, si) != cd(0, 0)) push(wl, si, at(wl, wr, so, si));
    }
    rp = &mixR_ptr[(size_t)s * (Dm * d + 1)];
    for (int row = 0; row <= Dm * d; ++row) {
      rp[row] = (int)ents.size();
      if (row == Dm * d || row >= Dl * d) continue;
      const int wl = row / d, so = row % d;
      for (int wr = 0; wr < Dr; ++wr)
        for (int si = 0; si < d; ++si)
          if (at(wl, wr, so, si) != cd(0, 0)) push(wr, si, at(wl, wr, so, si));
    }
  }
  for (int s = 0; s + 1 < L; ++s) {
    const int Dl = m->mpoD[s], Du = m->mpoD[s + 1], Dr = m->mpoD[s + 2];
    const auto& W1 = m->W[s];
    const auto& W2 = m->W[s + 1];
    int* rp = &mix2_ptr[(size_t)s * (Dm * d * d + 1)];
    for (int row = 0; row <= Dm * d * d; ++row) {
      rp[row] = (int)ents.size();
      if (row == Dm * d * d || row >= Dr * d * d) continue;
      const int wr = row / (d * d), s1o = (row / d) % d, s2o = row % d;
      for (int wl = 0; wl < Dl; ++wl)
        for (int s1 = 0; s1 < d; ++s1)
          for (int s2 = 0; s2 < d; ++s2) {
            cd v = 0;
            for (int u = 0; u < Du; ++u)
              v += W1[(((long)wl * Du + u) * d + s1o) * d + s1] * W2[(((long)u * Dr + wr) * d + s2o) * d + s2];
            if (v != cd(0, 0)) push(wl, s1 * d + s2, v);
          }
    }
  }
  // MPO observables: right-environment rows (w, s_out) -> (w', s_in) per site
  int oDm = 1;
  for (const auto& D : m->omD) oDm = std::max(oDm, *std::max_element(D.begin(), D.end()));
  P.oDmax = oDm;
  pl.oD.clear();
  pl.omix_ptr.assign((size_t)std::max(n_mobs, 1) * L * (oDm * d + 1), 0);
  for (int q = 0; q < n_mobs; ++q) {
    const auto& D = m->omD[q];
    pl.oD.insert(pl.oD.end(), D.begin(), D.end());
    for (int s = 0; s < L; ++s) {
      const int Dl = D[s], Dr = D[s + 1];
      const auto& W = m->oW[q][s];
      int* rp = &pl.omix_ptr[((size_t)q * L + s) * (oDm * d + 1)];
      for (int row = 0; row <= oDm * d; ++row) {
        rp[row] = (int)ents.size();
        if (row == oDm * d || row >= Dl * d) continue;
        const int wl = row / d, so = row % d;
        for (int wr = 0; wr < Dr; ++wr)
          for (int si = 0; si < d; ++si) {
            const cd v = W[(((long)wl * Dr + wr) * d + so) * d + si];
            if (v != cd(0, 0)) push(wr, si, v);
          }
      }
    }
  }


  // ---- structure of the effective Hamiltonians -------------------------------
  // With the sites left of bond b left-canonical, the left environment L_b
  // has a channel st[b] that is exactly the identity (the channel that has
  // only carried W's identity blocks from the left boundary); with the sites
  // right of b right-canonical, R_b has such a channel en[b].  Every block
  // O = W[wl][wr] of a one- or two-site operator then falls in one class:
  //   wl = st, wr = en : O M                        (local)
  //   wl = st          : (O M) R[wr]                (right class)
  //   wr = en          : L[wl] (O M)                (left class)
  //   otherwise        : L[wl] (O M) R[wr]          (two-sided)
  // A nearest-neighbour Hamiltonian has no two-sided block, so H^eff M is
  // two single products, L-side and R-side, plus a local term: no
  // intermediate tensor of D chi d chi elements.  The bond operator keeps
  // its two-sided channels (L[w] C R[w]).  If a site has a two-sided block
  // or an environment has no identity channel, the generic three-stage
  // contraction is used everywhere (structured = 0).
  {
    auto& st = pl.env_st; auto& en = pl.env_en;
    st.assign(L + 1, -1); en.assign(L + 1, -1);
    auto blk = [&](int s, int wl, int wr, int so, int si) {
      const int Dr = m->mpoD[s + 1];
      return m->W[s][(((long)wl * Dr + wr) * d + so) * d + si];
    };
    auto is_id = [&](int s, int wl, int wr) {
      for (int so = 0; so < d; ++so)
        for (int si = 0; si < d; ++si)
          if (blk(s, wl, wr, so, si) != (so == si ? cd(1, 0) : cd(0, 0))) return false;
      return true;
    };
    auto is_zero = [&](int s, int wl, int wr) {
      for (int so = 0; so < d; ++so)
        for (int si = 0; si < d; ++si)
          if (blk(s, wl, wr, so, si) != cd(0, 0)) return false;
      return true;
    };
    st[0] = 0;
    for (int s = 0; s < L && st[s] >= 0; ++s) {
      const int Dl = m->mpoD[s], Dr = m->mpoD[s + 1];
      for (int wr = 0; wr < Dr && st[s + 1] < 0; ++wr) {
        bool ok = is_id(s, st[s], wr);
        for (int wl = 0; wl < Dl && ok; ++wl) ok = wl == st[s] || is_zero(s, wl, wr);
        if (ok) st[s + 1] = wr;
      }
    }
    en[L] = 0;
    for (int s = L - 1; s >= 0 && en[s + 1] >= 0; --s) {
      const int Dl = m->mpoD[s], Dr = m->mpoD[s + 1];
      for (int wl = 0; wl < Dl && en[s] < 0; ++wl) {
        bool ok = is_id(s, wl, en[s + 1]);
        for (int wr = 0; wr < Dr && ok; ++wr) ok = wr == en[s + 1] || is_zero(s, wl, wr);
        if (ok) en[s] = wl;
      }
    }
    bool structured = true;
    // one (dp = d) and two (dp = d^2) site operators: per site a left-class
    // and a right-class list of channels with the physical mixing of each,
    // as CSR rows (batch b, s_out) -> (0, s_in, value), and the local term
    auto classify = [&](int nsite, int s, std::vector<int>& ptr, std::vector<int>& chan, std::vector<int>& cnt,
                        std::vector<double>& loc) {
      const int dp = nsite == 1 ? d : d * d;
      const int Dl = m->mpoD[s], Dr = m->mpoD[s + nsite];
      const int sl = st[s], er = en[s + nsite];
      if (sl < 0 || er < 0) { structured = false; return; }
      // the dp x dp block (wl, wr) of the operator
      auto op = [&](int wl, int wr, int so, int si) {
        if (nsite == 1) return blk(s, wl, wr, so, si);
        cd v = 0;
        const int s1o = so / d, s2o = so % d, s1 = si / d, s2 = si % d;
        for (int u = 0; u < m->mpoD[s + 1]; ++u) {
          const int Du = m->mpoD[s + 1];
          v += m->W[s][(((long)wl * Du + u) * d + s1o) * d + s1] *
               m->W[s + 1][(((long)u * Dr + wr) * d + s2o) * d + s2];
        }
        return v;
      };
      auto nonzero = [&](int wl, int wr) {
        for (int so = 0; so < dp; ++so)
          for (int si = 0; si < dp; ++si)
            if (op(wl, wr, so, si) != cd(0, 0)) return true;
        return false;
      };
      double* lo = &loc[(size_t)s * dp * dp * 2];
      int* pL = &ptr[((size_t)s * 2 + 0) * (Dm * dp + 1)];
      int* pR = &ptr[((size_t)s * 2 + 1) * (Dm * dp + 1)];
      int* cL = &chan[((size_t)s * 2 + 0) * Dm];
      int* cR = &chan[((size_t)s * 2 + 1) * Dm];
      int nL = 0, nR = 0;
      std::vector<int> wls, wrs;
      for (int wl = 0; wl < Dl; ++wl)
        for (int wr = 0; wr < Dr; ++wr) {
          if (!nonzero(wl, wr)) continue;
          if (wl == sl && wr == er) {
            for (int so = 0; so < dp; ++so)
              for (int si = 0; si < dp; ++si) {
                lo[2 * (so * dp + si)] += op(wl, wr, so, si).real();
                lo[2 * (so * dp + si) + 1] += op(wl, wr, so, si).imag();
              }
          } else if (wl == sl) {
            wrs.push_back(wr);
          } else if (wr == er) {
            wls.push_back(wl);
          } else {
            structured = false;
          }
        }
      // left class: batch b is channel wls[b] of L, mixing W[wls[b]][er]
      for (int b = 0; b < (int)wls.size(); ++b) cL[nL++] = wls[b];
      for (int row = 0; row <= Dm * dp; ++row) {
        pL[row] = (int)ents.size();
        if (row == Dm * dp || row / dp >= nL) continue;
        const int wl = cL[row / dp], so = row % dp;
        for (int si = 0; si < dp; ++si)
          if (op(wl, er, so, si) != cd(0, 0)) push(0, si, op(wl, er, so, si));
      }
      for (int b = 0; b < (int)wrs.size(); ++b) cR[nR++] = wrs[b];
      for (int row = 0; row <= Dm * dp; ++row) {
        pR[row] = (int)ents.size();
        if (row == Dm * dp || row / dp >= nR) continue;
        const int wr = cR[row / dp], so = row % dp;
        for (int si = 0; si < dp; ++si)
          if (op(sl, wr, so, si) != cd(0, 0)) push(0, si, op(sl, wr, so, si));
      }
      cnt[(size_t)s * 2 + 0] = nL;
      cnt[(size_t)s * 2 + 1] = nR;
    };
    const int L2 = std::max(L - 1, 1);
    pl.sptr1.assign((size_t)L * 2 * (Dm * d + 1), 0);
    pl.schan1.assign((size_t)L * 2 * Dm, 0);
    pl.sn1.assign((size_t)L * 2, 0);
    pl.sloc1.assign((size_t)L * d * d * 2, 0.0);
    pl.sptr2.assign((size_t)L2 * 2 * (Dm * d * d + 1), 0);
    pl.schan2.assign((size_t)L2 * 2 * Dm, 0);
    pl.sn2.assign((size_t)L2 * 2, 0);
    pl.sloc2.assign((size_t)L2 * d * d * d * d * 2, 0.0);
    for (int s = 0; s < L && structured; ++s) classify(1, s, pl.sptr1, pl.schan1, pl.sn1, pl.sloc1);
    for (int s = 0; s + 1 < L && structured; ++s) classify(2, s, pl.sptr2, pl.schan2, pl.sn2, pl.sloc2);
    // bond operators: the channels of bond b other than st[b] and en[b]
    pl.lr_chan.assign((size_t)(L + 1) * Dm, 0);
    pl.lr_n.assign(L + 1, 0);
    for (int b = 1; b < L && structured; ++b) {
      if (st[b] < 0 || en[b] < 0) { structured = false; break; }
      int n2 = 0;
      for (int w = 0; w < m->mpoD[b]; ++w)
        if (w != st[b] && w != en[b]) pl.lr_chan[(size_t)b * Dm + n2++] = w;
      pl.lr_n[b] = n2;
    }
    P.structured = structured && !opt.generic_heff ? 1 : 0;
  }

  // ---- dissipators, jumps, observables ------------------------------------
  auto& Dh = pl.Dh; auto& Df = pl.Df;
  Dh.assign((size_t)L * 8, 0.0); Df.assign((size_t)L * 8, 0.0);
  for (int s = 0; s < L; ++s) {
    cd G[4] = {0, 0, 0, 0};
    for (int j = 0; j < m->n_jump; ++j) {
      if (m->jsite[j] != s) continue;
      const cd* Lj = &m->jop[(size_t)j * 4];
      for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
          for (int c = 0; c < 2; ++c) G[a * 2 + b] += m->jrate[j] * std::conj(Lj[c * 2 + a]) * Lj[c * 2 + b];
    }
    cd h[4], f[4];
    dissipator2(G, 0.5 * dt, h);
    dissipator2(G, dt, f);
    for (int e = 0; e < 4; ++e) {
      Dh[(size_t)s * 8 + 2 * e] = h[e].real(); Dh[(size_t)s * 8 + 2 * e + 1] = h[e].imag();
      Df[(size_t)s * 8 + 2 * e] = f[e].real(); Df[(size_t)s * 8 + 2 * e + 1] = f[e].imag();
    }
  }
  auto& jptr = pl.jptr; auto& jidx = pl.jidx;
  jptr.assign(L + 1, 0);
  for (int s = 0; s < L; ++s) {
    jptr[s] = (int)jidx.size();
    for (int j = 0; j < m->n_jump; ++j)
      if (m->jsite[j] == s) jidx.push_back(j);
  }
  jptr[L] = (int)jidx.size();
  auto& optr = pl.optr; auto& oidx = pl.oidx;
  optr.assign(L + 1, 0);
  for (int s = 0; s < L; ++s) {
    optr[s] = (int)oidx.size();
    for (int o = 0; o < n_obs; ++o)
      if (obs_site[o] == s) oidx.push_back(o);
  }
  optr[L] = (int)oidx.size();
  auto& jopd = pl.jopd; auto& initd = pl.initd;
  jopd.assign(m->jop.size() * 2, 0.0); initd.assign(m->init.size() * 2, 0.0);
  for (size_t i = 0; i < m->jop.size(); ++i) { jopd[2 * i] = m->jop[i].real(); jopd[2 * i + 1] = m->jop[i].imag(); }
  for (size_t i = 0; i < m->init.size(); ++i) { initd[2 * i] = m->init[i].real(); initd[2 * i + 1] = m->init[i].imag(); }
  pl.obsd.assign(obs_op ? obs_op : (const double*)nullptr, obs_op ? obs_op + 2L * n_obs * d * d : (const double*)nullptr);

  // ---- MPS layout: bond b holds at most min(chi_cap, d^b, d^(L-b)) ----------
  auto& bcap = pl.bcap;
  bcap.assign(L + 1, 0);
  for (int b = 0; b <= L; ++b) {
    long c1 = 1, c2 = 1;
    for (int i = 0; i < b && c1 < chi_cap; ++i) c1 *= d;
    for (int i = 0; i < L - b && c2 < chi_cap; ++i) c2 *= d;
    bcap[b] = (int)std::min<long>(chi_cap, std::min(c1, c2));
  }
  auto& soff = pl.soff;
  soff.assign(L + 1, 0);
  for (int s = 0; s < L; ++s) soff[s + 1] = soff[s] + (long)bcap[s] * d * bcap[s + 1];
  P.mps_cap = std::max<long>(soff[L], 1);
  // Psi(0) as an MPS: bonds within the caps, tensors to the device layout
  auto& init_t = pl.init_t;
  if (!m->init_bond.empty()) {
    for (int b = 0; b <= L; ++b)
      if (m->init_bond[b] > bcap[b])
        return fail(m, TJM_E_INVAL, "initial MPS bond " + std::to_string(b) + " exceeds min(chi_cap, d^l, d^(L-l))");
    init_t.assign(2 * P.mps_cap, 0.0);
    long off = 0;
    for (int l = 0; l < L; ++l) {
      const int a = m->init_bond[l], bb = m->init_bond[l + 1];
      for (int q = 0; q < d; ++q)
        for (int i = 0; i < a; ++i)
          for (int j = 0; j < bb; ++j) {
            const cd x = m->init_mps[off + ((long)q * a + i) * bb + j];    // M_l[s][a][b]
            const long e = soff[l] + ((long)i * d + q) * bb + j;           // device M[a][s][b]
            init_t[2 * e] = x.real(); init_t[2 * e + 1] = x.imag();
          }
      off += (long)d * a * bb;
    }
  }
  const int chic = *std::max_element(bcap.begin(), bcap.end());

  // ---- worker scratch layout ---------------------------------------------
  const long csz = P.mixed ? 8 : 16;
  P.vec_cap = (long)chic * chic * d * d;
  P.env_cap = (long)std::max(Dm, 2) * chic * chic;   // also holds an FP64 chi x chi transfer environment
  P.t_cap = (long)Dm * P.vec_cap;
  P.mat_cap = (long)d * chic * d * chic;
  long o = 0;
  P.off_env = o; o = align256(o + (long)(L + 2) * P.env_cap * csz);
  P.off_smps = o; o = align256(o + P.mps_cap * 16);
  P.off_Q = o; o = align256(o + (long)opt.krylov_max * P.vec_cap * 16);
  P.off_w = o; o = align256(o + P.vec_cap * 16);
  P.off_v = o; o = align256(o + P.vec_cap * 16);
  P.off_T1 = o; o = align256(o + P.t_cap * csz);
  P.off_X = o; o = align256(o + P.mat_cap * 16);
  P.off_Y = o; o = align256(o + P.mat_cap * 16);
  P.off_Z = o; o = align256(o + P.mat_cap * 16);
  P.off_C = o; o = align256(o + P.mat_cap * 16);
  P.off_wts = o; o = align256(o + (long)std::max(m->n_jump, 1) * 8);
  P.oenv_cap = n_mobs ? (long)oDm * chic * chic : 0;
  P.ot_cap = n_mobs ? (long)oDm * chic * d * chic : 0;
  P.off_oenv = o; o = align256(o + 2 * P.oenv_cap * 16);
  P.off_ot = o; o = align256(o + P.ot_cap * 16);
  P.scratch_stride = o;

  pl.per_traj = (double)P.mps_cap * 16 + (L + 1) * 4.0 + (n + 1) * n_out * 8.0 + 2.0 * n * 4 +
                (P.record_bonds ? (double)n * (L + 1) * 4 : 0.0) + TJM_NSTAT * 8 + 4;
  return TJM_OK;
}

// Resident workgroups for a plan on a device: blocks per CU times CUs,
// capped by opt.workers and by the trajectory count.
static tjm_status plan_workers(tjm_model* m, const Plan& pl, const tjm_options& opt, long* workers) {
  hipDeviceProp_t prop;
  HIPCHK(m, hipGetDeviceProperties(&prop, opt.device));
  int bpc = 1;
  HIPCHK(m, tjm_blocks_per_cu(pl.P.mixed, pl.P.L, &bpc));
  if (bpc < 1) return fail(m, TJM_E_UNSUPPORTED, "kernel does not fit on a compute unit");
  long w = (long)bpc * prop.multiProcessorCount;
  if (opt.workers > 0) w = std::min<long>(w, opt.workers);
  *workers = std::min<long>(w, pl.P.n_traj);
  return TJM_OK;
}

static tjm_status select_device(tjm_model* m, const tjm_options& opt) {
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(m, TJM_E_DEVICE, "no HIP device");
  if (opt.device < 0 || opt.device >= ndev) return fail(m, TJM_E_INVAL, "device ordinal out of range");
  HIPCHK(m, hipSetDevice(opt.device));
  return TJM_OK;
}

tjm_status tjm_run_footprint(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                             const int* obs_site, const double* obs_op, const tjm_options* opt_in,
                             size_t* bytes, int* workers) {
  if (!m || !bytes || !workers) return fail(m, TJM_E_INVAL, "NULL argument");
  tjm_options opt;
  tjm_default_options(&opt);
  if (opt_in) opt = *opt_in;
  Plan pl;
  tjm_status st = plan_run(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, 0, opt, pl);
  if (st != TJM_OK) return st;
  if ((st = select_device(m, opt)) != TJM_OK) return st;
  long w = 1;
  if ((st = plan_workers(m, pl, opt, &w)) != TJM_OK) return st;
  double b = vec_bytes(pl.ents) + vec_bytes(pl.mixL_ptr) + vec_bytes(pl.mixR_ptr) + vec_bytes(pl.mix2_ptr) +
             vec_bytes(pl.sptr1) + vec_bytes(pl.schan1) + vec_bytes(pl.sn1) + vec_bytes(pl.sloc1) +
             vec_bytes(pl.sptr2) + vec_bytes(pl.schan2) + vec_bytes(pl.sn2) + vec_bytes(pl.sloc2) +
             vec_bytes(pl.env_st) + vec_bytes(pl.env_en) + vec_bytes(pl.lr_chan) + vec_bytes(pl.lr_n) +
             vec_bytes(pl.Dh) + vec_bytes(pl.Df) + vec_bytes(pl.jopd) + vec_bytes(m->jrate) +
             vec_bytes(m->jsite) + vec_bytes(pl.jptr) + vec_bytes(pl.jidx) + vec_bytes(pl.optr) +
             vec_bytes(pl.oidx) + vec_bytes(pl.obsd) + vec_bytes(pl.initd) + vec_bytes(pl.init_t) +
             vec_bytes(m->init_bond) + vec_bytes(pl.soff) + vec_bytes(pl.bcap) + vec_bytes(m->mpoD) +
             vec_bytes(pl.oD) + vec_bytes(pl.omix_ptr);
  b += pl.per_traj * n_traj + (double)w * pl.P.scratch_stride + 256;
  b += 2.0 * 8 * (pl.n + 1) * std::max(pl.P.n_obs, 1);   // reduction outputs
  b += 64.0 * 1024 * 64;                                  // allocation granularity, 64 allocations
  *bytes = (size_t)b;
  *workers = (int)w;
  return TJM_OK;
}

// Device allocations and uploads of a planned run.  With pool_scratch the
// workers' scratch is that pool (pool_workers slots of pool_stride bytes,
// at least the plan's stride) instead of an allocation of the run's own.
static tjm_status alloc_run(tjm_model* m, Plan& pl, const tjm_options& opt, int n_traj, Run* r,
                            char* pool_scratch, long pool_stride, int pool_workers,
                            hipStream_t pool_stream = nullptr) {
  const int L = m->L;
  const long n = pl.n;
  r->n_traj = n_traj; r->n_steps = (int)n; r->n_obs = pl.P.n_obs; r->record_bonds = pl.P.record_bonds;
  r->use_graph = opt.graph ? 1 : 0;
  r->P = pl.P;
  TjmParams& P = r->P;
  auto bail = [&](tjm_status st, const std::string& msg) { return fail(m, st, msg); };
#define RCHK(expr)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return bail(e_ == hipErrorOutOfMemory ? TJM_E_NOMEM : TJM_E_DEVICE,                      \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                          \
  } while (0)
  if (pool_scratch) {
    if (pool_stride < P.scratch_stride) return bail(TJM_E_INVAL, "job does not fit the scratch pool");
    r->workers = pool_workers;
  } else {
    long workers = 1;
    tjm_status stw = plan_workers(m, pl, opt, &workers);
    if (stw != TJM_OK) return stw;
    size_t freeb = 0, totalb = 0;
    RCHK(hipMemGetInfo(&freeb, &totalb));
    const double avail = 0.85 * (double)freeb - pl.per_traj * n_traj;
    if (avail < (double)P.scratch_stride) return bail(TJM_E_NOMEM, "not enough device memory for the run");
    workers = std::min<long>(workers, (long)(avail / (double)P.scratch_stride));
    r->workers = (int)std::max<long>(workers, 1);
  }
  // ---- uploads ---------------------------------------------------------------
  // Every copy and zero fill is ordered on the run's stream, ahead of the
  // launches, so runs on other streams of the device are not waited for.
  if (pool_scratch) {
    r->no_fill = true;
    r->stream = pool_stream;
    r->own_stream = false;
  } else {
    RCHK(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
  }
  RCHK(hipEventCreate(&r->ev0));
  RCHK(hipEventCreate(&r->ev1));
  RCHK(upload(r, m->mpoD, (int**)&P.mpoD));
  MixEnt* dents = nullptr;
  RCHK(upload(r, pl.ents, &dents));
  P.mixL = dents; P.mixR = dents; P.mix2 = dents;
  RCHK(upload(r, pl.mixL_ptr, (int**)&P.mixL_ptr));
  RCHK(upload(r, pl.mixR_ptr, (int**)&P.mixR_ptr));
  RCHK(upload(r, pl.mix2_ptr, (int**)&P.mix2_ptr));
  RCHK(upload(r, pl.oD, (int**)&P.oD));
  RCHK(upload(r, pl.omix_ptr, (int**)&P.omixR_ptr));
  RCHK(upload(r, pl.sptr1, (int**)&P.s1_ptr));
  RCHK(upload(r, pl.schan1, (int**)&P.s1_chan));
  RCHK(upload(r, pl.sn1, (int**)&P.s1_n));
  RCHK(upload(r, pl.sloc1, (double**)&P.s1_loc));
  RCHK(upload(r, pl.sptr2, (int**)&P.s2_ptr));
  RCHK(upload(r, pl.schan2, (int**)&P.s2_chan));
  RCHK(upload(r, pl.sn2, (int**)&P.s2_n));
  RCHK(upload(r, pl.sloc2, (double**)&P.s2_loc));
  RCHK(upload(r, pl.env_st, (int**)&P.env_st));
  RCHK(upload(r, pl.env_en, (int**)&P.env_en));
  RCHK(upload(r, pl.lr_chan, (int**)&P.lr_chan));
  RCHK(upload(r, pl.lr_n, (int**)&P.lr_n));
  RCHK(upload(r, pl.Dh, (double**)&P.Dhalf));
  RCHK(upload(r, pl.Df, (double**)&P.Dfull));
  RCHK(upload(r, pl.jopd, (double**)&P.jump_op));
  RCHK(upload(r, m->jrate, (double**)&P.jump_rate));
  RCHK(upload(r, m->jsite, (int**)&P.jump_site));
  RCHK(upload(r, pl.jptr, (int**)&P.jptr));
  RCHK(upload(r, pl.jidx, (int**)&P.jidx));
  RCHK(upload(r, pl.optr, (int**)&P.optr));
  RCHK(upload(r, pl.oidx, (int**)&P.oidx));
  RCHK(upload(r, pl.obsd, (double**)&P.obs_op));
  RCHK(upload(r, pl.initd, (double**)&P.init_sites));
  P.init_mps = m->init_bond.empty() ? 0 : 1;
  RCHK(upload(r, pl.init_t, (double**)&P.init_tensors));
  RCHK(upload(r, m->init_bond, (int**)&P.init_bonds));
  RCHK(upload(r, pl.soff, (long**)&P.site_off));
  RCHK(upload(r, pl.bcap, (int**)&P.bond_cap));
  void* p = nullptr;
  RCHK(dalloc(r, (size_t)n_traj * P.mps_cap * 16, &p)); P.mps = (double*)p;
  RCHK(dalloc(r, (size_t)n_traj * (L + 1) * 4, &p)); P.bonds = (int*)p;
  RCHK(dalloc(r, (size_t)n_traj * (n + 1) * std::max(P.n_obs, 1) * 8, &p)); P.obs = (double*)p; r->d_obs = P.obs;
  RCHK(dalloc(r, (size_t)n_traj * 2 * n * 4, &p)); P.jlog = (int*)p; r->d_jlog = P.jlog;
  if (r->record_bonds) {
    RCHK(dalloc(r, (size_t)n_traj * n * (L + 1) * 4, &p)); P.blog = (int*)p; r->d_blog = P.blog;
  }
  RCHK(dalloc(r, (size_t)n_traj * TJM_NSTAT * 8, &p)); P.tstats = (unsigned long long*)p; r->d_stats = P.tstats;
  RCHK(dalloc(r, (size_t)n_traj * 4, &p)); P.tflags = (int*)p; r->d_flags = P.tflags;
  if (pool_scratch) {
    P.scratch = pool_scratch;
    P.scratch_stride = pool_stride;
  } else {
    RCHK(dalloc(r, (size_t)r->workers * P.scratch_stride, &p)); P.scratch = (char*)p;
  }
  RCHK(dalloc(r, 256, &p)); P.counter = (int*)p;
  if (pool_scratch) {
    const size_t entries = (size_t)(n + 1) * std::max(P.n_obs, 1);
    RCHK(hipHostMalloc((void**)&r->h_mean, entries * 8, hipHostMallocCoherent));
    RCHK(hipHostMalloc((void**)&r->h_sem, entries * 8, hipHostMallocCoherent));
    RCHK(hipHostMalloc((void**)&r->h_stats, (TJM_NSTAT + 1) * 8, hipHostMallocCoherent));
    P.serve_mean = r->h_mean;
    P.serve_sem = r->h_sem;
    P.serve_stats = r->h_stats;
  }

  // the host tables of the plan must outlive their copies
  RCHK(hipStreamSynchronize(r->stream));

  return TJM_OK;
#undef RCHK
}

extern "C" tjm_status tjm_run_begin(tjm_model* m, int n_traj, double dt, double T, int chi_max,
                                    int n_obs, const int* obs_site, const double* obs_op,
                                    uint64_t seed, const tjm_options* opt_in) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  if (m->run) return fail(m, TJM_E_BUSY, "a run is already in progress on this model");
  tjm_options opt;
  tjm_default_options(&opt);
  if (opt_in) opt = *opt_in;
  Plan pl;
  tjm_status st0 = plan_run(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, seed, opt, pl);
  if (st0 != TJM_OK) return st0;
  if ((st0 = select_device(m, opt)) != TJM_OK) return st0;
  Run* r = new Run();
  if ((st0 = alloc_run(m, pl, opt, n_traj, r, nullptr, 0, 0)) != TJM_OK) {
    free_run(r);
    return st0;
  }
  TjmParams& P = r->P;
  auto bail = [&](tjm_status st, const std::string& msg) {
    free_run(r);
    return fail(m, st, msg);
  };
#define RCHK(expr)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return bail(e_ == hipErrorOutOfMemory ? TJM_E_NOMEM : TJM_E_DEVICE,                      \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                          \
  } while (0)
  // ---- F_0 ------------------------------------------------------------------
  RCHK(tjm_launch_reset(P.counter, r->stream));
  RCHK(hipEventRecord(r->ev0, r->stream));
  RCHK(tjm_launch_step(P, 0, r->workers, r->stream));
  RCHK(hipEventRecord(r->ev1, r->stream));
  RCHK(hipStreamSynchronize(r->stream));
  float ms = 0;
  RCHK(hipEventElapsedTime(&ms, r->ev0, r->ev1));
  r->init_ms = ms;
  m->run = r;
#undef RCHK
  return TJM_OK;
}

// The launches of `steps` steps captured in one HIP graph on the run's
// stream and replayed once (reset and step kernel per step), with one host
// synchronisation at the end.  Events recorded inside a graph cannot be
// timed, so the replay is bracketed by the run's two events and the steps
// share its duration equally in the statistics.
static tjm_status advance_graph(tjm_model* m, Run* r, int steps) {
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  tjm_status st = TJM_OK;
  std::string msg;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == TJM_OK) {
      st = e == hipErrorOutOfMemory ? TJM_E_NOMEM : TJM_E_DEVICE;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
    return st == TJM_OK;
  };
  if (chk(hipStreamBeginCapture(r->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture")) {
    for (int i = 0; i < steps && st == TJM_OK; ++i) {
      chk(tjm_launch_reset(r->P.counter, r->stream), "reset");
      chk(tjm_launch_step(r->P, r->steps_done + 1 + i, r->workers, r->stream), "step");
    }
    const hipError_t e = hipStreamEndCapture(r->stream, &g);
    chk(e, "hipStreamEndCapture");
  }
  if (st == TJM_OK) chk(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  if (st == TJM_OK) chk(hipEventRecord(r->ev0, r->stream), "hipEventRecord");
  if (st == TJM_OK) chk(hipGraphLaunch(ge, r->stream), "hipGraphLaunch");
  if (st == TJM_OK) chk(hipEventRecord(r->ev1, r->stream), "hipEventRecord");
  if (st == TJM_OK) chk(hipStreamSynchronize(r->stream), "hipStreamSynchronize");
  float ms = 0;
  if (st == TJM_OK) chk(hipEventElapsedTime(&ms, r->ev0, r->ev1), "hipEventElapsedTime");
  if (st == TJM_OK) {
    r->step_ms_last = ms / steps;
    r->step_ms_total += ms;
    r->step_launches += steps;
    r->steps_done += steps;
  }
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  if (st != TJM_OK) return fail(m, st, msg);
  return TJM_OK;
}

extern "C" tjm_status tjm_run_advance(tjm_model* m, int steps) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  Run* r = m->run;
  if (!r) return fail(m, TJM_E_BUSY, "no run in progress");
  if (steps < 0 || r->steps_done + steps > r->n_steps) return fail(m, TJM_E_BUSY, "advance past the last step");
  if (r->use_graph && steps > 0) return advance_graph(m, r, steps);
  for (int i = 0; i < steps; ++i) {
    const int k = r->steps_done + 1;
    HIPCHK(m, tjm_launch_reset(r->P.counter, r->stream));
    HIPCHK(m, hipEventRecord(r->ev0, r->stream));
    HIPCHK(m, tjm_launch_step(r->P, k, r->workers, r->stream));
    HIPCHK(m, hipEventRecord(r->ev1, r->stream));
    HIPCHK(m, hipStreamSynchronize(r->stream));
    float ms = 0;
    HIPCHK(m, hipEventElapsedTime(&ms, r->ev0, r->ev1));
    r->step_ms_last = ms;
    r->step_ms_total += ms;
    r->step_launches++;
    r->steps_done = k;
  }
  return TJM_OK;
}

static void collect_stats(tjm_model* m, Run* r) {
  tjm_stats& s = m->last;
  std::memset(&s, 0, sizeof(s));
  s.n_traj = r->n_traj; s.n_steps = r->n_steps; s.steps_done = r->steps_done; s.workers = r->workers;
  s.init_kernel_ms = r->init_ms;
  s.step_kernel_ms_total = r->step_ms_total;
  s.step_kernel_ms_last = r->step_ms_last;
  s.step_launches = r->step_launches;
  s.device_bytes = r->bytes;
  std::vector<unsigned long long> st((size_t)r->n_traj * TJM_NSTAT);
  if (hipMemcpy(st.data(), r->d_stats, st.size() * 8, hipMemcpyDeviceToHost) != hipSuccess) return;
  for (int t = 0; t < r->n_traj; ++t) {
    const unsigned long long* q = &st[(size_t)t * TJM_NSTAT];
    for (int i = 0; i < 8; ++i) s.phase_s[i] += 1e-8 * (double)q[TJM_ST_T_TOTAL + i];
    s.cmac_mfma += q[TJM_ST_CMAC_MFMA]; s.cmac_mix += q[TJM_ST_CMAC_MIX];
    s.krylov_iters += q[TJM_ST_KRYLOV]; s.expm_calls += q[TJM_ST_EXPM];
    s.one_site += q[TJM_ST_ONE_SITE]; s.two_site += q[TJM_ST_TWO_SITE];
    s.factorizations += q[TJM_ST_FACT]; s.jumps += q[TJM_ST_JUMPS];
  }
  std::vector<int> fl(r->n_traj);
  if (hipMemcpy(fl.data(), r->d_flags, fl.size() * 4, hipMemcpyDeviceToHost) != hipSuccess) return;
  for (int t = 0; t < r->n_traj; ++t) s.failed_traj += fl[t] != 0;
}

extern "C" tjm_status tjm_get_stats(const tjm_model* m, tjm_stats* out) {
  if (!m || !out) return fail(nullptr, TJM_E_INVAL, "NULL argument");
  if (m->run) collect_stats(const_cast<tjm_model*>(m), m->run);
  *out = m->last;
  return TJM_OK;
}

extern "C" tjm_status tjm_run_end(tjm_model* m, double* mean, double* sem, double* per_traj_obs,
                                  int32_t* jump_log, int32_t* bond_log) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  Run* r = m->run;
  if (!r) return fail(m, TJM_E_BUSY, "no run in progress");
  tjm_status st = TJM_OK;
  std::string msg;
  const long entries = (long)(r->n_steps + 1) * r->n_obs;
  auto chk = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && st == TJM_OK) {
      st = TJM_E_DEVICE;
      msg = std::string(what) + ": " + hipGetErrorString(e);
    }
  };
  if (r->steps_done != r->n_steps) { st = TJM_E_BUSY; msg = "run ended before its last step"; }
  if (st == TJM_OK && entries > 0 && (mean || sem)) {
    double *dm = nullptr, *ds = nullptr;
    chk(hipMalloc((void**)&dm, (size_t)entries * 8), "hipMalloc");
    chk(hipMalloc((void**)&ds, (size_t)entries * 8), "hipMalloc");
    if (st == TJM_OK) {
      chk(tjm_launch_reduce(r->d_obs, r->n_traj, entries, dm, ds, r->stream), "reduce");
      chk(hipStreamSynchronize(r->stream), "sync");
      if (mean) chk(hipMemcpy(mean, dm, (size_t)entries * 8, hipMemcpyDeviceToHost), "copy mean");
      if (sem) chk(hipMemcpy(sem, ds, (size_t)entries * 8, hipMemcpyDeviceToHost), "copy sem");
    }
    if (dm) (void)hipFree(dm);
    if (ds) (void)hipFree(ds);
  }
  if (st == TJM_OK && per_traj_obs && entries > 0)
    chk(hipMemcpy(per_traj_obs, r->d_obs, (size_t)r->n_traj * entries * 8, hipMemcpyDeviceToHost), "copy obs");
  if (st == TJM_OK && jump_log)
    chk(hipMemcpy(jump_log, r->d_jlog, (size_t)r->n_traj * 2 * r->n_steps * 4, hipMemcpyDeviceToHost), "copy jlog");
  if (st == TJM_OK && bond_log) {
    if (!r->d_blog) { st = TJM_E_INVAL; msg = "bond_log requested without record_bonds"; }
    else chk(hipMemcpy(bond_log, r->d_blog, (size_t)r->n_traj * r->n_steps * (m->L + 1) * 4, hipMemcpyDeviceToHost), "copy blog");
  }
  if (st == TJM_OK) {
    std::vector<int> fl(r->n_traj);
    chk(hipMemcpy(fl.data(), r->d_flags, (size_t)r->n_traj * 4, hipMemcpyDeviceToHost), "copy flags");
    for (int t = 0; t < r->n_traj && st == TJM_OK; ++t)
      if (fl[t]) { st = TJM_E_NUMERIC; msg = "non-finite norm in trajectory " + std::to_string(t); }
  }
  collect_stats(m, r);
  free_run(r);
  m->run = nullptr;
  if (st != TJM_OK) return fail(m, st, msg);
  return TJM_OK;
}

extern "C" tjm_status tjm_run_read(tjm_model* m, double* per_traj_obs, int32_t* jump_log, int32_t* bond_log) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  Run* r = m->run;
  if (!r) return fail(m, TJM_E_BUSY, "no run in progress");
  if (bond_log && !r->d_blog) return fail(m, TJM_E_INVAL, "bond_log requested without record_bonds");
  const long entries = (long)(r->n_steps + 1) * r->n_obs;
  HIPCHK(m, hipStreamSynchronize(r->stream));
  if (per_traj_obs && entries > 0)
    HIPCHK(m, hipMemcpy(per_traj_obs, r->d_obs, (size_t)r->n_traj * entries * 8, hipMemcpyDeviceToHost));
  if (jump_log)
    HIPCHK(m, hipMemcpy(jump_log, r->d_jlog, (size_t)r->n_traj * 2 * r->n_steps * 4, hipMemcpyDeviceToHost));
  if (bond_log)
    HIPCHK(m, hipMemcpy(bond_log, r->d_blog, (size_t)r->n_traj * r->n_steps * (m->L + 1) * 4, hipMemcpyDeviceToHost));
  return TJM_OK;
}

extern "C" tjm_status tjm_run_traces(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                                     const int* obs_site, const double* obs_op, uint64_t seed,
                                     const tjm_options* opt, double* mean, double* sem, double* per_traj_obs,
                                     int32_t* jump_log, int32_t* bond_log) {
  tjm_status st = tjm_run_begin(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, seed, opt);
  if (st != TJM_OK) return st;
  st = tjm_run_advance(m, m->run->n_steps);
  if (st != TJM_OK) {
    std::string keep = m->err;
    tjm_run_end(m, nullptr, nullptr, nullptr, nullptr, nullptr);
    m->err = keep;
    return st;
  }
  return tjm_run_end(m, mean, sem, per_traj_obs, jump_log, bond_log);
}

extern "C" tjm_status tjm_run(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                              const int* obs_site, const double* obs_op, uint64_t seed,
                              const tjm_options* opt, double* mean, double* sem) {
  return tjm_run_traces(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, seed, opt, mean, sem,
                        nullptr, nullptr, nullptr);
}

// ---- jobs of the pooled server ---------------------------------------------
// A job runs whole trajectories in the server's resident kernel; its workers'
// scratch is the server's pool, so it holds only its own tables, MPSs and
// outputs.

tjm_status tjm_pool_plan(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                         const int* obs_site, const double* obs_op, const tjm_options* opt_in, long* stride,
                         size_t* bytes) {
  if (!m) return fail(nullptr, TJM_E_INVAL, "model is NULL");
  tjm_options opt;
  tjm_default_options(&opt);
  if (opt_in) opt = *opt_in;
  Plan pl;
  tjm_status st = plan_run(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, 0, opt, pl);
  if (st != TJM_OK) return st;
  if (opt.graph) return fail(m, TJM_E_INVAL, "graph capture does not apply to server jobs");
  double b = vec_bytes(pl.ents) + vec_bytes(pl.mixL_ptr) + vec_bytes(pl.mixR_ptr) + vec_bytes(pl.mix2_ptr) +
             vec_bytes(pl.sptr1) + vec_bytes(pl.schan1) + vec_bytes(pl.sn1) + vec_bytes(pl.sloc1) +
             vec_bytes(pl.sptr2) + vec_bytes(pl.schan2) + vec_bytes(pl.sn2) + vec_bytes(pl.sloc2) +
             vec_bytes(pl.env_st) + vec_bytes(pl.env_en) + vec_bytes(pl.lr_chan) + vec_bytes(pl.lr_n) +
             vec_bytes(pl.Dh) + vec_bytes(pl.Df) + vec_bytes(pl.jopd) + vec_bytes(m->jrate) +
             vec_bytes(m->jsite) + vec_bytes(pl.jptr) + vec_bytes(pl.jidx) + vec_bytes(pl.optr) +
             vec_bytes(pl.oidx) + vec_bytes(pl.obsd) + vec_bytes(pl.initd) + vec_bytes(pl.init_t) +
             vec_bytes(m->init_bond) + vec_bytes(pl.soff) + vec_bytes(pl.bcap) + vec_bytes(m->mpoD) +
             vec_bytes(pl.oD) + vec_bytes(pl.omix_ptr);
  b += pl.per_traj * n_traj + 256;
  b += 2.0 * 8 * (pl.n + 1) * std::max(pl.P.n_obs, 1);
  b += 64.0 * 1024 * 64;
  *stride = pl.P.scratch_stride;
  *bytes = (size_t)b;
  return TJM_OK;
}

tjm_status tjm_pool_prepare(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                            const int* obs_site, const double* obs_op, uint64_t seed, const tjm_options* opt_in,
                            char* scratch, long stride, int workers, TjmParams* d_slot, hipStream_t stream,
                            void** job, TjmParams* Pout) {
  if (!m || !job || !Pout || !scratch || !d_slot || !stream) return fail(m, TJM_E_INVAL, "NULL argument");
  tjm_options opt;
  tjm_default_options(&opt);
  if (opt_in) opt = *opt_in;
  Plan pl;
  tjm_status st = plan_run(m, n_traj, dt, T, chi_max, n_obs, obs_site, obs_op, seed, opt, pl);
  if (st != TJM_OK) return st;
  if ((st = select_device(m, opt)) != TJM_OK) return st;
  Run* r = new Run();
  if ((st = alloc_run(m, pl, opt, n_traj, r, scratch, stride, workers, stream)) != TJM_OK) {
    free_run(r);
    return st;
  }
  // the kernel parameters into the server's slot, on the same stream
  void* pin = nullptr;
  hipError_t e = hipHostMalloc(&pin, sizeof(TjmParams), hipHostMallocDefault);
  if (e == hipSuccess) {
    r->host_allocs.push_back(pin);
    std::memcpy(pin, &r->P, sizeof(TjmParams));
    e = hipMemcpyAsync(d_slot, pin, sizeof(TjmParams), hipMemcpyHostToDevice, r->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(r->stream);   // tables uploaded
  if (e != hipSuccess) {
    free_run(r);
    return fail(m, TJM_E_DEVICE, std::string("job upload: ") + hipGetErrorString(e));
  }
  *job = r;
  *Pout = r->P;
  return TJM_OK;
}

tjm_status tjm_pool_finish(tjm_model* m, void* job, double* mean, double* sem, tjm_stats* stats) {
  Run* r = (Run*)job;
  if (!m || !r) return fail(m, TJM_E_INVAL, "NULL argument");
  // the serve kernel has reduced the job into r's host-coherent buffers; no
  // device work here (the resident kernel may still be running)
  tjm_stats& s = m->last;
  std::memset(&s, 0, sizeof(s));
  s.n_traj = r->n_traj; s.n_steps = r->n_steps; s.steps_done = r->n_steps; s.workers = r->workers;
  s.device_bytes = r->bytes;
  const unsigned long long* q = r->h_stats;
  for (int i = 0; i < 8; ++i) s.phase_s[i] = 1e-8 * (double)q[TJM_ST_T_TOTAL + i];
  s.cmac_mfma = q[TJM_ST_CMAC_MFMA]; s.cmac_mix = q[TJM_ST_CMAC_MIX];
  s.krylov_iters = q[TJM_ST_KRYLOV]; s.expm_calls = q[TJM_ST_EXPM];
  s.one_site = q[TJM_ST_ONE_SITE]; s.two_site = q[TJM_ST_TWO_SITE];
  s.factorizations = q[TJM_ST_FACT]; s.jumps = q[TJM_ST_JUMPS];
  s.failed_traj = (int)q[TJM_NSTAT];
  if (stats) *stats = s;
  if (s.failed_traj) return fail(m, TJM_E_NUMERIC, std::to_string(s.failed_traj) + " trajectories with a non-finite norm");
  const size_t entries = (size_t)(r->n_steps + 1) * r->n_obs;
  if (mean && entries) std::memcpy(mean, r->h_mean, entries * 8);
  if (sem && entries) std::memcpy(sem, r->h_sem, entries * 8);
  return TJM_OK;
}

void tjm_pool_release(void* job) { free_run((Run*)job); }

extern "C" const char* tjm_last_error(const tjm_model* m) {
  return m ? m->err.c_str() : g_create_err.c_str();
}

tjm_model* tjm_model_copy(const tjm_model* m) {
  if (!m) return nullptr;
  tjm_model* c = new (std::nothrow) tjm_model();
  if (!c) return nullptr;
  try {
    c->L = m->L; c->d = m->d; c->mpoD = m->mpoD; c->W = m->W;
    c->n_jump = m->n_jump; c->jsite = m->jsite; c->jop = m->jop; c->jrate = m->jrate;
    c->init = m->init; c->init_bond = m->init_bond; c->init_mps = m->init_mps;
    c->omD = m->omD; c->oW = m->oW;
  } catch (...) {
    delete c;
    return nullptr;
  }
  return c;
}

int tjm_model_d(const tjm_model* m) { return m ? m->d : 0; }
int tjm_model_n_mpo_obs(const tjm_model* m) { return m ? (int)m->oW.size() : 0; }
int tjm_model_L(const tjm_model* m) { return m ? m->L : 0; }
int tjm_model_Dmax(const tjm_model* m) {
  return m && !m->mpoD.empty() ? *std::max_element(m->mpoD.begin(), m->mpoD.end()) : 0;
}
tjm_status tjm_model_fail(tjm_model* m, tjm_status st, const char* msg) { return fail(m, st, msg); }
int tjm_model_busy(const tjm_model* m) { return m && m->run ? 1 : 0; }

extern "C" void tjm_destroy(tjm_model* m) {
  if (!m) return;
  free_run(m->run);
  delete m;
}

// --------------------------------------------------------------------------
// self-test entry points
// --------------------------------------------------------------------------
namespace {
struct DevScope {
  std::vector<void*> ps;
  ~DevScope() { for (void* p : ps) (void)hipFree(p); }
  template <typename T> hipError_t put(const T* h, long n, T** d) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<long>(n, 1) * sizeof(T));
    if (e != hipSuccess) return e;
    ps.push_back(p);
    *d = (T*)p;
    if (h && n > 0) return hipMemcpy(p, h, n * sizeof(T), hipMemcpyHostToDevice);
    return hipMemset(p, 0, std::max<long>(n, 1) * sizeof(T));
  }
};
}  // namespace

#define STCHK(expr)                                                         \
  do {                                                                      \
    hipError_t e_ = (expr);                                                 \
    if (e_ != hipSuccess) return fail(nullptr, TJM_E_DEVICE, hipGetErrorString(e_)); \
  } while (0)

extern "C" tjm_status tjm_selftest_cgemm(int precision, int M, int N, int K, int nb, int sum_batches,
                                         const double* A, int lda, long bsA, int transA, int conjA,
                                         const double* B, int ldb, long bsB, int transB, int conjB,
                                         double* C, int ldc, long csC, int accumulate,
                                         long a_elems, long b_elems, long c_elems) {
  if (M < 1 || N < 1 || K < 1 || M > 512 || N > 512 || K > 512 || nb < 1 || nb > 16)
    return fail(nullptr, TJM_E_INVAL, "gemm sizes out of range");
  if (!A || !B || !C || a_elems < 1 || b_elems < 1 || c_elems < 1) return fail(nullptr, TJM_E_INVAL, "NULL buffer");
  // every addressed element must be inside the buffers
  long amax = (long)(nb - 1) * bsA + (transA ? (long)(K - 1) * lda + (M - 1) : (long)(M - 1) * lda + (K - 1));
  long bmax = (long)(nb - 1) * bsB + (transB ? (long)(N - 1) * ldb + (K - 1) : (long)(K - 1) * ldb + (N - 1));
  long cmax = (long)(sum_batches ? 0 : nb - 1) * csC + (long)(M - 1) * ldc + (N - 1);
  if (amax >= a_elems || bmax >= b_elems || cmax >= c_elems || bsA < 0 || bsB < 0 || csC < 0)
    return fail(nullptr, TJM_E_INVAL, "gemm operand out of buffer bounds");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, TJM_E_DEVICE, "no HIP device");
  DevScope ds;
  double *dA, *dB, *dC;
  STCHK(ds.put(A, 2 * a_elems, &dA));
  STCHK(ds.put(B, 2 * b_elems, &dB));
  STCHK(ds.put(C, 2 * c_elems, &dC));
  STCHK(tjm_launch_st_cgemm(precision == TJM_PREC_MIXED, M, N, K, nb, sum_batches, dA, lda, bsA, transA, conjA,
                            dB, ldb, bsB, transB, conjB, dC, ldc, csC, accumulate));
  STCHK(hipDeviceSynchronize());
  STCHK(hipMemcpy(C, dC, 2 * c_elems * 8, hipMemcpyDeviceToHost));
  return TJM_OK;
}

extern "C" tjm_status tjm_selftest_qr(int m, int n, const double* X, double* Q, double* R) {
  if (m < 1 || n < 1 || m > 128 || n > 128 || !X || !Q || !R) return fail(nullptr, TJM_E_INVAL, "qr sizes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, TJM_E_DEVICE, "no HIP device");
  const int k = std::min(m, n);
  DevScope ds;
  double *dX, *dQ, *dR, *dV;
  STCHK(ds.put(X, 2L * m * n, &dX));
  STCHK(ds.put((const double*)nullptr, 2L * m * k, &dQ));
  STCHK(ds.put((const double*)nullptr, 2L * k * n, &dR));
  STCHK(ds.put((const double*)nullptr, 2L * m * k, &dV));
  STCHK(tjm_launch_st_qr(m, n, dX, dQ, dR, dV));
  STCHK(hipDeviceSynchronize());
  STCHK(hipMemcpy(Q, dQ, 2L * m * k * 8, hipMemcpyDeviceToHost));
  STCHK(hipMemcpy(R, dR, 2L * k * n * 8, hipMemcpyDeviceToHost));
  return TJM_OK;
}

extern "C" tjm_status tjm_selftest_svd(int m, int n, const double* G, double discard, int cap, double deg_tol,
                                       int absorb_left, double* left, double* right, double* S, int* k) {
  if (m < 1 || n < 1 || (absorb_left ? m : n) > 128 || std::max(m, n) > 256 || cap < 1 || !G || !left || !right ||
      !S || !k)
    return fail(nullptr, TJM_E_INVAL, "svd sizes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, TJM_E_DEVICE, "no HIP device");
  const int nc = absorb_left ? m : n, p = absorb_left ? n : m;
  DevScope ds;
  double *dG, *dl, *dr, *dS, *dW, *dU, *dT;
  int* dk;
  STCHK(ds.put(G, 2L * m * n, &dG));
  STCHK(ds.put((const double*)nullptr, 2L * m * nc, &dl));
  STCHK(ds.put((const double*)nullptr, 2L * nc * n, &dr));
  STCHK(ds.put((const double*)nullptr, nc, &dS));
  STCHK(ds.put((const double*)nullptr, 2L * p * nc, &dW));
  STCHK(ds.put((const double*)nullptr, 2L * nc * p, &dU));
  STCHK(ds.put((const double*)nullptr, 2L * m * n, &dT));
  STCHK(ds.put((const int*)nullptr, 1, &dk));
  STCHK(tjm_launch_st_svd(m, n, dG, discard, cap, deg_tol, absorb_left, dl, dr, dS, dk, dW, dU, dT, 0));
  STCHK(hipDeviceSynchronize());
  STCHK(hipMemcpy(k, dk, 4, hipMemcpyDeviceToHost));
  const int kk = *k;
  STCHK(hipMemcpy(left, dl, 2L * m * kk * 8, hipMemcpyDeviceToHost));
  STCHK(hipMemcpy(right, dr, 2L * kk * n * 8, hipMemcpyDeviceToHost));
  STCHK(hipMemcpy(S, dS, (long)kk * 8, hipMemcpyDeviceToHost));
  return TJM_OK;
}

extern "C" tjm_status tjm_selftest_expm(int n, const double* H, const double* v, double t, int krylov_max,
                                        double tol, double* out, int* iters) {
  if (n < 1 || n > 512 || krylov_max < 1 || krylov_max > 32 || !H || !v || !out || !iters)
    return fail(nullptr, TJM_E_INVAL, "expm sizes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, TJM_E_DEVICE, "no HIP device");
  DevScope ds;
  double *dH, *dv, *dQ, *dw;
  int* dit;
  STCHK(ds.put(H, 2L * n * n, &dH));
  STCHK(ds.put(v, 2L * n, &dv));
  STCHK(ds.put((const double*)nullptr, 2L * n * krylov_max, &dQ));
  STCHK(ds.put((const double*)nullptr, 2L * n, &dw));
  STCHK(ds.put((const int*)nullptr, 1, &dit));
  STCHK(tjm_launch_st_expm(n, dH, dv, t, krylov_max, tol, dQ, dw, dit));
  STCHK(hipDeviceSynchronize());
  STCHK(hipMemcpy(out, dv, 2L * n * 8, hipMemcpyDeviceToHost));
  STCHK(hipMemcpy(iters, dit, 4, hipMemcpyDeviceToHost));
  return TJM_OK;
}

extern "C" tjm_status tjm_selftest_philox(int count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out) {
  if (count < 1 || count > (1 << 20) || !ctr || !out) return fail(nullptr, TJM_E_INVAL, "philox sizes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, TJM_E_DEVICE, "no HIP device");
  DevScope ds;
  uint32_t *dc, *dout;
  STCHK(ds.put(ctr, 4L * count, &dc));
  STCHK(ds.put((const uint32_t*)nullptr, 4L * count, &dout));
  STCHK(tjm_launch_st_philox(count, dc, k0, k1, dout));
  STCHK(hipDeviceSynchronize());
  STCHK(hipMemcpy(out, dout, 16L * count, hipMemcpyDeviceToHost));
  return TJM_OK;
}

extern "C" tjm_status tjm_selftest_copy(long n_bytes, int reps, double* avg_ms) {
  if (n_bytes < 16 || n_bytes % 16 != 0 || n_bytes > (16L << 30) || reps < 1 || reps > 1000 || !avg_ms)
    return fail(nullptr, TJM_E_INVAL, "copy sizes");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(nullptr, TJM_E_DEVICE, "no HIP device");
  DevScope ds;
  char *src, *dst;
  STCHK(ds.put((const char*)nullptr, n_bytes, &src));
  STCHK(ds.put((const char*)nullptr, n_bytes, &dst));
  hipDeviceProp_t prop;
  STCHK(hipGetDeviceProperties(&prop, 0));
  hipEvent_t e0, e1;
  STCHK(hipEventCreate(&e0));
  STCHK(hipEventCreate(&e1));
  STCHK(hipDeviceSynchronize());
  STCHK(hipEventRecord(e0, 0));
  for (int i = 0; i < reps; ++i) STCHK(tjm_launch_st_copy(src, dst, n_bytes / 16, 8 * prop.multiProcessorCount, 0));
  STCHK(hipEventRecord(e1, 0));
  STCHK(hipEventSynchronize(e1));
  float ms = 0;
  STCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *avg_ms = ms / reps;
  return TJM_OK;
}
