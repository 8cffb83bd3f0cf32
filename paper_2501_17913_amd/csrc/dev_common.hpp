// Complex arithmetic, deterministic workgroup reductions and the
// counter-based random stream used by the jump process.
#pragma once
#include <dev_platform.hpp>

template <typename T> struct cplx { T re, im; };

template <typename T> TJM_DEV cplx<T> cmk(T r, T i) { cplx<T> z; z.re = r; z.im = i; return z; }
template <typename T> TJM_DEV cplx<T> operator+(cplx<T> a, cplx<T> b) { return cmk(a.re + b.re, a.im + b.im); }
template <typename T> TJM_DEV cplx<T> operator-(cplx<T> a, cplx<T> b) { return cmk(a.re - b.re, a.im - b.im); }
template <typename T> TJM_DEV cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T> TJM_DEV cplx<T> operator*(T s, cplx<T> a) { return cmk(s * a.re, s * a.im); }
template <typename T> TJM_DEV cplx<T> conjg(cplx<T> a) { return cmk(a.re, -a.im); }
template <typename T> TJM_DEV T abs2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
// conj(a) * b
template <typename T> TJM_DEV cplx<T> cdotc(cplx<T> a, cplx<T> b) {
  return cmk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T, typename S> TJM_DEV cplx<T> ccast(cplx<S> a) { return cmk((T)a.re, (T)a.im); }

typedef cplx<double> zd;
typedef cplx<float> zf;

// Load of element i of a complex array in global memory.  The pointer is
// cast to the global address space: inside a separately compiled device
// function a pointer argument is generic, and a generic (flat) load is
// counted by the LDS wait counter too, so every wait for an LDS read would
// also wait for it; a global load is not.
template <typename S> TJM_DEV cplx<S> gload(const cplx<S>* p, long i) {
  typedef S v2 __attribute__((ext_vector_type(2)));
  typedef const __attribute__((address_space(1))) v2 gv2;
  const v2 v = ((gv2*)p)[i];
  return cmk(v.x, v.y);
}

// Store of element i of a complex array in global memory (same reason).
template <typename S> TJM_DEV void gstore(cplx<S>* p, long i, cplx<S> x) {
  typedef S v2 __attribute__((ext_vector_type(2)));
  typedef __attribute__((address_space(1))) v2 gv2;
  v2 v;
  v.x = x.re;
  v.y = x.im;
  ((gv2*)p)[i] = v;
}

// The same for any trivially copyable value (tables of the run).
template <typename V> TJM_DEV V gload_v(const V* p, long i) {
  typedef const __attribute__((address_space(1))) V gV;
  return ((gV*)p)[i];
}

// c ? a : b on complex values, as two scalar selects (a conditional on
// struct lvalues becomes a select of addresses, which keeps a register
// array in scratch memory)
template <typename T> TJM_DEV cplx<T> csel(bool c, cplx<T> a, cplx<T> b) {
  return cmk(c ? a.re : b.re, c ? a.im : b.im);
}

// LDS scratch every workgroup routine may use for reductions and broadcasts.
struct BlkScratch {
  double red[TJM_NWAVE * 4];
  double bcast[8];
  int ibcast[8];
};

// Sum of one double over the workgroup; every thread receives it.  The order
// of additions is fixed (butterfly in each wavefront, then waves in order),
// so the result does not depend on scheduling.
TJM_DEV double blk_sum(double v, BlkScratch& S) {
  v = tjm_grp_sum<TJM_WAVE>(v);
  if (tjm_lane() == 0) S.red[tjm_wave()] = v;
  tjm_sync();
  double s = 0.0;
  for (int w = 0; w < TJM_NWAVE; ++w) s += S.red[w];
  tjm_sync();
  return s;
}

// Two (or up to four) simultaneous sums.
TJM_DEV void blk_sum2(double& a, double& b, BlkScratch& S) {
  a = tjm_grp_sum<TJM_WAVE>(a);
  b = tjm_grp_sum<TJM_WAVE>(b);
  if (tjm_lane() == 0) { S.red[2 * tjm_wave()] = a; S.red[2 * tjm_wave() + 1] = b; }
  tjm_sync();
  double sa = 0.0, sb = 0.0;
  for (int w = 0; w < TJM_NWAVE; ++w) { sa += S.red[2 * w]; sb += S.red[2 * w + 1]; }
  tjm_sync();
  a = sa; b = sb;
}

TJM_DEV void blk_sum4(double& a, double& b, double& c, double& d, BlkScratch& S) {
  a = tjm_grp_sum<TJM_WAVE>(a); b = tjm_grp_sum<TJM_WAVE>(b);
  c = tjm_grp_sum<TJM_WAVE>(c); d = tjm_grp_sum<TJM_WAVE>(d);
  if (tjm_lane() == 0) {
    S.red[4 * tjm_wave()] = a; S.red[4 * tjm_wave() + 1] = b;
    S.red[4 * tjm_wave() + 2] = c; S.red[4 * tjm_wave() + 3] = d;
  }
  tjm_sync();
  double sa = 0, sb = 0, sc = 0, sd = 0;
  for (int w = 0; w < TJM_NWAVE; ++w) {
    sa += S.red[4 * w]; sb += S.red[4 * w + 1]; sc += S.red[4 * w + 2]; sd += S.red[4 * w + 3];
  }
  tjm_sync();
  a = sa; b = sb; c = sc; d = sd;
}

// Sum of v over groups of g consecutive lanes (g a power of two <= 64, a
// run-time value); all lanes of the group receive the group's sum.
template <int G>
TJM_DEV void grp_sum4_t(double& a, double& b, double& c, double& d) {
  a = tjm_grp_sum<G>(a); b = tjm_grp_sum<G>(b); c = tjm_grp_sum<G>(c); d = tjm_grp_sum<G>(d);
}

TJM_DEV void grp_sum4(double& a, double& b, double& c, double& d, int g) {
  switch (g) {
    case 1: break;
    case 2: grp_sum4_t<2>(a, b, c, d); break;
    case 4: grp_sum4_t<4>(a, b, c, d); break;
    case 8: grp_sum4_t<8>(a, b, c, d); break;
    case 16: grp_sum4_t<16>(a, b, c, d); break;
    case 32: grp_sum4_t<32>(a, b, c, d); break;
    default: grp_sum4_t<64>(a, b, c, d); break;
  }
}

TJM_DEV void grp_sum2(double& a, double& b, int g) {
  double c = 0.0, d = 0.0;
  grp_sum4(a, b, c, d, g);
}

TJM_DEV double grp_sum(double v, int g) {
  double b = 0.0, c = 0.0, d = 0.0;
  grp_sum4(v, b, c, d, g);
  return v;
}

// --------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of
// (c0,c1,c2,c3) -> (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)),
// key bumped by the golden-ratio Weyl constants between rounds.
// Stream layout of the jump process: key = (seed lo, seed hi), counter =
// (trajectory, step, branch, 0); branch 0 = jump process of the sampling
// MPS (step 0 is F_0), branch 1 = the sampling layer applied at that step.
// --------------------------------------------------------------------------
TJM_DEV void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint32_t hi0 = tjm_mulhi(M0, c[0]), lo0 = M0 * c[0];
    uint32_t hi1 = tjm_mulhi(M1, c[2]), lo1 = M1 * c[2];
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

TJM_DEV double u53(uint32_t a, uint32_t b) {
  return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
}

TJM_DEV void tjm_draws(uint64_t seed, uint32_t traj, uint32_t step, uint32_t branch,
                       double& eps, double& r) {
  uint32_t c[4] = {traj, step, branch, 0u};
  philox4x32_10(c, (uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32));
  eps = u53(c[0], c[1]);
  r = u53(c[2], c[3]);
}

// Mean and standard error over trajectories of entry e of obs[n_traj][entries]
// (Eq. TJMExpVal), the trajectories summed in index order: the same
// arithmetic wherever a job's outputs are reduced.
TJM_DEV void tjm_reduce_entry(const double* obs, int n_traj, long entries, long e, double* mean, double* sem) {
  double s = 0.0;
  for (int t = 0; t < n_traj; ++t) s += obs[(long)t * entries + e];
  const double mu = s / n_traj;
  double q = 0.0;
  for (int t = 0; t < n_traj; ++t) {
    const double x = obs[(long)t * entries + e] - mu;
    q += x * x;
  }
  mean[e] = mu;
  sem[e] = n_traj > 1 ? sqrt(q / ((double)(n_traj - 1) * n_traj)) : 0.0;
}
