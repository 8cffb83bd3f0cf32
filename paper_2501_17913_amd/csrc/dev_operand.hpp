// Operands of the workgroup GEMM.
//
// An operand is any object with
//   bool trans;                      which index is contiguous
//   typedef ... raw_t;               one staged element between its load
//                                    and its store to LDS
//   template <int NE> void fetch(int b, const int* i, const int* k,
//                                const bool* ok, raw_t* r) const;
//   template <typename T> cplx<T> value(const raw_t& r, bool ok) const;
//   template <typename T> cplx<T> get(int b, int i, int k) const;
// fetch issues the loads of NE elements of batch b and returns without
// waiting for them: the address of an element outside the product (ok
// false) is clamped into the operand, so that every load is unconditional
// and all of them are in flight together.  value converts a loaded element
// to the compute type T, zero where ok is false; the GEMM calls it only when
// it stores the chunk to LDS, so the next chunk's loads overlap the current
// chunk on the matrix cores.  get returns one element (i, k) of batch b,
// which must be in range.  trans = false means k (the second index) runs
// contiguously in memory, trans = true means i does; the stager walks the
// contiguous index across neighbouring threads.
#pragma once
#include <dev_common.hpp>
#include "tjm_params.h"

// A stored complex matrix: op(X) with X row-major (leading dimension ld) as
// cplx<S>; batch b starts bs elements after batch b-1.
//   trans = false: op(X)[i][k] = X[i][k]     trans = true: op(X)[i][k] = X[k][i]
//   conj applies complex conjugation on top.
template <typename S> struct CMat {
  typedef cplx<S> raw_t;
  const cplx<S>* p;
  int ld;
  long bs;
  bool trans;
  bool conj;
  TJM_DEV long off(int i, int k) const { return trans ? ((long)k * ld + i) : ((long)i * ld + k); }
  template <typename T> TJM_DEV cplx<T> get(int b, int i, int k) const {
    const cplx<S> v = gload(p, (long)b * bs + off(i, k));
    return cmk((T)v.re, conj ? (T)(-v.im) : (T)v.im);
  }
  template <int NE>
  TJM_DEV void fetch(int b, const int* ii, const int* kk, const bool* ok, raw_t* r) const {
    const cplx<S>* base = p + (long)b * bs;
#pragma unroll
    for (int u = 0; u < NE; ++u) r[u] = gload(base, ok[u] ? off(ii[u], kk[u]) : 0L);
  }
  template <typename T> TJM_DEV cplx<T> value(const raw_t& v, bool ok) const {
    const T re = (T)v.re, im = conj ? (T)(-v.im) : (T)v.im;
    return cmk(ok ? re : (T)0, ok ? im : (T)0);
  }
};

template <typename S> TJM_DEV CMat<S> cmat(const cplx<S>* p, int ld, long bs = 0,
                                           bool trans = false, bool conj = false) {
  CMat<S> m; m.p = p; m.ld = ld; m.bs = bs; m.trans = trans; m.conj = conj; return m;
}

// A stack of row-major matrices (ld, consecutive matrices cs elements
// apart) of which batch b takes matrix chan[b]: the channels of an
// environment that one class of effective-Hamiltonian terms uses.
template <typename S> struct ChanMat {
  typedef cplx<S> raw_t;
  const cplx<S>* p;
  int ld;
  long cs;
  const int* chan;
  bool trans;
  template <typename T> TJM_DEV cplx<T> get(int b, int i, int k) const {
    const cplx<S> v = gload(p, (long)gload_v(chan, b) * cs + (long)i * ld + k);
    return cmk((T)v.re, (T)v.im);
  }
  template <int NE>
  TJM_DEV void fetch(int b, const int* ii, const int* kk, const bool* ok, raw_t* r) const {
    const cplx<S>* base = p + (long)gload_v(chan, b) * cs;
#pragma unroll
    for (int u = 0; u < NE; ++u) r[u] = gload(base, ok[u] ? (long)ii[u] * ld + kk[u] : 0L);
  }
  template <typename T> TJM_DEV cplx<T> value(const raw_t& v, bool ok) const {
    return cmk(ok ? (T)v.re : (T)0, ok ? (T)v.im : (T)0);
  }
};

template <typename S> TJM_DEV ChanMat<S> chan_mat(const cplx<S>* p, int ld, long cs, const int* chan) {
  ChanMat<S> m; m.p = p; m.ld = ld; m.cs = cs; m.chan = chan; m.trans = false; return m;
}

// one mixing entry, loaded field by field from global memory
TJM_DEV MixEnt gload_ent(const MixEnt* ent, int q) {
  const MixEnt* e = ent + q;
  MixEnt m;
  m.w = gload_v(&e->w, 0);
  m.s = gload_v(&e->s, 0);
  m.re = gload_v(&e->re, 0);
  m.im = gload_v(&e->im, 0);
  return m;
}

// sum over the nonzeros (wi, si, v) of one mixing row of v * x(wi, si)
template <typename T, typename S>
TJM_DEV cplx<T> mix_row(const int* rp, const MixEnt* ent, int row, const cplx<S>* base, long sw, long ss) {
  T xr = 0, xi = 0;
  const int q1 = gload_v(rp, row + 1);
  for (int q = gload_v(rp, row); q < q1; ++q) {
    const MixEnt m = gload_ent(ent, q);
    const cplx<S> x = gload(base, (long)m.w * sw + (long)m.s * ss);
    const T mr = (T)m.re, mi = (T)m.im;
    xr += mr * (T)x.re - mi * (T)x.im;
    xi += mr * (T)x.im + mi * (T)x.re;
  }
  return cmk(xr, xi);
}

// NE mixed elements, in FP64; element u sums row row[u] at offset base[u].
// When all rows agree (the staging layouts make them agree) the row's
// nonzeros are read once and the NE source loads of each nonzero are issued
// together (clamped to the start of the source where ok is false).
template <typename S, int NE>
TJM_DEV void mix_fetch(const int* rp, const MixEnt* ent, const cplx<S>* src, long sw, long ss,
                       const int* row, const int* base, const bool* ok, zd* out) {
  // only in-range elements name a mixing row (an out-of-range one may not)
  int r0 = -1;
  bool same = true;
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    out[u] = cmk(0.0, 0.0);
    if (!ok[u]) continue;
    if (r0 < 0) r0 = row[u];
    else same = same && row[u] == r0;
  }
  if (r0 < 0) return;
  if (same) {
    const int q1 = gload_v(rp, r0 + 1);
    for (int q = gload_v(rp, r0); q < q1; ++q) {
      const MixEnt m = gload_ent(ent, q);
      const long off = (long)m.w * sw + (long)m.s * ss;
      cplx<S> x[NE];
#pragma unroll
      for (int u = 0; u < NE; ++u) x[u] = gload(src, ok[u] ? base[u] + off : off);
#pragma unroll
      for (int u = 0; u < NE; ++u) {
        const double xr = ok[u] ? (double)x[u].re : 0.0, xi = ok[u] ? (double)x[u].im : 0.0;
        out[u].re += m.re * xr - m.im * xi;
        out[u].im += m.re * xi + m.im * xr;
      }
    }
  } else {
#pragma unroll
    for (int u = 0; u < NE; ++u)
      if (ok[u]) out[u] = mix_row<double>(rp, ent, row[u], src + base[u], sw, ss);
  }
}

// The MPO-mixed stage-1 result, formed while it is staged (never stored).
// src holds, for every input channel wi, the rows (a, si) of width nb_:
// src[wi][a][si][b] at wi * sw + a * sa + si * ss + b.  For output channel
// wo (the batch):
//   MixRows:  op_wo[(a, so)][b] = sum_{(wi, si, v) in row (wo, so)} v src[wi][a][si][b]
//   MixCols:  op_wo[a][(so, b)] = the same sum
// with the mixing rows indexed wo * dph + so.
template <typename S> struct MixRows {
  typedef zd raw_t;
  const cplx<S>* src;
  const int* rp;
  const MixEnt* ent;
  int dph;
  long sw, sa, ss;
  bool trans;
  template <typename T> TJM_DEV cplx<T> get(int wo, int i, int b) const {
    const int a = i / dph, so = i - a * dph;
    return mix_row<T>(rp, ent, wo * dph + so, src + (long)a * sa + b, sw, ss);
  }
  template <int NE>
  TJM_DEV void fetch(int wo, const int* ii, const int* kk, const bool* ok, raw_t* out) const {
    int row[NE], base[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int a = ii[u] / dph, so = ii[u] - a * dph;
      row[u] = wo * dph + so;
      base[u] = a * (int)sa + kk[u];
    }
    mix_fetch<S, NE>(rp, ent, src, sw, ss, row, base, ok, out);
  }
  template <typename T> TJM_DEV cplx<T> value(const raw_t& v, bool) const { return cmk((T)v.re, (T)v.im); }
};

template <typename S> struct MixCols {
  typedef zd raw_t;
  const cplx<S>* src;
  const int* rp;
  const MixEnt* ent;
  int dph, nb_;
  long sw, sa, ss;
  bool trans;
  template <typename T> TJM_DEV cplx<T> get(int wo, int a, int k) const {
    const int so = k / nb_, b = k - so * nb_;
    return mix_row<T>(rp, ent, wo * dph + so, src + (long)a * sa + b, sw, ss);
  }
  template <int NE>
  TJM_DEV void fetch(int wo, const int* aa, const int* kk, const bool* ok, raw_t* out) const {
    int row[NE], base[NE];
#pragma unroll
    for (int u = 0; u < NE; ++u) {
      const int so = kk[u] / nb_, b = kk[u] - so * nb_;
      row[u] = wo * dph + so;
      base[u] = aa[u] * (int)sa + b;
    }
    mix_fetch<S, NE>(rp, ent, src, sw, ss, row, base, ok, out);
  }
  template <typename T> TJM_DEV cplx<T> value(const raw_t& v, bool) const { return cmk((T)v.re, (T)v.im); }
};

template <typename S>
TJM_DEV MixRows<S> mix_rows(const cplx<S>* src, const int* rp, const MixEnt* ent, int dph, long sw, long sa,
                            long ss) {
  MixRows<S> m; m.src = src; m.rp = rp; m.ent = ent; m.dph = dph; m.sw = sw; m.sa = sa; m.ss = ss;
  m.trans = false; return m;
}

template <typename S>
TJM_DEV MixCols<S> mix_cols(const cplx<S>* src, const int* rp, const MixEnt* ent, int dph, int nb_, long sw,
                            long sa, long ss) {
  MixCols<S> m; m.src = src; m.rp = rp; m.ent = ent; m.dph = dph; m.nb_ = nb_; m.sw = sw; m.sa = sa;
  m.ss = ss; m.trans = false; return m;
}
