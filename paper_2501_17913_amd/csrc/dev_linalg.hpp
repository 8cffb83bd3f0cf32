// FP64 workgroup factorisations and the Lanczos matrix exponential.
//
//   blk_qr        Householder QR of an m x n complex matrix, explicit thin Q,
//                 R with a real non-negative diagonal.
//   blk_svd       one-sided (Hestenes) Jacobi SVD with the truncation rule of
//                 the sweep code; singular values to high relative accuracy.
//   blk_expm      exp(-i t H) v by Lanczos with full re-orthogonalisation;
//                 the small tridiagonal exponential by scaled Taylor series.
// All matrices are row-major complex<double> in global scratch memory.
#pragma once
#include <dev_lds.hpp>

// st(e, ld(e)) for every e < n (n >= 1), each thread's eight entries loaded
// before any of them is stored, so that their loads are in flight together.
// For maps whose stores do not feed their own loads.
template <class Ld, class St>
TJM_DEV void blk_map(int n, Ld ld, St st) {
  for (int base = 0; base < n; base += 8 * TJM_NT) {
    zd buf[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + tjm_tid() + u * TJM_NT;
      buf[u] = ld(e < n ? e : n - 1);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = base + tjm_tid() + u * TJM_NT;
      if (e < n) st(e, buf[u]);
    }
  }
}

// --------------------------------------------------------------------------
// Householder QR.  X (m x n, ld n, m <= 128) is destroyed.  On return Q
// (m x k, ld k) and R (k x n, ld n) hold the thin factors, k = min(m, n),
// with diag(R) real >= 0.
//
// Reflector of column j (x = rows j.. of the current column, x0 its first
// entry): beta = -(x0/|x0|) ||x||, v = x with v0 = x0 - beta,
// H_j = I - (2/||v||^2) v v^H; a zero column gives H_j = I.  Each step
// copies v to LDS once; groups of QR_TPC threads own one trailing column,
// each thread a strided set of its rows held in registers between the dot
// product and the update; the group that updates column j+1 also returns
// its norm below the diagonal for the next step.
// --------------------------------------------------------------------------
// The elimination: on return X holds the reflectors below the diagonal with
// their heads v0 on it, the rest of R above it; H holds beta_j (the
// diagonal of R) and ||v_j||^2.
TJM_DEV void qr_reduce(int m, int n, zd* X, QrLds& H, BlkScratch& S) {
  const int k = m < n ? m : n;
  const int tid = tjm_tid();
  const int ngrp = TJM_NT / QR_TPC;
  const int g = tid / QR_TPC, gl = tid % QR_TPC;
  double a2 = 0.0;
  for (int i = tid; i < m; i += TJM_NT) a2 += abs2(X[(long)i * n]);
  a2 = blk_sum(a2, S);
  for (int j = 0; j < k; ++j) {
    const int mr = m - j;
    if (j > 0) a2 = H.a2next;
    const zd x0 = X[(long)j * n + j];
    const double ax0 = sqrt(abs2(x0));
    const double al = sqrt(a2);
    zd beta = cmk(0.0, 0.0), v0 = x0;
    double vn = 0.0;
    if (al > 0.0) {
      const zd ph = ax0 > 0.0 ? cmk(x0.re / ax0, x0.im / ax0) : cmk(1.0, 0.0);
      beta = cmk(-ph.re * al, -ph.im * al);
      v0 = x0 - beta;                             // v0 = x0 + ph * alpha
      vn = 2.0 * al * (al + ax0);
    }
    for (int i = tid; i < mr; i += TJM_NT) H.v[i] = i == 0 ? v0 : X[(long)(j + i) * n + j];
    if (tid == 0) { H.vnorm2[j] = vn; H.bre[j] = beta.re; H.bim[j] = beta.im; }
    tjm_sync();
    const double f = vn > 0.0 ? 2.0 / vn : 0.0;
    for (int c = j + 1 + g; c < n; c += ngrp) {
      zd x[QR_RPT];
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < QR_RPT; ++t) {
        const int i = gl + QR_TPC * t;
        x[t] = i < mr ? X[(long)(j + i) * n + c] : cmk(0.0, 0.0);
        const zd p = cdotc(i < mr ? H.v[i] : cmk(0.0, 0.0), x[t]);
        sr += p.re; si += p.im;
      }
      if (vn > 0.0) {
        grp_sum2(sr, si, QR_TPC);
        const zd sc = cmk(f * sr, f * si);
#pragma unroll
        for (int t = 0; t < QR_RPT; ++t) {
          const int i = gl + QR_TPC * t;
          if (i < mr) {
            x[t] = x[t] - sc * H.v[i];
            X[(long)(j + i) * n + c] = x[t];
          }
        }
      }
      if (c == j + 1) {                           // norm of the next column below its diagonal
        double q = 0.0;
#pragma unroll
        for (int t = 0; t < QR_RPT; ++t) {
          const int i = gl + QR_TPC * t;
          if (i >= 1 && i < mr) q += abs2(x[t]);
        }
        q = grp_sum(q, QR_TPC);
        if (gl == 0) H.a2next = q;
      }
    }
    if (tid == 0) X[(long)j * n + j] = v0;        // reflector head, for Q
    tjm_sync();
  }
}

TJM_DEVNI void blk_qr_global(int m, int n, zd* X, zd* Q, zd* R) {
  QrLds& H = tjm_lds.qr;
  BlkScratch& S = tjm_lds.S;
  const int k = m < n ? m : n;
  const int tid = tjm_tid();
  const int ngrp = TJM_NT / QR_TPC;
  const int g = tid / QR_TPC, gl = tid % QR_TPC;
  qr_reduce(m, n, X, H, S);
  // R (upper triangle of X, diagonal beta), then the gauge fix
  for (int e = tid; e < k * n; e += TJM_NT) {
    int i = e / n, c = e % n;
    zd v = cmk(0.0, 0.0);
    if (c > i) v = X[(long)i * n + c];
    else if (c == i) v = cmk(H.bre[i], H.bim[i]);
    R[(long)i * n + c] = v;
  }
  // Q = H_0 ... H_{k-1} [I; 0]
  for (int e = tid; e < m * k; e += TJM_NT) {
    int i = e / k, c = e % k;
    Q[(long)i * k + c] = cmk(i == c ? 1.0 : 0.0, 0.0);
  }
  tjm_sync();
  for (int j = k - 1; j >= 0; --j) {
    const double vn = H.vnorm2[j];
    if (!(vn > 0.0)) continue;                    // identity reflector
    const int mr = m - j;
    for (int i = tid; i < mr; i += TJM_NT) H.v[i] = X[(long)(j + i) * n + j];
    tjm_sync();
    const double f = 2.0 / vn;
    for (int c = j + g; c < k; c += ngrp) {
      zd x[QR_RPT];
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int t = 0; t < QR_RPT; ++t) {
        const int i = gl + QR_TPC * t;
        x[t] = i < mr ? Q[(long)(j + i) * k + c] : cmk(0.0, 0.0);
        const zd p = cdotc(i < mr ? H.v[i] : cmk(0.0, 0.0), x[t]);
        sr += p.re; si += p.im;
      }
      grp_sum2(sr, si, QR_TPC);
      const zd sc = cmk(f * sr, f * si);
#pragma unroll
      for (int t = 0; t < QR_RPT; ++t) {
        const int i = gl + QR_TPC * t;
        if (i < mr) Q[(long)(j + i) * k + c] = x[t] - sc * H.v[i];
      }
    }
    tjm_sync();
  }
  // diag(R) real >= 0: row j of R times conj(ph_j), column j of Q times ph_j
  for (int e = tid; e < k * n; e += TJM_NT) {
    int i = e / n;
    double br = H.bre[i], bi = H.bim[i], ab = sqrt(br * br + bi * bi);
    if (ab > 0.0) R[e] = cmk(br / ab, -bi / ab) * R[e];
  }
  for (int e = tid; e < m * k; e += TJM_NT) {
    int c = e % k;
    double br = H.bre[c], bi = H.bim[c], ab = sqrt(br * br + bi * bi);
    if (ab > 0.0) Q[e] = cmk(br / ab, bi / ab) * Q[e];
  }
  tjm_sync();
}

// --------------------------------------------------------------------------
// The same Householder QR with the matrix held in registers, for m <= 128
// rows and n <= 64 columns (every site tensor of a bond of at most 64).
// Thread t owns column c = t / 4 and the rows g + 4 i (g = t % 4,
// i < 32) of it; the four threads of a column are neighbouring lanes of one
// wavefront, so a column's sums are two lane shuffles.
//   Reduction, step j: the owners of column j form its reflector and
//   publish it in LDS, one barrier, and every later column is updated in
//   registers against it; the next step's owners start at once (the
//   reflector buffer alternates, so one barrier per column suffices).  No
//   global memory is touched inside the loop, so the barriers wait for
//   nothing but LDS.  Each column's reflector stays in its owners'
//   registers (rows below the diagonal; v0 in LDS).
//   Then R is written, and the reflectors go to V (m x k, global scratch)
//   in one pass.
//   Formation of Q = H_0 ... H_{k-1} [I; 0] in the same registers: the
//   reflectors are staged in LDS in blocks of QRF_VB (the next block's
//   loads in flight while the current one is applied), and a block is
//   applied without barriers, since a column's update needs only its own
//   four threads.
// Same reflectors, signs and gauge as blk_qr_global (which serves larger
// shapes).  X may alias Q or R.
// With adj the matrix factorised is A = X^H for X of n x m (ld m), and the
// factors are written adjoint: Q^H (k x m, ld m) to Q and R^H (n x k, ld k)
// to R, plus R itself (k x n) to Rk if it is non-null; this is the LQ
// X = R^H Q^H of a site tensor without transposed copies.
// --------------------------------------------------------------------------
static_assert(TJM_NT == 4 * QRF_COLS, "one column per four threads");
constexpr int QRF_VB = 8;                          // reflectors per LDS block of the Q formation
static_assert(2 * QRF_VB * QRF_ROWS * 16 <= GEMM_LDS_BYTES, "two reflector blocks fit the staging area");

// One reflector application to a column held in registers (rows g + 4 i,
// i < QRF_RPT): x <- x - (2/vn) (v^H x) v; the four threads of the column
// reduce the product by two shuffles.  The reflector buffer vb holds zeros
// outside the rows [j, m) of the reflector, so no row needs a mask.  The
// entries of vb are read eight at a time into registers, all eight reads
// issued before the first is used, so that one LDS latency covers eight
// rows.
TJM_DEV void qrf_reflect(zd* x, const zd* vb, int g, double vn) {
  // four independent FMA chains: sum conj(v) x = (a + b) + i (c - e)
  double sa = 0.0, sb = 0.0, sc = 0.0, se = 0.0;
#pragma unroll
  for (int i0 = 0; i0 < QRF_RPT; i0 += 8) {
    zd vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = vb[g + 4 * (i0 + u)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      sa = fma(vv[u].re, x[i0 + u].re, sa);
      sb = fma(vv[u].im, x[i0 + u].im, sb);
      sc = fma(vv[u].re, x[i0 + u].im, sc);
      se = fma(vv[u].im, x[i0 + u].re, se);
    }
    __builtin_amdgcn_sched_barrier(0);            // keep the next batch's reads after this one
  }
  double sr = sa + sb, si = sc - se;
  sr = tjm_grp_sum<4>(sr);
  si = tjm_grp_sum<4>(si);
  const double f = 2.0 / vn;
  const double ar = f * sr, ai = f * si;
#pragma unroll
  for (int i0 = 0; i0 < QRF_RPT; i0 += 8) {
    zd vv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) vv[u] = vb[g + 4 * (i0 + u)];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      x[i0 + u].re = fma(ai, vv[u].im, fma(-ar, vv[u].re, x[i0 + u].re));
      x[i0 + u].im = fma(-ai, vv[u].re, fma(-ar, vv[u].im, x[i0 + u].im));
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Reduction of the register QR: X (or X^H) to R, the reflectors to V
// (m x k, column j's reflector at V + j m, rows [j, m)); the reflectors'
// scalars stay in tjm_lds.qrf.
TJM_DEVNI void qrf_reduce(int m, int n, const zd* X, zd* R, zd* V, bool adj, zd* Rk) {
  QrfLds& H = tjm_lds.qrf;
  const int tid = tjm_tid();
  const int c = tid >> 2, g = tid & 3;
  const int k = m < n ? m : n;
  const bool live = c < n;
  zd x[QRF_RPT];
#pragma unroll
  for (int i = 0; i < QRF_RPT; ++i) {
    const int r = g + 4 * i;
    const bool on = live && r < m;
    const zd e = gload(X, on ? (adj ? (long)c * m + r : (long)r * n + c) : 0L);
    x[i] = csel(on, adj ? conjg(e) : e, cmk(0.0, 0.0));
  }
  tjm_sync();                                     // X is read before Q or R may overwrite it
  for (int j = 0; j < k; ++j) {
    zd* vb = H.v[j & 1];
    if (c == j) {
      // reflector of column j: x0 = X[j][j], beta = -(x0/|x0|) ||x||,
      // v = x with v0 = x0 - beta, ||v||^2 = 2 ||x|| (||x|| + |x0|); the
      // buffer gets the rows >= j of the column and zeros above (rows from
      // m on are zero in x)
      double a2 = 0.0;
#pragma unroll
      for (int i = 0; i < QRF_RPT; ++i) {
        const int r = g + 4 * i;
        const zd e = csel(r >= j, x[i], cmk(0.0, 0.0));
        a2 += abs2(e);
        vb[r] = e;
      }
      a2 = tjm_grp_sum<4>(a2);
      __builtin_amdgcn_wave_barrier();
      const zd x0 = vb[j];                        // written by a lane of this wavefront
      const double ax0 = sqrt(abs2(x0)), al = sqrt(a2);
      zd beta = cmk(0.0, 0.0), v0 = x0;
      double vn = 0.0;
      if (al > 0.0) {
        const zd ph = ax0 > 0.0 ? cmk(x0.re / ax0, x0.im / ax0) : cmk(1.0, 0.0);
        beta = cmk(-ph.re * al, -ph.im * al);
        v0 = x0 - beta;
        vn = 2.0 * al * (al + ax0);
      }
      __builtin_amdgcn_wave_barrier();
      if (g == 0) { vb[j] = v0; H.bre[j] = beta.re; H.bim[j] = beta.im; H.vn[j] = vn; H.v0[j] = v0; }
    }
    tjm_sync();
    if (live && c > j) {
      const double vn = H.vn[j];
      if (vn > 0.0) qrf_reflect(x, vb, g, vn);
    }
  }
  tjm_sync();                                     // every reflector read; H.v free
  // R: row r of the upper triangle times conj(ph_r), diagonal |beta_r|;
  // the reflector of column c (v0 on the diagonal, x below it) to V
#pragma unroll
  for (int i = 0; i < QRF_RPT; ++i) {
    const int r = g + 4 * i;
    if (live && r < k) {
      const double br = H.bre[r], bi = H.bim[r], ab = sqrt(br * br + bi * bi);
      const zd ph = ab > 0.0 ? cmk(br / ab, -bi / ab) : cmk(1.0, 0.0);
      const zd dg = ab > 0.0 ? cmk(ab, 0.0) : cmk(br, bi);
      const zd val = csel(r < c, ph * x[i], csel(r == c, dg, cmk(0.0, 0.0)));
      if (adj) {
        gstore(R, (long)c * k + r, conjg(val));
        if (Rk) gstore(Rk, (long)r * n + c, val);
      } else {
        gstore(R, (long)r * n + c, val);
      }
    }
    if (c < k && r >= c && r < m) gstore(V, (long)c * m + r, csel(r == c, H.v0[c], x[i]));
  }
  tjm_sync();                                     // V complete and visible
}

// Formation of Q = H_0 ... H_{k-1} [I; 0] from the reflectors in V, in
// registers (the layout of the reduction), written as Q (m x k) or, with
// adj, Q^H (k x m).
TJM_DEVNI void qrf_form(int m, int n, zd* Q, const zd* V, bool adj) {
  QrfLds& H = tjm_lds.qrf;
  const int tid = tjm_tid();
  const int c = tid >> 2, g = tid & 3;
  const int k = m < n ? m : n;
  const bool qlive = c < k;
  zd q[QRF_RPT];
#pragma unroll
  for (int i = 0; i < QRF_RPT; ++i) q[i] = cmk((qlive && g + 4 * i == c) ? 1.0 : 0.0, 0.0);
  zd* blkbuf = (zd*)tjm_lds.gemm;                 // 2 x QRF_VB x QRF_ROWS
  constexpr int PER = QRF_VB * QRF_ROWS / TJM_NT; // staged entries per thread
  const int nblk = (k + QRF_VB - 1) / QRF_VB;
  // block b holds reflectors j = jb .. jb + QRF_VB - 1 (jb = b QRF_VB), in
  // rows [jj][row], zero outside the rows [j, m) of each; blocks are applied
  // from the last one down
  zd nxt[PER];
  auto fetch = [&](int bi) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int e = tid + u * TJM_NT, jj = e / QRF_ROWS, r = e % QRF_ROWS, j = bi * QRF_VB + jj;
      const bool on = j < k && r >= j && r < m;
      nxt[u] = csel(on, gload(V, on ? (long)j * m + r : 0L), cmk(0.0, 0.0));
    }
  };
  auto stage = [&](int bi) {
    zd* dst = blkbuf + (bi & 1) * (QRF_VB * QRF_ROWS);
#pragma unroll
    for (int u = 0; u < PER; ++u) dst[tid + u * TJM_NT] = nxt[u];
  };
  if (nblk > 0) { fetch(nblk - 1); stage(nblk - 1); }
  tjm_sync();
  for (int bi = nblk - 1; bi >= 0; --bi) {
    if (bi > 0) fetch(bi - 1);                    // in flight while this block is applied
    const zd* cur = blkbuf + (bi & 1) * (QRF_VB * QRF_ROWS);
    for (int jj = QRF_VB - 1; jj >= 0; --jj) {
      const int j = bi * QRF_VB + jj;
      if (j >= k) continue;
      const double vn = H.vn[j];
      if (qlive && c >= j && vn > 0.0) qrf_reflect(q, cur + jj * QRF_ROWS, g, vn);
    }
    if (bi > 0) stage(bi - 1);                    // the other buffer: read by nobody now
    tjm_sync();
  }
  // column c of Q times ph_c
  if (qlive) {
    const double br = H.bre[c], bi = H.bim[c], ab = sqrt(br * br + bi * bi);
    const zd ph = ab > 0.0 ? cmk(br / ab, bi / ab) : cmk(1.0, 0.0);
#pragma unroll
    for (int i = 0; i < QRF_RPT; ++i) {
      const int r = g + 4 * i;
      if (r < m) {
        if (adj) gstore(Q, (long)c * m + r, conjg(ph * q[i]));
        else gstore(Q, (long)r * k + c, ph * q[i]);
      }
    }
  }
  tjm_sync();
}

TJM_DEV void blk_qr_regs(int m, int n, const zd* X, zd* Q, zd* R, zd* V, bool adj, zd* Rk) {
  qrf_reduce(m, n, X, R, V, adj, Rk);
  qrf_form(m, n, Q, V, adj);
}

// Thin QR X = Q R (k = min(m, n), diag(R) real >= 0) of an m x n matrix,
// m <= 128; V is m x k scratch.  X is destroyed.
TJM_DEV void blk_qr(int m, int n, zd* X, zd* Q, zd* R, zd* V) {
  if (m <= QRF_ROWS && n <= QRF_COLS) blk_qr_regs(m, n, X, Q, R, V, false, nullptr);
  else blk_qr_global(m, n, X, Q, R);
}

// --------------------------------------------------------------------------
// Truncation rank of a non-increasing spectrum s_0 >= s_1 >= ... (n values,
// read through s(i)); run by one thread.  Smallest k >= 1 with
// sum_{i>=k} s_i^2 <= discard * sum s_i^2 (the tail accumulated from the
// end), capped at cap; a cap that cuts a multiplet (s_{k-1} - s_k <=
// deg_tol s_0) is lowered until it does not.
// --------------------------------------------------------------------------
template <class F>
TJM_DEV int trunc_rank(F s, int n, double discard, int cap, double deg_tol) {
  double total = 0.0;
  for (int i = 0; i < n; ++i) total += s(i) * s(i);
  const double thr = discard * total;
  int k = n;
  double tail = 0.0;                      // tail(n) = 0 <= thr unless discard < 0
  if (!(0.0 <= thr)) k = n;
  else {
    for (int kk = n - 1; kk >= 1; --kk) {
      tail += s(kk) * s(kk);              // = sum_{i >= kk} s_i^2
      if (tail <= thr) k = kk; else break;
    }
  }
  if (k > cap) {
    k = cap;
    while (k > 1 && s(k - 1) - s(k) <= deg_tol * s(0)) --k;
  }
  return k < 1 ? 1 : k;
}

// --------------------------------------------------------------------------
// One-sided Jacobi SVD of G (m x n, row-major ld n), truncated.
//   left  (m x k, ld k)  = U        or U S   (absorb_left)
//   right (k x n, ld n)  = S V^H    or V^H
// Returns k.  The factor without S must come out orthonormal to rounding (it
// becomes a left- or right-canonical site tensor), so the Jacobi rotations
// act on the columns of G (absorb_left = false: U) or of G^H (absorb_left =
// true: V); the factor carrying S is then one FP64 matrix-core product with
// G (U^H G = S V^H, or G V = U S), read before any output is written, so
// `left` or `right` may alias G.  Work arrays: Wc and Uc (p x nc each), Tg
// (m x n), with p, nc the row and column counts of the rotated matrix;
// nc <= 128.
// --------------------------------------------------------------------------
// Round-robin pairing of np (even) players: in round rnd, pair pr meets
// players a < b; over np - 1 rounds every pair meets once.
TJM_DEV void rr_pair(int np, int rnd, int pr, int& a, int& b) {
  if (pr == 0) { a = rnd; b = np - 1; }
  else { a = (rnd + pr) % (np - 1); b = (rnd - pr + (np - 1)) % (np - 1); }
  if (a > b) { const int t = a; a = b; b = t; }
}

// One cyclic sweep of one-sided Jacobi rotations over the ncol columns of W
// (column-major, p rows, the LDS work area tjm_lds.gemm): every pair once, the pairs
// of a round in parallel, one thread group per pair.  With n1 > 0 only the
// pairs between the first n1 columns and the others are visited: in round
// r, column i meets column n1 + (i + r) mod max(n1, ncol - n1).  A pair whose columns
// are not orthogonal to tol is rotated to orthogonality (complex Jacobi
// rotation of the 2 x 2 Gram matrix); columns of weight below zero2 are left
// alone.  SL.rotated records a rotation, SL.offmax the largest relative
// off-diagonal |w_a^H w_b| / (|w_a| |w_b|) measured.  Ends with a barrier.
constexpr int JAC_RPT = 8;           // rows per thread a pair keeps in registers

// The rounds of one sweep with TPP threads per pair (a group of TPP
// neighbouring lanes, so the sums are DPP moves and shuffles within the
// group): each thread holds rows gl + TPP t (t < JAC_RPT) of both columns,
// which cover the p <= JAC_RPT * TPP rows in one pass.  Loads are
// unconditional (rows beyond p read row 0 and are zeroed), so all 2 JAC_RPT
// of a pair are in flight together.
template <int TPP>
TJM_DEV void jacobi_rounds(int p, int ncol, int n1, double zero2, double tol, double& offm, bool& rot) {
  zd* W = (zd*)tjm_lds.gemm;             // the columns, staged in LDS
  constexpr int NGRP = TJM_NT / TPP;
  const int tid = tjm_tid();
  const int g = tid / TPP, gl = tid % TPP;
  const int np = (ncol + 1) & ~1;        // players, a dummy if ncol is odd
  const int n2 = ncol - n1;
  const int mx = n1 > n2 ? n1 : n2;
  const int npair = n1 > 0 ? mx : np / 2;
  const int nrnd = n1 > 0 ? mx : np - 1;
  for (int rnd = 0; rnd < nrnd; ++rnd) {
    for (int pr = g; pr < npair; pr += NGRP) {
      int a, b;
      bool on;
      if (n1 > 0) {
        const int j = (pr + rnd) % mx;
        a = pr; b = n1 + j;
        on = pr < n1 && j < n2;
      } else {
        rr_pair(np, rnd, pr, a, b);
        on = b < ncol;
      }
      if (!on) continue;                 // uniform over the group
      zd* wa = W + a * p;
      zd* wb = W + b * p;
      zd x[JAC_RPT], y[JAC_RPT];
#pragma unroll
      for (int t = 0; t < JAC_RPT; ++t) {
        const int r = gl + TPP * t;
        const int rc = r < p ? r : 0;
        x[t] = wa[rc];
        y[t] = wb[rc];
      }
      double aa = 0.0, bb = 0.0, cr = 0.0, ci = 0.0;
#pragma unroll
      for (int t = 0; t < JAC_RPT; ++t) {
        const bool in = gl + TPP * t < p;
        x[t] = csel(in, x[t], cmk(0.0, 0.0));
        y[t] = csel(in, y[t], cmk(0.0, 0.0));
        aa = fma(x[t].re, x[t].re, fma(x[t].im, x[t].im, aa));
        bb = fma(y[t].re, y[t].re, fma(y[t].im, y[t].im, bb));
        cr = fma(x[t].re, y[t].re, fma(x[t].im, y[t].im, cr));      // conj(x) y
        ci = fma(x[t].re, y[t].im, fma(-x[t].im, y[t].re, ci));
      }
      aa = tjm_grp_sum<TPP>(aa); bb = tjm_grp_sum<TPP>(bb);
      cr = tjm_grp_sum<TPP>(cr); ci = tjm_grp_sum<TPP>(ci);
      if (!(aa > zero2 && bb > zero2)) continue;
      const double ac = hypot(cr, ci);
      const double sab = sqrt(aa) * sqrt(bb);     // no overflow for large norms
      const double rel = ac / sab;
      offm = fmax(offm, rel == rel ? rel : 1.0);
      if (ac > tol * sab) {
        const double inv = 1.0 / ac;
        const double zeta = 0.5 * (bb - aa) * inv;
        const double az = fabs(zeta);
        double t = az > 1e150 ? 0.5 / az : 1.0 / (az + sqrt(1.0 + zeta * zeta));
        if (zeta < 0.0) t = -t;
        const double cs = rsqrt(1.0 + t * t), sn = cs * t;
        const zd eph = cmk(cr * inv, -ci * inv);  // conj(c)/|c|
#pragma unroll
        for (int q = 0; q < JAC_RPT; ++q) {
          const int r = gl + TPP * q;
          const zd yy = eph * y[q];
          if (r < p) {
            wa[r] = cs * x[q] - sn * yy;
            wb[r] = sn * x[q] + cs * yy;
          }
        }
        rot = true;
      }
    }
    tjm_sync();
  }
}

TJM_DEVNI void jacobi_sweep(int p, int ncol, int n1, double zero2, double tol) {
  SvdLds& SL = tjm_lds.sv;
  const int np = (ncol + 1) & ~1;
  const int n2 = ncol - n1;
  const int mx = n1 > n2 ? n1 : n2;
  const int npair = n1 > 0 ? mx : np / 2;
  // as many pairs at once as the workgroup holds, but enough threads per
  // pair that each keeps at most JAC_RPT rows of the two columns (p <=
  // JAC_RPT * 64); a group lies within one wavefront
  int tpp = TJM_WAVE < 64 ? TJM_WAVE : 64;
  while (tpp > 1 && tpp * npair > TJM_NT) tpp >>= 1;
  while (tpp < 64 && tpp < TJM_WAVE && tpp < TJM_NT && tpp * JAC_RPT < p) tpp <<= 1;
  // this thread's largest relative off-diagonal and whether it rotated,
  // merged into SL once at the end (not by an LDS atomic per pair and round)
  double offm = 0.0;
  bool rot = false;
  switch (tpp) {
    case 1: jacobi_rounds<1>(p, ncol, n1, zero2, tol, offm, rot); break;
    case 2: jacobi_rounds<2>(p, ncol, n1, zero2, tol, offm, rot); break;
    case 4: jacobi_rounds<4>(p, ncol, n1, zero2, tol, offm, rot); break;
    case 8: jacobi_rounds<8>(p, ncol, n1, zero2, tol, offm, rot); break;
    case 16: jacobi_rounds<16>(p, ncol, n1, zero2, tol, offm, rot); break;
    case 32: jacobi_rounds<32>(p, ncol, n1, zero2, tol, offm, rot); break;
    default: jacobi_rounds<64>(p, ncol, n1, zero2, tol, offm, rot); break;
  }
  for (int s = TJM_WAVE / 2; s > 0; s >>= 1) offm = fmax(offm, tjm_shfl_xor(offm, s));
  const bool wrot = __any(rot);
  if (tjm_lane() == 0) {
    // offm >= 0: the bits of a non-negative double order like its value
    atomicMax(&SL.offmax, (unsigned long long)__double_as_longlong(offm));
    if (wrot) atomicOr(&SL.rotated, 1);
  }
  tjm_sync();
}

TJM_DEVNI int blk_svd(int m, int n, const zd* G, zd* left, zd* right, bool absorb_left,
                      double discard, int cap, double deg_tol, zd* Wc, zd* Uc, zd* Tg) {
  SvdLds& SL = tjm_lds.sv;
  BlkScratch& S = tjm_lds.S;
  void* glds = tjm_lds.gemm;
  const int tid = tjm_tid();
  const bool tr = absorb_left;           // rotate the columns of G^H (-> V)
  const int p = tr ? n : m;              // rows of the working matrix
  // Preconditioning: the rotated matrix is R^H from a Householder QR of
  // G (tr) or of G^H, X = Q R.  It has the Gram matrix R^H R = X^H X of the
  // matrix it replaces, hence the same singular values and rotated-side
  // singular vectors, only r = min(m, n) columns, and a graded,
  // near-triangular form on which the sweeps converge in far fewer rounds
  // than on G itself when the spectrum decays (Drmac and Veselic, SIAM J.
  // Matrix Anal. Appl. 29 (2008)).
  const int xr = tr ? m : n;             // rows of X (columns of X = p)
  const bool pre = xr <= QR_MROWS;
  const int nc = pre ? (m < n ? m : n) : (tr ? m : n);   // columns of the working matrix
  // the working matrix is rotated in LDS (glds, SVD_LDS_BYTES) when it fits,
  // else in the global array Wc; glds is free until the final product
  double f2 = 0.0;
  if (pre) {
    blk_map(xr * p, [&](int e) {
      const int i = e / p, c = e % p;    // X[i][c]
      return tr ? gload(G, (long)i * n + c) : conjg(gload(G, (long)c * n + i));
    }, [&](int e, zd x) { gstore(Tg, e, x); });
    tjm_sync();
    QrLds& H = *(QrLds*)glds;
    qr_reduce(xr, p, Tg, H, S);
    for (int j = tid; j < nc; j += TJM_NT) Tg[(long)j * p + j] = cmk(H.bre[j], H.bim[j]);
    tjm_sync();                          // H (in glds) is dead from here
  }
  if ((long)p * nc * 16 <= SVD_LDS_BYTES) Wc = (zd*)glds;
  blk_map(p * nc, [&](int e) {
    const int c = e / p, r = e % p;      // Wc[c][r] = Gw[r][c]
    zd x;
    if (pre) x = csel(r < c, cmk(0.0, 0.0), conjg(gload(Tg, (long)c * p + r)));   // (R^H)[r][c]
    else x = tr ? conjg(gload(G, (long)c * n + r)) : gload(G, (long)r * n + c);
    return x;
  }, [&](int e, zd x) { Wc[e] = x; f2 += abs2(x); });
  // columns below 1e-14 ||G||_F carry weight < 1e-28 of the total, far
  // below any truncation threshold: they are not rotated (rotating them only
  // stirs rounding noise and never converges)
  const double zero2 = 1e-28 * blk_sum(f2, S);
  const double tol = 2.220446049250313e-16 * sqrt((double)p);
  // convergence is quadratic: a sweep that started with every relative
  // off-diagonal below 1e-3 sqrt(tol) leaves them far below tol, so no
  // further sweep is needed to confirm it
  const double quad = 1e-3 * sqrt(tol);
  // A working matrix too large for LDS is swept in column blocks of bw
  // columns (block one-sided Jacobi): each block is staged in LDS alone for
  // the pairs within it, then two blocks at a time, the block pairs in the
  // same round-robin as single columns, for the pairs across them.  Every
  // column pair is visited once per sweep, and the matrix is read and
  // written nb times per sweep instead of once per column pair.
  const bool in_lds = (long)p * nc * 16 <= SVD_LDS_BYTES;
  const int bw = in_lds ? nc : SVD_LDS_BYTES / (32 * p);   // >= 2 for p <= 1024
  const bool blocked = !in_lds;
  const int nb = blocked ? (nc + bw - 1) / bw : 1;
  const int nbp = (nb + 1) & ~1;
  zd* Lc = (zd*)tjm_lds.gemm;
  for (int sweep = 0; sweep < 40 && nc >= 2; ++sweep) {
    if (tid == 0) { SL.rotated = 0; SL.offmax = 0ull; }
    tjm_sync();
    if (!blocked) {
      jacobi_sweep(p, nc, 0, zero2, tol);
    } else {
      // stage columns [c0, c0 + cI) and [c1, c1 + cJ) in Lc, or write them
      // back; eight entries per thread in flight
      auto move = [&](bool in, int c0, int cI, int c1, int cJ) {
        const int tot = (cI + cJ) * p;
        for (int base = 0; base < tot; base += 8 * TJM_NT) {
          zd buf[8];
          long gi[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            int e = base + tid + u * TJM_NT;
            e = e < tot ? e : tot - 1;
            const int c = e / p, r = e % p;
            gi[u] = (long)(c < cI ? c0 + c : c1 + c - cI) * p + r;
            buf[u] = in ? gload(Wc, gi[u]) : Lc[e];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int e = base + tid + u * TJM_NT;
            if (e < tot) {
              if (in) Lc[e] = buf[u];
              else gstore(Wc, gi[u], buf[u]);
            }
          }
        }
        tjm_sync();
      };
      for (int I = 0; I < nb; ++I) {
        const int c0 = I * bw, cI = nc - c0 < bw ? nc - c0 : bw;
        move(true, c0, cI, 0, 0);
        jacobi_sweep(p, cI, 0, zero2, tol);
        move(false, c0, cI, 0, 0);
      }
      for (int rnd = 0; rnd < nbp - 1; ++rnd)
        for (int pr = 0; pr < nbp / 2; ++pr) {
          int I, J;
          rr_pair(nbp, rnd, pr, I, J);
          if (J >= nb) continue;
          const int c0 = I * bw, cI = nc - c0 < bw ? nc - c0 : bw;
          const int c1 = J * bw, cJ = nc - c1 < bw ? nc - c1 : bw;
          move(true, c0, cI, c1, cJ);
          jacobi_sweep(p, cI + cJ, cI, zero2, tol);
          move(false, c0, cI, c1, cJ);
        }
    }
    if (SL.rotated == 0 || __longlong_as_double((long long)SL.offmax) < quad) break;
    tjm_sync();
  }
  // singular values, descending order (stable in the column index)
  for (int c = tjm_wave(); c < nc; c += TJM_NWAVE) {
    double a = 0.0;
    for (int r = tjm_lane(); r < p; r += TJM_WAVE) a += abs2(Wc[(long)c * p + r]);
    a = grp_sum(a, TJM_WAVE);
    if (tjm_lane() == 0) SL.s[c] = sqrt(a);
  }
  tjm_sync();
  // a non-finite norm sorts as -1, so the order is a permutation whatever
  // the data (the trajectory is flagged later by its norm check)
  for (int c = tid; c < nc; c += TJM_NT) {
    double sc = SL.s[c];
    if (!(sc == sc) || sc > 1.7e308) sc = -1.0;
    int rank = 0;
    for (int i = 0; i < nc; ++i) {
      double si = SL.s[i];
      if (!(si == si) || si > 1.7e308) si = -1.0;
      if (si > sc || (si == sc && i < c)) ++rank;
    }
    SL.order[rank] = c;
  }
  tjm_sync();
  if (tid == 0) {
    auto sv = [&](int i) { return SL.s[SL.order[i]]; };
    int k = trunc_rank(sv, nc, discard, cap, deg_tol);
    while (k > 1 && sv(k - 1) <= 0.0) --k;   // never keep an exact zero
    SL.k = k;
  }
  tjm_sync();
  const int k = SL.k;
  // kept orthonormal vectors of Gw in sorted order: Uc[j][r] = w_{o_j}[r] / s
  blk_map(k * p, [&](int e) {
    const int j = e / p, r = e % p, o = SL.order[j];
    return (1.0 / SL.s[o]) * Wc[(long)o * p + r];
  }, [&](int e, zd x) { gstore(Uc, e, x); });
  tjm_sync();
  if (!tr) {
    // G = U S V^H with U from the rotated columns: right = U^H G = S V^H
    blk_cgemm<double>(k, n, m, 1, true, cmat((const zd*)Uc, p, 0, false, true), cmat(G, n), Tg, n, 0, false, glds);
    tjm_sync();
    blk_map(m * k, [&](int e) { const int r = e / k, j = e % k; return gload(Uc, (long)j * p + r); },
            [&](int e, zd x) { gstore(left, e, x); });
    blk_map(k * n, [&](int e) { return gload(Tg, e); }, [&](int e, zd x) { gstore(right, e, x); });
  } else {
    // G^H = V S U^H with V from the rotated columns: left = G V = U S
    blk_cgemm<double>(m, k, n, 1, true, cmat(G, n), cmat((const zd*)Uc, p, 0, true, false), Tg, k, 0, false, glds);
    tjm_sync();
    blk_map(k * n, [&](int e) { const int j = e / n, c = e % n; return conjg(gload(Uc, (long)j * p + c)); },
            [&](int e, zd x) { gstore(right, e, x); });
    blk_map(m * k, [&](int e) { return gload(Tg, e); }, [&](int e, zd x) { gstore(left, e, x); });
  }
  tjm_sync();
  return k;
}

// --------------------------------------------------------------------------
// Lanczos exponential.  v (n complex doubles) is replaced by exp(-i t H) v.
// Op must provide  void apply(const zd* q, zd* w)  (a collective call that
// leaves w complete for all threads).  Q holds up to m_max - 1 basis vectors
// of length n, w is an n-vector of scratch.  Returns the Krylov dimension
// used.
//
// The basis is stored unnormalised: q_i = s_i B_i with B_0 = v itself (no
// copy) and B_i = Q + (i-1) n, the scales s_i in LDS.  H is applied to B_j
// (H q_j = s_j H B_j), and the Gram-Schmidt pass writes the orthogonalised
// vector straight into B_{j+1} with s_{j+1} = 1/||.||: no separate
// normalisation pass.  The arithmetic of the basis, the projections and the
// small exponential is FP64 throughout.
// --------------------------------------------------------------------------
// exp(-i t T) e_0 for the symmetric tridiagonal T = tridiag(beta, alpha, beta)
// of size m <= 32: shift by alpha_0, split t into s pieces with
// |t/s| * ||T - alpha_0||_inf <= 1/2 (Gershgorin) and sum 18 Taylor terms per
// piece (remainder below 1e-21 of the norm).  On a 64-wide wavefront lane i
// owns row i and takes its neighbours' terms by shuffle; otherwise one thread
// walks the rows.
TJM_DEV void tridiag_exp_e0(int m, double t, LanczosLds& Lz) {
  const double mu = Lz.alpha[0];
  if constexpr (TJM_WAVE >= TJM_KMAX) {
    if (tjm_wave() != 0) return;
    const int i = tjm_lane();
    const double a = (i < m) ? Lz.alpha[i] - mu : 0.0;
    const double bl = (i > 0 && i < m) ? Lz.beta[i - 1] : 0.0;      // T[i][i-1]
    const double br = (i + 1 < m) ? Lz.beta[i] : 0.0;               // T[i][i+1]
    double gers = fabs(a) + bl + br;
    for (int s = TJM_WAVE / 2; s > 0; s >>= 1) gers = fmax(gers, tjm_shfl_xor(gers, s));
    int pieces = (int)ceil(fabs(t) * gers / 0.5);
    if (pieces < 1) pieces = 1;
    const double h = t / pieces;
    const int up = (i + 1) & (TJM_WAVE - 1), dn = (i + TJM_WAVE - 1) & (TJM_WAVE - 1);
    double ur = (i == 0) ? 1.0 : 0.0, ui = 0.0;
    for (int pc = 0; pc < pieces; ++pc) {
      double tr = ur, ti = ui;
      for (int kk = 1; kk <= 18; ++kk) {
        const double upr = tjm_shfl(tr, up), upi = tjm_shfl(ti, up);
        const double dnr = tjm_shfl(tr, dn), dni = tjm_shfl(ti, dn);
        const double yr = a * tr + bl * dnr + br * upr;
        const double yi = a * ti + bl * dni + br * upi;
        const double f = h / kk;
        tr = (i < m) ? f * yi : 0.0;            // (-i f)(yr + i yi)
        ti = (i < m) ? -f * yr : 0.0;
        ur += tr; ui += ti;
      }
    }
    if (i < m) {
      const double cr = cos(t * mu), ci = -sin(t * mu);
      Lz.cre[i] = cr * ur - ci * ui;
      Lz.cim[i] = cr * ui + ci * ur;
    }
  } else {
    if (tjm_tid() != 0) return;
    double gers = 0.0;
    for (int i = 0; i < m; ++i) {
      double g = fabs(Lz.alpha[i] - mu) + (i > 0 ? Lz.beta[i - 1] : 0.0) + (i + 1 < m ? Lz.beta[i] : 0.0);
      gers = fmax(gers, g);
    }
    int pieces = (int)ceil(fabs(t) * gers / 0.5);
    if (pieces < 1) pieces = 1;
    const double h = t / pieces;
    double* ur = Lz.ur;
    double* ui = Lz.ui;
    double* tr = Lz.tr;
    double* ti = Lz.ti;
    for (int i = 0; i < m; ++i) { ur[i] = (i == 0) ? 1.0 : 0.0; ui[i] = 0.0; }
    for (int pc = 0; pc < pieces; ++pc) {
      for (int i = 0; i < m; ++i) { tr[i] = ur[i]; ti[i] = ui[i]; }
      for (int kk = 1; kk <= 18; ++kk) {
        const double f = h / kk;
        double prev_r = 0.0, prev_i = 0.0;
        for (int i = 0; i < m; ++i) {
          double yr = (Lz.alpha[i] - mu) * tr[i], yi = (Lz.alpha[i] - mu) * ti[i];
          if (i > 0) { yr += Lz.beta[i - 1] * prev_r; yi += Lz.beta[i - 1] * prev_i; }
          if (i + 1 < m) { yr += Lz.beta[i] * tr[i + 1]; yi += Lz.beta[i] * ti[i + 1]; }
          prev_r = tr[i]; prev_i = ti[i];
          tr[i] = f * yi;
          ti[i] = -f * yr;
          ur[i] += tr[i]; ui[i] += ti[i];
        }
      }
    }
    const double cr = cos(t * mu), ci = -sin(t * mu);
    for (int i = 0; i < m; ++i) {
      Lz.cre[i] = cr * ur[i] - ci * ui[i];
      Lz.cim[i] = cr * ui[i] + ci * ur[i];
    }
  }
}

// Lanczos vector kernels.  Each streams the n entries (thread stride
// TJM_NT, two entries per thread in flight) and reads NB basis vectors
// B_u = bp[u] per entry with all NB loads issued together.
//
// Projections h_u = sum_e conj(B_u[e]) w[e]: each wave's sum to
// Lz.red[wave][2 (i0 + u)] (real) and + 1 (imaginary).
template <int NB>
TJM_DEV void lz_project(const zd* const* bp, const zd* w, int n, int i0, LanczosLds& Lz) {
  double hr[NB], hi[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) { hr[u] = 0.0; hi[u] = 0.0; }
#pragma unroll 2
  for (int e = tjm_tid(); e < n; e += TJM_NT) {
    const zd x = gload(w, e);
    zd b[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) b[u] = gload(bp[u], e);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      hr[u] = fma(b[u].re, x.re, fma(b[u].im, x.im, hr[u]));
      hi[u] = fma(b[u].re, x.im, fma(-b[u].im, x.re, hi[u]));
    }
  }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    hr[u] = tjm_grp_sum<TJM_WAVE>(hr[u]);
    hi[u] = tjm_grp_sum<TJM_WAVE>(hi[u]);
    if (tjm_lane() == 0) {
      Lz.red[tjm_wave()][2 * (i0 + u)] = hr[u];
      Lz.red[tjm_wave()][2 * (i0 + u) + 1] = hi[u];
    }
  }
}

// The projections of one Lanczos iteration in one pass: for the block of
// basis vectors bp[0..NB) (indices i0 + u), d_u = B_u^H w, e_u = B_u^H B_j
// and f_u = B_u^H B_{j-1}, this wavefront's parts written to red[(wave *
// TJM_KMAX + i0 + u) * 6 + (d re, d im, e re, e im, f re, f im)].
template <int NB>
TJM_DEV void lz_project3(const zd* const* bp, const zd* w, const zd* Bj, const zd* Bp, int n, int i0,
                         double* red) {
  double a[NB][6];
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int k = 0; k < 6; ++k) a[u][k] = 0.0;
  for (int e = tjm_tid(); e < n; e += TJM_NT) {
    const zd x = gload(w, e), y = gload(Bj, e), z = gload(Bp, e);
    zd b[NB];
#pragma unroll
    for (int u = 0; u < NB; ++u) b[u] = gload(bp[u], e);
#pragma unroll
    for (int u = 0; u < NB; ++u) {
      a[u][0] = fma(b[u].re, x.re, fma(b[u].im, x.im, a[u][0]));
      a[u][1] = fma(b[u].re, x.im, fma(-b[u].im, x.re, a[u][1]));
      a[u][2] = fma(b[u].re, y.re, fma(b[u].im, y.im, a[u][2]));
      a[u][3] = fma(b[u].re, y.im, fma(-b[u].im, y.re, a[u][3]));
      a[u][4] = fma(b[u].re, z.re, fma(b[u].im, z.im, a[u][4]));
      a[u][5] = fma(b[u].re, z.im, fma(-b[u].im, z.re, a[u][5]));
    }
  }
#pragma unroll
  for (int u = 0; u < NB; ++u)
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double s = tjm_grp_sum<TJM_WAVE>(a[u][k]);
      if (tjm_lane() == 0) red[((long)tjm_wave() * TJM_KMAX + i0 + u) * 6 + k] = s;
    }
}

// x_k + sum_u c_u B_u[e_k] for two entries e_0, e_1 and the coefficients
// c_u = (cr[u], ci[u]) (LDS)
template <int NB>
TJM_DEV void lz_comb(const zd* const* bp, const double* cr, const double* ci, int e0, int e1, zd& x0, zd& x1) {
  zd b0[NB], b1[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) { b0[u] = gload(bp[u], e0); b1[u] = gload(bp[u], e1); }
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    x0.re = fma(cr[u], b0[u].re, fma(-ci[u], b0[u].im, x0.re));
    x0.im = fma(cr[u], b0[u].im, fma(ci[u], b0[u].re, x0.im));
    x1.re = fma(cr[u], b1[u].re, fma(-ci[u], b1[u].im, x1.re));
    x1.im = fma(cr[u], b1[u].im, fma(ci[u], b1[u].re, x1.im));
  }
}

// out[e] = f * in[e] + sum_{i < nb} c_i B_i[e] (c_i in LDS), for every e; in
// may be null (then 0); out may be in or one of the B_i (each entry is read
// before it is written, by the same thread; the two entries a thread
// handles at once are distinct).  Returns this thread's part of ||out||^2.
template <class Basis>
TJM_DEV double lz_axpy(Basis basis, int nb, const double* cr, const double* ci, const zd* in, double f, zd* out,
                       int n) {
  double nrm = 0.0;
  for (int e0 = tjm_tid(); e0 < n; e0 += 2 * TJM_NT) {
    const bool ok1 = e0 + TJM_NT < n;
    const int e1 = ok1 ? e0 + TJM_NT : e0;
    zd x0 = cmk(0.0, 0.0), x1 = cmk(0.0, 0.0);
    if (in) { x0 = f * gload(in, e0); x1 = f * gload(in, e1); }
    int i0 = 0;
    for (; i0 + 8 <= nb; i0 += 8) {
      const zd* bp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) bp[u] = basis(i0 + u);
      lz_comb<8>(bp, cr + i0, ci + i0, e0, e1, x0, x1);
    }
    if (nb - i0 >= 4) {
      const zd* bp[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) bp[u] = basis(i0 + u);
      lz_comb<4>(bp, cr + i0, ci + i0, e0, e1, x0, x1);
      i0 += 4;
    }
    if (nb - i0 >= 2) {
      const zd* bp[2] = {basis(i0), basis(i0 + 1)};
      lz_comb<2>(bp, cr + i0, ci + i0, e0, e1, x0, x1);
      i0 += 2;
    }
    if (nb - i0 >= 1) {
      const zd* bp[1] = {basis(i0)};
      lz_comb<1>(bp, cr + i0, ci + i0, e0, e1, x0, x1);
    }
    gstore(out, e0, x0);
    nrm += abs2(x0);
    if (ok1) { gstore(out, e1, x1); nrm += abs2(x1); }
  }
  return nrm;
}

template <class Op>
TJM_DEVNI int blk_expm(Op& op, zd* v, int n, double t, int m_max, double tol, zd* Q, zd* w) {
  LanczosLds& Lz = tjm_lds.lz;
  BlkScratch& S = tjm_lds.S;
  const int tid = tjm_tid();
  double b0 = 0.0;
#pragma unroll 4
  for (int e = tid; e < n; e += TJM_NT) b0 += abs2(gload(v, e));
  b0 = sqrt(blk_sum(b0, S));
  if (b0 == 0.0) return 0;
  if (m_max > TJM_KMAX) m_max = TJM_KMAX;
  if (m_max > n) m_max = n;
  auto basis = [=](int i) -> zd* { return i == 0 ? v : Q + (long)(i - 1) * n; };
  if (tid == 0) Lz.scale[0] = 1.0 / b0;
  tjm_sync();
  int used = 0;
  for (int j = 0; j < m_max; ++j) {
    op.apply(basis(j), w);                           // w = H B_j = (H q_j) / s_j
    const int nq = j + 1;
    const double sj = Lz.scale[j];
    // The iteration in the oracle's order: alpha_j = Re q_j^H H q_j, then
    // w1 = H q_j - alpha_j q_j - beta_{j-1} q_{j-1}, then one classical
    // Gram-Schmidt pass of w1 against q_0..q_j.  w1 is never stored: one
    // pass over the basis gives d_i = B_i^H w, e_i = B_i^H B_j and f_i =
    // B_i^H B_{j-1} (with w = H B_j, alpha_j = s_j^2 Re d_j), so that
    // q_i^H w1 = s_i (s_j d_i + c_j e_i + c_p f_i) with c_j = -alpha_j s_j and
    // c_p = -beta_{j-1} s_{j-1}.  The overlaps e_i and f_i of the stored
    // vectors carry their orthogonality error into the projections, which is
    // what removing the three-term part first achieves: orthogonalising the
    // raw product would multiply that error by |H q_j| / beta_j (the energy
    // over the residual) per iteration and lose orthogonality within a few
    // iterations on long chains.
    const zd* Bj = basis(j);
    const zd* Bp = basis(j > 0 ? j - 1 : 0);
    double* red = (double*)tjm_lds.gemm;            // free between products
    for (int i0 = 0; i0 < nq; i0 += 8) {
      const int nu = nq - i0 < 8 ? nq - i0 : 8;
      const zd* bp[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) bp[u] = basis(i0 + (u < nu ? u : 0));
      switch (nu) {
        case 1: lz_project3<1>(bp, w, Bj, Bp, n, i0, red); break;
        case 2: lz_project3<2>(bp, w, Bj, Bp, n, i0, red); break;
        case 3: lz_project3<3>(bp, w, Bj, Bp, n, i0, red); break;
        case 4: lz_project3<4>(bp, w, Bj, Bp, n, i0, red); break;
        case 5: lz_project3<5>(bp, w, Bj, Bp, n, i0, red); break;
        case 6: lz_project3<6>(bp, w, Bj, Bp, n, i0, red); break;
        case 7: lz_project3<7>(bp, w, Bj, Bp, n, i0, red); break;
        default: lz_project3<8>(bp, w, Bj, Bp, n, i0, red); break;
      }
    }
    tjm_sync();
    {
      double dj = 0.0;
      for (int wv = 0; wv < TJM_NWAVE; ++wv) dj += red[((long)wv * TJM_KMAX + j) * 6];
      const double aj = dj * sj * sj;
      const double cj = -aj * sj;
      const double cp = j > 0 ? -Lz.beta[j - 1] * Lz.scale[j - 1] : 0.0;
      for (int i = tid; i < nq; i += TJM_NT) {
        double v6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        for (int wv = 0; wv < TJM_NWAVE; ++wv)
          for (int k = 0; k < 6; ++k) v6[k] += red[((long)wv * TJM_KMAX + i) * 6 + k];
        const double si = Lz.scale[i];
        const double hr = si * (sj * v6[0] + cj * v6[2] + cp * v6[4]);
        const double hi = si * (sj * v6[1] + cj * v6[3] + cp * v6[5]);
        Lz.hre[i] = hr; Lz.him[i] = hi;
        // coefficient of B_i in w' = s_j w + c_j B_j + c_p B_{j-1} - sum_i h_i s_i B_i
        Lz.hsre[i] = -hr * si + (i == j ? cj : 0.0) + (j > 0 && i == j - 1 ? cp : 0.0);
        Lz.hsim[i] = -hi * si;
        if (i == j) Lz.alpha[j] = aj;
      }
    }
    tjm_sync();
    // w' = w1 - sum_i h_i q_i, into B_{j+1} (w itself where the basis is
    // full: w' is then only needed for beta)
    zd* nb = j + 1 < m_max ? basis(j + 1) : w;
    double bn = lz_axpy(basis, nq, Lz.hsre, Lz.hsim, w, sj, nb, n);
    bn = sqrt(blk_sum(bn, S));
    tridiag_exp_e0(j + 1, t, Lz);
    tjm_sync();
    if (tid == 0) {
      double cj = sqrt(Lz.cre[j] * Lz.cre[j] + Lz.cim[j] * Lz.cim[j]);
      Lz.done = (bn * cj <= tol || j == m_max - 1) ? 1 : 0;
      Lz.beta[j] = bn;
      Lz.scale[j + 1 < TJM_KMAX ? j + 1 : j] = 1.0 / bn;
    }
    tjm_sync();
    used = j + 1;
    if (Lz.done) break;
  }
  // v = b0 * sum_i c_i q_i = b0 * sum_i (c_i s_i) B_i, in place (B_0 = v is
  // read before it is written, entry by entry)
  for (int i = tid; i < used; i += TJM_NT) {
    Lz.hsre[i] = b0 * Lz.scale[i] * Lz.cre[i];
    Lz.hsim[i] = b0 * Lz.scale[i] * Lz.cim[i];
  }
  tjm_sync();
  lz_axpy(basis, used, Lz.hsre, Lz.hsim, nullptr, 0.0, v, n);
  tjm_sync();
  return used;
}
