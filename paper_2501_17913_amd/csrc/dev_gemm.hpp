// Workgroup complex GEMM on CDNA4 matrix cores.
//
// A complex product C = A B is computed as a real product of the embeddings
//     Ar[i][2k+p]        = (Re A[i][k], Im A[i][k])[p]
//     Br[2k+p][2j+q]     = [[Re B, Im B], [-Im B, Re B]][p][q]  (of B[k][j])
// so that Cr[i][2j+q] = (Re C[i][j], Im C[i][j])[q]: 8 real flops per complex
// multiply-add, no extra work.  The real product runs on
// v_mfma_{f64,f32}_16x16x4 (16 rows x 8 complex columns per instruction, two
// complex k per instruction); interleaved (re, im) storage is the A operand
// as is, the B operand is expanded when its fragment is read.  Operand
// panels go through LDS; ragged edges are zero-padded there and masked on
// the store.
#pragma once
#include <dev_common.hpp>

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Output layout of one 16 x 16 result: lane group q = lane/16 and register
// r of a lane hold row row(q, r) of column lane%16.
template <> struct Mfma<double> {
  typedef v4d acc_t;
  static TJM_DEV int row(int q, int r) { return 4 * r + q; }
  static TJM_DEV acc_t zero() { acc_t z = {0.0, 0.0, 0.0, 0.0}; return z; }
  static TJM_DEV acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Mfma<float> {
  typedef v4f acc_t;
  static TJM_DEV int row(int q, int r) { return 4 * q + r; }
  static TJM_DEV acc_t zero() { acc_t z = {0.f, 0.f, 0.f, 0.f}; return z; }
  static TJM_DEV acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// A complex matrix operand op(X) with X stored row-major (leading dimension
// ld) as cplx<S>; batch b starts bs elements after batch b-1.
//   trans = false: op(X)[i][k] = X[i][k]     trans = true: op(X)[i][k] = X[k][i]
//   conj applies complex conjugation on top.
template <typename S> struct CMat {
  const cplx<S>* p;
  int ld;
  long bs;
  bool trans;
  bool conj;
};

template <typename S> TJM_DEV CMat<S> cmat(const cplx<S>* p, int ld, long bs = 0,
                                           bool trans = false, bool conj = false) {
  CMat<S> m; m.p = p; m.ld = ld; m.bs = bs; m.trans = trans; m.conj = conj; return m;
}

template <typename T, typename S>
TJM_DEV cplx<T> cmat_get(const CMat<S>& m, int b, int i, int k) {
  const cplx<S>* q = m.p + (long)b * m.bs + (m.trans ? ((long)k * m.ld + i) : ((long)i * m.ld + k));
  cplx<S> v = *q;
  return cmk((T)v.re, m.conj ? (T)(-v.im) : (T)v.im);
}

// LDS staging of one k-chunk: A panel (BM x BK) stored k-major, B panel
// (BK x BN) stored row-major, both converted to the compute type; padded rows
// keep the fragment reads free of bank conflicts.
constexpr int GEMM_BM = 64, GEMM_BN = 32, GEMM_BK = 16;
constexpr int GEMM_APAD = GEMM_BM + 2, GEMM_BPAD = GEMM_BN + 2;
constexpr int GEMM_LDS_BYTES = (GEMM_BK * GEMM_APAD + GEMM_BK * GEMM_BPAD) * 16;

template <typename T, typename S>
TJM_DEV void stage_a(const CMat<S>& A, int b, int i0, int k0, int M, int K, cplx<T>* As) {
  // element (i, k) of the panel; walk the index that is contiguous in memory
  for (int e = tjm_tid(); e < GEMM_BM * GEMM_BK; e += TJM_NT) {
    int i, k;
    if (A.trans) { i = e % GEMM_BM; k = e / GEMM_BM; }
    else { k = e % GEMM_BK; i = e / GEMM_BK; }
    cplx<T> v = cmk((T)0, (T)0);
    if (i0 + i < M && k0 + k < K) v = cmat_get<T>(A, b, i0 + i, k0 + k);
    As[k * GEMM_APAD + i] = v;
  }
}

template <typename T, typename S>
TJM_DEV void stage_b(const CMat<S>& B, int b, int k0, int j0, int K, int N, cplx<T>* Bs) {
  for (int e = tjm_tid(); e < GEMM_BK * GEMM_BN; e += TJM_NT) {
    int k, j;
    if (B.trans) { k = e % GEMM_BK; j = e / GEMM_BK; }
    else { j = e % GEMM_BN; k = e / GEMM_BN; }
    cplx<T> v = cmk((T)0, (T)0);
    if (k0 + k < K && j0 + j < N) v = cmat_get<T>(B, b, k0 + k, j0 + j);
    Bs[k * GEMM_BPAD + j] = v;
  }
}

// Small products: each wavefront owns 32 x 16 complex blocks and feeds the
// matrix cores straight from memory (no LDS, no workgroup barriers).
template <typename T, typename SA, typename SB, typename SC>
TJM_DEV void wave_cgemm(int M, int N, int K, int nb, bool sum_batches,
                        const CMat<SA>& A, const CMat<SB>& B,
                        cplx<SC>* C, int ldc, long cs, bool accumulate) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = tjm_lane();
  const int r16 = lane & 15;
  const int q = lane >> 4;
  const int kq = q >> 1;
  const int kp = q & 1;
  const int cpart = r16 & 1;
  const int nti = (M + 31) / 32, ntj = (N + 15) / 16;
  const int nout = sum_batches ? 1 : nb;
  const int nitems = nout * nti * ntj;
  for (int it = tjm_wave(); it < nitems; it += TJM_NWAVE) {
    const int ob = it / (nti * ntj);
    const int rem = it - ob * (nti * ntj);
    const int i0 = (rem / ntj) * 32;
    const int j0 = (rem % ntj) * 16;
    acc_t acc[2][2];
    acc[0][0] = Mfma<T>::zero(); acc[0][1] = Mfma<T>::zero();
    acc[1][0] = Mfma<T>::zero(); acc[1][1] = Mfma<T>::zero();
    const int b_lo = sum_batches ? 0 : ob;
    const int b_hi = sum_batches ? nb : ob + 1;
    for (int b = b_lo; b < b_hi; ++b) {
      for (int k0 = 0; k0 < K; k0 += 2) {
        const int kc = k0 + kq;
        const bool kin = kc < K;
        T av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const int row = i0 + 16 * t + r16;
          T v = (T)0;
          if (kin && row < M) {
            cplx<T> e = cmat_get<T>(A, b, row, kc);
            v = kp ? e.im : e.re;
          }
          av[t] = v;
          const int col = j0 + 8 * t + (r16 >> 1);
          T w = (T)0;
          if (kin && col < N) {
            cplx<T> e = cmat_get<T>(B, b, kc, col);
            w = (kp == cpart) ? e.re : (kp ? -e.im : e.im);
          }
          bv[t] = w;
        }
        acc[0][0] = Mfma<T>::mma(av[0], bv[0], acc[0][0]);
        acc[0][1] = Mfma<T>::mma(av[0], bv[1], acc[0][1]);
        acc[1][0] = Mfma<T>::mma(av[1], bv[0], acc[1][0]);
        acc[1][1] = Mfma<T>::mma(av[1], bv[1], acc[1][1]);
      }
    }
    cplx<SC>* Cb = C + (long)ob * cs;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        const int col = j0 + 8 * tj + (r16 >> 1);
        if (col >= N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + 16 * ti + Mfma<T>::row(q, r);
          if (row >= M) continue;
          SC* dst = cpart ? &Cb[(long)row * ldc + col].im : &Cb[(long)row * ldc + col].re;
          SC v = (SC)acc[ti][tj][r];
          *dst = accumulate ? (SC)(*dst + v) : v;
        }
      }
  }
}

// C (M x N, row-major ldc, element type SC)
//   sum_batches = true : C  = [C +] sum_{b<nb} op(A_b) op(B_b)
//   sum_batches = false: C_b = [C_b +] op(A_b) op(B_b), C_b = C + b*cs
// T selects the matrix-core precision (double: f64 MFMA, float: f32 MFMA with
// fp32 accumulation).  All threads of the workgroup call it together; the
// workgroup walks 64 x 32 (complex) output tiles, staging k-chunks of 16 in
// LDS (`lds`, GEMM_LDS_BYTES); wavefront w owns the 32 x 16 sub-tile
// (w / 2, w % 2).  The caller synchronises before reading C.
template <typename T, typename SA, typename SB, typename SC>
TJM_DEV void blk_cgemm(int M, int N, int K, int nb, bool sum_batches,
                       const CMat<SA>& A, const CMat<SB>& B,
                       cplx<SC>* C, int ldc, long cs, bool accumulate, void* lds) {
  typedef typename Mfma<T>::acc_t acc_t;
  if (M <= 0 || N <= 0) return;
  if (M < 32 || N < 16 || K < 8) {
    wave_cgemm<T>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate);
    return;
  }
  cplx<T>* As = (cplx<T>*)lds;
  cplx<T>* Bs = As + GEMM_BK * GEMM_APAD;
  const int lane = tjm_lane();
  const int r16 = lane & 15;
  const int q = lane >> 4;           // k sub-index 0..3 inside one instruction
  const int kq = q >> 1;             // complex k offset 0/1
  const int kp = q & 1;              // real/imag part of the k index
  const int cpart = r16 & 1;         // real/imag part of the output column
  const int wi = (tjm_wave() >> 1) * 32;   // sub-tile origin inside the tile
  const int wj = (tjm_wave() & 1) * 16;
  const int nti = (M + GEMM_BM - 1) / GEMM_BM, ntj = (N + GEMM_BN - 1) / GEMM_BN;
  const int nout = sum_batches ? 1 : nb;
  const int ntiles = nout * nti * ntj;
  for (int it = 0; it < ntiles; ++it) {
    const int ob = it / (nti * ntj);
    const int rem = it - ob * (nti * ntj);
    const int i0 = (rem / ntj) * GEMM_BM;
    const int j0 = (rem % ntj) * GEMM_BN;
    acc_t acc[2][2];
    acc[0][0] = Mfma<T>::zero(); acc[0][1] = Mfma<T>::zero();
    acc[1][0] = Mfma<T>::zero(); acc[1][1] = Mfma<T>::zero();
    const int b_lo = sum_batches ? 0 : ob;
    const int b_hi = sum_batches ? nb : ob + 1;
    for (int b = b_lo; b < b_hi; ++b) {
      for (int k0 = 0; k0 < K; k0 += GEMM_BK) {
        stage_a<T>(A, b, i0, k0, M, K, As);
        stage_b<T>(B, b, k0, j0, K, N, Bs);
        tjm_sync();
        const int kend = K - k0 < GEMM_BK ? K - k0 : GEMM_BK;
        for (int kk = 0; kk < kend; kk += 2) {
          const int kc = kk + kq;                 // < GEMM_BK; zero-padded past K
          T av[2], bv[2];
#pragma unroll
          for (int t = 0; t < 2; ++t) {
            const cplx<T> ea = As[kc * GEMM_APAD + wi + 16 * t + r16];
            av[t] = kp ? ea.im : ea.re;
            const cplx<T> eb = Bs[kc * GEMM_BPAD + wj + 8 * t + (r16 >> 1)];
            bv[t] = (kp == cpart) ? eb.re : (kp ? -eb.im : eb.im);
          }
          acc[0][0] = Mfma<T>::mma(av[0], bv[0], acc[0][0]);
          acc[0][1] = Mfma<T>::mma(av[0], bv[1], acc[0][1]);
          acc[1][0] = Mfma<T>::mma(av[1], bv[0], acc[1][0]);
          acc[1][1] = Mfma<T>::mma(av[1], bv[1], acc[1][1]);
        }
        tjm_sync();
      }
    }
    cplx<SC>* Cb = C + (long)ob * cs;
#pragma unroll
    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) {
        const int col = j0 + wj + 8 * tj + (r16 >> 1);
        if (col >= N) continue;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i0 + wi + 16 * ti + Mfma<T>::row(q, r);
          if (row >= M) continue;
          SC* dst = cpart ? &Cb[(long)row * ldc + col].im : &Cb[(long)row * ldc + col].re;
          SC v = (SC)acc[ti][tj][r];
          *dst = accumulate ? (SC)(*dst + v) : v;
        }
      }
  }
}
