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
#include <dev_operand.hpp>

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

// LDS staging of one k-chunk: A panel (BM x BK) stored k-major, B panel
// (BK x BN) stored row-major, both converted to the compute type; padded rows
// keep the fragment reads free of bank conflicts.  A chunk is first loaded
// into registers (so the loads of chunk c+1 are in flight while chunk c runs
// on the matrix cores), then stored to LDS.
// The k-chunk is 32 complex for f32 and 16 for f64 operands, so that both
// fill the same staging area (and a chunk keeps the matrix cores busy long
// enough to hide the next chunk's loads).
// Tile shapes: the workgroup computes BM x BN (complex) output tiles, its
// four wavefronts the (BM/2) x (BN/2) quarters, each as TI x TJ
// instructions of 16 rows x 8 complex columns.  64 x 32 is the default; the
// wide shapes 64 x 128 and 128 x 64 read each operand panel of a 64 x 128
// (or 128 x 64) product once instead of four (two) times.
template <typename T> struct GemmK { static constexpr int BK = 16; };
template <> struct GemmK<float> { static constexpr int BK = 32; };
constexpr int GEMM_BM = 64, GEMM_BN = 32;
constexpr int GEMM_LDS_BYTES = 64 * 1024;          // staging area of every tile shape
template <typename T, int BM, int BN> struct GemmT {
  // a wide tile takes k-chunks of 16 in either precision: a chunk still
  // keeps the matrix cores busy for 128 instructions per wavefront, and the
  // staging registers stay within budget next to 16 accumulators
  static constexpr int BK = BM * BN > GEMM_BM * GEMM_BN ? 16 : GemmK<T>::BK;
  static constexpr int APAD = BM + 2, BPAD = BN + 2;
  static constexpr int AE = BM * BK / TJM_NT;      // A elements per thread
  static constexpr int BE = BK * BN / TJM_NT;      // B elements per thread
  static constexpr int TI = BM / 32, TJ = BN / 16; // instructions per wavefront quarter
  static_assert(AE * TJM_NT == BM * BK && BE * TJM_NT == BK * BN,
                "the workgroup must tile the staging panels exactly");
  static_assert((BK * APAD + BK * BPAD) * (int)sizeof(cplx<T>) <= GEMM_LDS_BYTES, "staging fits its LDS area");
};

// panel coordinates of the u-th element a thread stages
template <int BM, int BK> TJM_DEV void a_coord(bool trans, int u, int& i, int& k) {
  const int e = tjm_tid() + u * TJM_NT;
  if (trans) { i = e % BM; k = e / BM; }
  else { k = e % BK; i = e / BK; }
}
template <int BN, int BK> TJM_DEV void b_coord(bool trans, int u, int& k, int& j) {
  const int e = tjm_tid() + u * TJM_NT;
  if (trans) { k = e % BK; j = e / BK; }
  else { j = e % BN; k = e / BN; }
}

// The raw elements of one k-chunk a thread stages, between their loads and
// their conversion and store to LDS.
template <typename T, int BM, int BN, class OA, class OB> struct GemmStage {
  typedef GemmT<T, BM, BN> G;
  typename OA::raw_t ra[G::AE];
  typename OB::raw_t rb[G::BE];
  bool oa[G::AE], ob[G::BE];
};

template <typename T, int BM, int BN, class OA, class OB>
TJM_DEV void gemm_load(const OA& A, const OB& B, int b, int i0, int j0, int k0, int M, int N, int K,
                       GemmStage<T, BM, BN, OA, OB>& st) {
  typedef GemmT<T, BM, BN> G;
  constexpr int BK = G::BK, AE = G::AE, BE = G::BE;
  int ia[AE], ka[AE], kb[BE], jb[BE];
#pragma unroll
  for (int u = 0; u < AE; ++u) {
    int i, k;
    a_coord<BM, BK>(A.trans, u, i, k);
    ia[u] = i0 + i; ka[u] = k0 + k;
    st.oa[u] = ia[u] < M && ka[u] < K;
  }
#pragma unroll
  for (int u = 0; u < BE; ++u) {
    int k, j;
    b_coord<BN, BK>(B.trans, u, k, j);
    kb[u] = k0 + k; jb[u] = j0 + j;
    st.ob[u] = kb[u] < K && jb[u] < N;
  }
  A.template fetch<AE>(b, ia, ka, st.oa, st.ra);
  B.template fetch<BE>(b, kb, jb, st.ob, st.rb);
}

template <typename T, int BM, int BN, class OA, class OB>
TJM_DEV void gemm_store(const OA& A, const OB& B, const GemmStage<T, BM, BN, OA, OB>& st, cplx<T>* As,
                        cplx<T>* Bs) {
  typedef GemmT<T, BM, BN> G;
  constexpr int BK = G::BK, AE = G::AE, BE = G::BE;
#pragma unroll
  for (int u = 0; u < AE; ++u) {
    int i, k;
    a_coord<BM, BK>(A.trans, u, i, k);
    As[k * G::APAD + i] = A.template value<T>(st.ra[u], st.oa[u]);
  }
#pragma unroll
  for (int u = 0; u < BE; ++u) {
    int k, j;
    b_coord<BN, BK>(B.trans, u, k, j);
    Bs[k * G::BPAD + j] = B.template value<T>(st.rb[u], st.ob[u]);
  }
}

// Lane constants of the real embedding (see the top of this file): lane
// (q = lane / 16, r16 = lane % 16) feeds A the part kp = q % 2 of its complex
// element, and B the entry [[Re, Im], [-Im, Re]][kp][cpart] (cpart = r16 % 2)
// of its complex element, i.e. fa Re + fb Im.  Arithmetic selects, so that the
// fragment reads are plain unconditional LDS loads.
template <typename T> struct EmbedLane {
  T aa, ab, fa, fb;
  TJM_DEV EmbedLane(int kp, int cpart) {
    aa = kp ? (T)0 : (T)1;
    ab = kp ? (T)1 : (T)0;
    fa = kp == cpart ? (T)1 : (T)0;
    fb = kp == cpart ? (T)0 : (kp ? (T)-1 : (T)1);
  }
  TJM_DEV T a(cplx<T> e) const { return aa * e.re + ab * e.im; }
  TJM_DEV T b(cplx<T> e) const { return fa * e.re + fb * e.im; }
};

// Small products: each wavefront owns (16 WI) x (8 WJ) complex blocks (32 x
// 16 by default) and feeds the matrix cores straight from memory (no LDS, no
// workgroup barriers).  Smaller blocks re-read the operands more often but
// give the smallest products enough blocks for all four wavefronts.
template <typename T, int WI = 2, int WJ = 2, class OA, class OB, typename SC>
TJM_DEV void wave_cgemm(int M, int N, int K, int nb, bool sum_batches,
                        const OA& A, const OB& B,
                        cplx<SC>* C, int ldc, long cs, bool accumulate) {
  typedef typename Mfma<T>::acc_t acc_t;
  const int lane = tjm_lane();
  const int r16 = lane & 15;
  const int q = lane >> 4;
  const int kq = q >> 1;
  const int kp = q & 1;
  const int cpart = r16 & 1;
  const EmbedLane<T> emb(kp, cpart);
  constexpr int RB = 16 * WI, CB = 8 * WJ;
  const int nti = (M + RB - 1) / RB, ntj = (N + CB - 1) / CB;
  const int nout = sum_batches ? 1 : nb;
  const int nitems = nout * nti * ntj;
  for (int it = tjm_wave(); it < nitems; it += TJM_NWAVE) {
    const int ob = it / (nti * ntj);
    const int rem = it - ob * (nti * ntj);
    const int i0 = (rem / ntj) * RB;
    const int j0 = (rem % ntj) * CB;
    acc_t acc[WI][WJ];
#pragma unroll
    for (int ti = 0; ti < WI; ++ti)
#pragma unroll
      for (int tj = 0; tj < WJ; ++tj) acc[ti][tj] = Mfma<T>::zero();
    const int b_lo = sum_batches ? 0 : ob;
    const int b_hi = sum_batches ? nb : ob + 1;
    for (int b = b_lo; b < b_hi; ++b) {
#pragma unroll 2
      for (int k0 = 0; k0 < K; k0 += 2) {
        const int kc = k0 + kq;
        const bool kin = kc < K;
        T av[WI], bv[WJ];
#pragma unroll
        for (int t = 0; t < WI; ++t) {
          const int row = i0 + 16 * t + r16;
          const bool oka = kin && row < M;
          const cplx<T> ea = A.template get<T>(b, oka ? row : 0, oka ? kc : 0);
          av[t] = oka ? emb.a(ea) : (T)0;
        }
#pragma unroll
        for (int t = 0; t < WJ; ++t) {
          const int col = j0 + 8 * t + (r16 >> 1);
          const bool okb = kin && col < N;
          const cplx<T> eb = B.template get<T>(b, okb ? kc : 0, okb ? col : 0);
          bv[t] = okb ? emb.b(eb) : (T)0;
        }
#pragma unroll
        for (int ti = 0; ti < WI; ++ti)
#pragma unroll
          for (int tj = 0; tj < WJ; ++tj) acc[ti][tj] = Mfma<T>::mma(av[ti], bv[tj], acc[ti][tj]);
      }
    }
    cplx<SC>* Cb = C + (long)ob * cs;
#pragma unroll
    for (int ti = 0; ti < WI; ++ti)
#pragma unroll
      for (int tj = 0; tj < WJ; ++tj) {
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
// workgroup walks BM x BN (complex) output tiles (GemmT), staging k-chunks in
// LDS (`lds`, GEMM_LDS_BYTES).  The caller synchronises before reading C, or
// before another product accumulates into it (small products return without
// a workgroup barrier).
template <typename T, int BM, int BN, class OA, class OB, typename SC>
TJM_DEV void blk_cgemm_t(int M, int N, int K, int nb, bool sum_batches,
                         const OA& A, const OB& B,
                         cplx<SC>* C, int ldc, long cs, bool accumulate, void* lds) {
  typedef typename Mfma<T>::acc_t acc_t;
  typedef GemmT<T, BM, BN> G;
  if (M <= 0 || N <= 0) return;
  if (M < 32 || N < 16 || K < 8) {
    wave_cgemm<T>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate);
    return;
  }
  constexpr int BK = G::BK, TI = G::TI, TJ = G::TJ;
  cplx<T>* As = (cplx<T>*)lds;
  cplx<T>* Bs = As + BK * G::APAD;
  const int lane = tjm_lane();
  const int r16 = lane & 15;
  const int q = lane >> 4;           // k sub-index 0..3 inside one instruction
  const int kq = q >> 1;             // complex k offset 0/1
  const int kp = q & 1;              // real/imag part of the k index
  const int cpart = r16 & 1;         // real/imag part of the output column
  const EmbedLane<T> emb(kp, cpart);
  const int wi = (tjm_wave() >> 1) * (BM / 2);   // quarter origin inside the tile
  const int wj = (tjm_wave() & 1) * (BN / 2);
  const int nti = (M + BM - 1) / BM, ntj = (N + BN - 1) / BN;
  const int nout = sum_batches ? 1 : nb;
  const int ntiles = nout * nti * ntj;
  const int nkc = (K + BK - 1) / BK;
  for (int it = 0; it < ntiles; ++it) {
    const int ob = it / (nti * ntj);
    const int rem = it - ob * (nti * ntj);
    const int i0 = (rem / ntj) * BM;
    const int j0 = (rem % ntj) * BN;
    acc_t acc[TI][TJ];
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = Mfma<T>::zero();
    const int b_lo = sum_batches ? 0 : ob;
    const int nchunk = (sum_batches ? nb : 1) * nkc;
    GemmStage<T, BM, BN, OA, OB> st;
    gemm_load<T, BM, BN>(A, B, b_lo, i0, j0, 0, M, N, K, st);
    for (int c = 0; c < nchunk; ++c) {
      tjm_sync();                                  // LDS free again
      gemm_store<T, BM, BN>(A, B, st, As, Bs);
      tjm_sync();
      if (c + 1 < nchunk) {                        // next chunk in flight
        const int cn = c + 1;
        gemm_load<T, BM, BN>(A, B, b_lo + cn / nkc, i0, j0, (cn % nkc) * BK, M, N, K, st);
      }
#pragma unroll 2
      for (int kk = 0; kk < BK; kk += 2) {         // zero-padded past K
        const int kc = kk + kq;
        T av[TI], bv[TJ];
#pragma unroll
        for (int t = 0; t < TI; ++t) av[t] = emb.a(As[kc * G::APAD + wi + 16 * t + r16]);
#pragma unroll
        for (int t = 0; t < TJ; ++t) bv[t] = emb.b(Bs[kc * G::BPAD + wj + 8 * t + (r16 >> 1)]);
#pragma unroll
        for (int ti = 0; ti < TI; ++ti)
#pragma unroll
          for (int tj = 0; tj < TJ; ++tj) acc[ti][tj] = Mfma<T>::mma(av[ti], bv[tj], acc[ti][tj]);
      }
    }
    cplx<SC>* Cb = C + (long)ob * cs;
#pragma unroll
    for (int ti = 0; ti < TI; ++ti)
#pragma unroll
      for (int tj = 0; tj < TJ; ++tj) {
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
  tjm_sync();                                      // LDS free for the caller
}

template <typename T, class OA, class OB, typename SC>
TJM_DEV void blk_cgemm(int M, int N, int K, int nb, bool sum_batches, const OA& A, const OB& B,
                       cplx<SC>* C, int ldc, long cs, bool accumulate, void* lds) {
  blk_cgemm_t<T, GEMM_BM, GEMM_BN>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
}

// The same with the tile choice of a run (tile_mode of the options, chosen
// per workload by the autotuner): bit 0 set keeps large products on the
// default tile (no wide shapes), bit 1 set computes small products in 16 x 8
// wavefront blocks.  Every choice sums each output's k terms in the same
// order, so the results do not depend on it.
template <typename T, class OA, class OB, typename SC>
TJM_DEV void blk_cgemm_mode(int mode, int M, int N, int K, int nb, bool sum_batches, const OA& A,
                            const OB& B, cplx<SC>* C, int ldc, long cs, bool accumulate, void* lds);

// The same with the tile shape chosen for the product's size: the wide
// shapes where the output spans them (64 x 128 or 128 x 64 for f32
// contractions, 64 x 64 for f64, whose accumulators take twice the
// registers), the default otherwise.
template <typename T, class OA, class OB, typename SC>
TJM_DEV void blk_cgemm_auto(int M, int N, int K, int nb, bool sum_batches, const OA& A, const OB& B,
                            cplx<SC>* C, int ldc, long cs, bool accumulate, void* lds) {
  if constexpr (sizeof(T) == 4) {
    if (M >= 48 && N >= 96)
      blk_cgemm_t<T, 64, 128>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
    else if (M >= 96 && N >= 48)
      blk_cgemm_t<T, 128, 64>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
    else
      blk_cgemm_t<T, GEMM_BM, GEMM_BN>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
  } else {
    if (M >= 48 && N >= 48)
      blk_cgemm_t<T, 64, 64>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
    else
      blk_cgemm_t<T, GEMM_BM, GEMM_BN>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
  }
}

template <typename T, class OA, class OB, typename SC>
TJM_DEV void blk_cgemm_mode(int mode, int M, int N, int K, int nb, bool sum_batches, const OA& A,
                            const OB& B, cplx<SC>* C, int ldc, long cs, bool accumulate, void* lds) {
  if (M <= 0 || N <= 0) return;
  if ((mode & 2) && (M < 32 || N < 16 || K < 8)) {
    wave_cgemm<T, 1, 1>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate);
    return;
  }
  if (mode & 1)
    blk_cgemm_t<T, GEMM_BM, GEMM_BN>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
  else
    blk_cgemm_auto<T>(M, N, K, nb, sum_batches, A, B, C, ldc, cs, accumulate, lds);
}
