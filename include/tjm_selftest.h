/*
 * tjm_selftest.h - unit entry points into the device building blocks of the
 * TJM library, for testing them in isolation against independent host
 * references.  Each call runs ONE workgroup of the same device routines
 * the TJM kernels use.  All pointers are host pointers; complex arrays are
 * interleaved (re, im) doubles; matrices are row-major.  Returns a
 * tjm_status (TJM_E_INVAL for sizes out of range, TJM_E_DEVICE on HIP
 * errors).
 */
#ifndef TJM_SELFTEST_H
#define TJM_SELFTEST_H

#include <stdint.h>
#include "tjm.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Complex GEMM on the matrix cores (the product of the effective-Hamiltonian
 * contractions, Fig. TDVP):  C = [C +] sum_b op(A_b) op(B_b)  (sum_batches=1)
 * or C_b = [C_b +] op(A_b) op(B_b).  op(X)[i][k] = X[i][k] or, with trans,
 * X[k][i]; conj conjugates.  precision: TJM_PREC_FP64 (f64 matrix cores) or
 * TJM_PREC_MIXED (operands rounded to complex64, f32 matrix cores with f32
 * accumulation).  A_b = A + b*bsA, B_b = B + b*bsB, C_b = C + b*csC
 * (element offsets).  M, N, K <= 512; nb <= 16.  The buffers must hold every
 * element the operation addresses.
 */
tjm_status tjm_selftest_cgemm(int precision, int M, int N, int K, int nb, int sum_batches,
                              const double *A, int lda, long bsA, int transA, int conjA,
                              const double *B, int ldb, long bsB, int transB, int conjB,
                              double *C, int ldc, long csC, int accumulate,
                              long a_elems, long b_elems, long c_elems);

/* Householder QR of X (m x n), m, n <= 128: Q (m x k), R (k x n), k = min(m,n),
 * diag(R) real >= 0. */
tjm_status tjm_selftest_qr(int m, int n, const double *X, double *Q, double *R);

/* Truncated one-sided Jacobi SVD of G (m x n), max(m, n) <= 256, and n <= 128
 * (absorb_left = 0) or m <= 128 (absorb_left = 1): left (m x k) = U or U S,
 * right (k x n) = S V^H or V^H; the factor without S is orthonormal to
 * rounding.  S receives the kept singular values (k doubles, descending),
 * *k the kept rank. */
tjm_status tjm_selftest_svd(int m, int n, const double *G, double discard, int cap,
                            double deg_tol, int absorb_left, double *left, double *right,
                            double *S, int *k);

/*
 * The same truncated SVD for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): G, left, right, S and k are DEVICE pointers of the caller
 * (layouts and sizes as tjm_selftest_svd; left needs m x min(m,n), right
 * min(m,n) x n complex doubles), and the work arrays live in a fixed 1.5 MiB
 * device array of the library (one per GPU, kept until the process ends;
 * its address is looked up once per device).  Limits: max(m, n) <= 256 and
 * n <= 128 (m <= 128 with absorb_left); larger sizes return TJM_E_INVAL.
 * The kernel is launched on `stream` (a hipStream_t; NULL = the null
 * stream) and the call returns without waiting; the caller synchronises
 * before reading the outputs.  No hipMalloc, hipFree or allocating library
 * call is made.  Every call on a GPU uses that GPU's one work array, so
 * calls that overlap on one GPU (other streams, other threads) race: the
 * caller orders them.  Messages go to tjm_last_error(NULL).
 */
tjm_status tjm_svd_noalloc(int m, int n, const double *G, double discard, int cap, double deg_tol,
                           int absorb_left, double *left, double *right, double *S, int *k, void *stream);

/* exp(-i t H) v by the Lanczos routine, H a dense Hermitian n x n matrix
 * (n <= 512) applied through the FP64 matrix-core GEMM.  *iters = Krylov
 * dimension used. */
tjm_status tjm_selftest_expm(int n, const double *H, const double *v, double t,
                             int krylov_max, double tol, double *out, int *iters);

/* Philox4x32-10 on the device: out[4*i..] for counters ctr[4*i..] and key. */
tjm_status tjm_selftest_philox(int count, const uint32_t *ctr, uint32_t k0, uint32_t k1,
                               uint32_t *out);

/* A plain device-to-device streaming copy of n_bytes (a multiple of 16, at
 * most 16 GiB) between two buffers the call allocates, launched reps times
 * (1..1000) on the null stream; *avg_ms receives the mean launch time.  It
 * reads and writes exactly n_bytes per launch, which calibrates the HBM
 * traffic counters (FETCH_SIZE, WRITE_SIZE) against known byte counts. */
tjm_status tjm_selftest_copy(long n_bytes, int reps, double *avg_ms);

#ifdef __cplusplus
}
#endif

#endif /* TJM_SELFTEST_H */
