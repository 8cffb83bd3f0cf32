// Small TJM kernels for CDNA4 (gfx950): work-queue reset, the trajectory
// average, the precision dispatch of the step kernels (tjm_step.hip), and
// the self-test kernels that run one building block as one workgroup.
#include <dev_tjm.hpp>
#include "tjm_internal.h"

__global__ void tjm_reset_kernel(int* c) { *c = 0; }

// Trajectory average (Eq. TJMExpVal) and its standard error, one thread per
// (time, observable) entry, trajectories summed in index order.
__global__ void tjm_reduce_kernel(const double* obs, int n_traj, long entries, double* mean,
                                  double* sem) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= entries) return;
  tjm_reduce_entry(obs, n_traj, entries, e, mean, sem);
}

size_t tjm_dyn_lds_bytes(int L) { return sizeof(int) * (size_t)(3 * L + 4); }

hipError_t tjm_blocks_per_cu(int mixed, int L, int* blocks) {
  return mixed ? tjm_blocks_per_cu_float(L, blocks) : tjm_blocks_per_cu_double(L, blocks);
}

hipError_t tjm_launch_reset(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(tjm_reset_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

hipError_t tjm_launch_step(const TjmParams& P, int k, int workers, hipStream_t s) {
  return P.mixed ? tjm_launch_step_float(P, k, workers, s) : tjm_launch_step_double(P, k, workers, s);
}

hipError_t tjm_launch_reduce(const double* obs, int n_traj, long entries, double* mean,
                             double* sem, hipStream_t s) {
  const int bs = 256;
  hipLaunchKernelGGL(tjm_reduce_kernel, dim3((entries + bs - 1) / bs), dim3(bs), 0, s, obs, n_traj,
                     entries, mean, sem);
  return hipGetLastError();
}

// --------------------------------------------------------------------------
// Self-test kernels: one workgroup running one building block.
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(TJM_NT) void st_cgemm_kernel(int M, int N, int K, int nb, int sum,
    const zd* A, int lda, long bsA, int tA, int cA, const zd* B, int ldb, long bsB, int tB, int cB,
    zd* C, int ldc, long cs, int acc) {
  blk_cgemm_auto<T>(M, N, K, nb, sum != 0, cmat(A, lda, bsA, tA != 0, cA != 0),
                    cmat(B, ldb, bsB, tB != 0, cB != 0), C, ldc, cs, acc != 0, tjm_lds.gemm);
}

__global__ __launch_bounds__(TJM_NT) void st_qr_kernel(int m, int n, zd* X, zd* Q, zd* R, zd* V) {
  blk_qr(m, n, X, Q, R, V);
}

__global__ __launch_bounds__(TJM_NT) void st_svd_kernel(int m, int n, const zd* G, double discard,
    int cap, double deg_tol, int absorb, zd* left, zd* right, double* Sout, int* kout, zd* Wc, zd* Uc, zd* Tg) {
  int k = blk_svd(m, n, G, left, right, absorb != 0, discard, cap, deg_tol, Wc, Uc, Tg);
  if (threadIdx.x == 0) *kout = k;
  for (int j = threadIdx.x; j < k; j += TJM_NT) Sout[j] = tjm_lds.sv.s[tjm_lds.sv.order[j]];
}

struct DenseOp {
  const zd* H;
  int n;
  TJM_DEVNI void apply(const zd* q, zd* y) {
    blk_cgemm<double>(n, 1, n, 1, true, cmat(H, n), cmat(q, 1), y, 1, 0, false, tjm_lds.gemm);
    tjm_sync();
  }
};

__global__ __launch_bounds__(TJM_NT) void st_expm_kernel(int n, const zd* H, zd* v, double t,
    int kmax, double tol, zd* Q, zd* w, int* iters) {
  DenseOp op{H, n};
  int it = blk_expm(op, v, n, t, kmax, tol, Q, w);
  if (threadIdx.x == 0) *iters = it;
}

__global__ void st_philox_kernel(int count, const uint32_t* ctr, uint32_t k0, uint32_t k1, uint32_t* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  uint32_t c[4] = {ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]};
  philox4x32_10(c, k0, k1);
  for (int j = 0; j < 4; ++j) out[4 * i + j] = c[j];
}

// Plain streaming copy (calibration of the HBM traffic counters): every
// byte of src is read once and every byte of dst written once.
__global__ void st_copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

hipError_t tjm_launch_st_copy(const void* src, void* dst, long n16, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(st_copy_kernel, dim3(blocks), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, n16);
  return hipGetLastError();
}

hipError_t tjm_launch_st_cgemm(int mixed, int M, int N, int K, int nb, int sum_batches,
                               const double* A, int lda, long bsA, int transA, int conjA,
                               const double* B, int ldb, long bsB, int transB, int conjB,
                               double* C, int ldc, long csC, int accumulate) {
  if (mixed)
    hipLaunchKernelGGL(st_cgemm_kernel<float>, dim3(1), dim3(TJM_NT), 0, 0, M, N, K, nb, sum_batches,
                       (const zd*)A, lda, bsA, transA, conjA, (const zd*)B, ldb, bsB, transB, conjB,
                       (zd*)C, ldc, csC, accumulate);
  else
    hipLaunchKernelGGL(st_cgemm_kernel<double>, dim3(1), dim3(TJM_NT), 0, 0, M, N, K, nb, sum_batches,
                       (const zd*)A, lda, bsA, transA, conjA, (const zd*)B, ldb, bsB, transB, conjB,
                       (zd*)C, ldc, csC, accumulate);
  return hipGetLastError();
}

hipError_t tjm_launch_st_qr(int m, int n, double* X, double* Q, double* R, double* V) {
  hipLaunchKernelGGL(st_qr_kernel, dim3(1), dim3(TJM_NT), 0, 0, m, n, (zd*)X, (zd*)Q, (zd*)R, (zd*)V);
  return hipGetLastError();
}

hipError_t tjm_launch_st_svd(int m, int n, const double* G, double discard, int cap, double deg_tol,
                             int absorb_left, double* left, double* right, double* S, int* k,
                             double* Wc, double* Uc, double* Tg, hipStream_t s) {
  hipLaunchKernelGGL(st_svd_kernel, dim3(1), dim3(TJM_NT), 0, s, m, n, (const zd*)G, discard, cap,
                     deg_tol, absorb_left, (zd*)left, (zd*)right, S, k, (zd*)Wc, (zd*)Uc, (zd*)Tg);
  return hipGetLastError();
}

hipError_t tjm_launch_st_expm(int n, const double* H, double* v, double t, int kmax, double tol,
                              double* Q, double* w, int* iters) {
  hipLaunchKernelGGL(st_expm_kernel, dim3(1), dim3(TJM_NT), 0, 0, n, (const zd*)H, (zd*)v, t, kmax, tol,
                     (zd*)Q, (zd*)w, iters);
  return hipGetLastError();
}

hipError_t tjm_launch_st_philox(int count, const uint32_t* ctr, uint32_t k0, uint32_t k1,
                                uint32_t* out) {
  const int bs = 64;
  hipLaunchKernelGGL(st_philox_kernel, dim3((count + bs - 1) / bs), dim3(bs), 0, 0, count, ctr, k0, k1, out);
  return hipGetLastError();
}
