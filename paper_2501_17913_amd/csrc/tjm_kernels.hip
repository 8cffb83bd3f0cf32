// TJM kernels for CDNA4 (gfx950).
//
// tjm_step_kernel is persistent: a grid of resident workgroups pulls
// trajectory indices from a device work counter, so trajectories with more
// work (jumps, larger bonds, more Lanczos iterations) do not stall the
// others.  One launch applies one step function to every trajectory; the
// per-trajectory MPS lives in HBM between launches, the environments,
// Krylov basis and factorisation workspaces are per-workgroup scratch.
#include <dev_tjm.hpp>
#include "tjm_internal.h"

template <typename Tc>
__global__ __launch_bounds__(TJM_NT, 2) void tjm_step_kernel(TjmParams P, int k) {
  __shared__ Lds sh;
  extern __shared__ int dyn[];
  Tjm<Tc> t(P, sh, dyn, (int)blockIdx.x);
  for (;;) {
    if (threadIdx.x == 0) sh.item = atomicAdd(P.counter, 1);
    __syncthreads();
    const int item = sh.item;
    __syncthreads();
    if (item >= P.n_traj) break;
    t.traj_step(item, k);
  }
}

// Psi(0) -> t = 0 observables and Phi = F_0 Psi(0), same work queue
template <typename Tc>
__global__ __launch_bounds__(TJM_NT, 2) void tjm_init_kernel(TjmParams P) {
  __shared__ Lds sh;
  extern __shared__ int dyn[];
  Tjm<Tc> t(P, sh, dyn, (int)blockIdx.x);
  for (;;) {
    if (threadIdx.x == 0) sh.item = atomicAdd(P.counter, 1);
    __syncthreads();
    const int item = sh.item;
    __syncthreads();
    if (item >= P.n_traj) break;
    t.traj_init(item);
  }
}

__global__ void tjm_reset_kernel(int* c) { *c = 0; }

// Trajectory average (Eq. TJMExpVal) and its standard error, one thread per
// (time, observable) entry, trajectories summed in index order.
__global__ void tjm_reduce_kernel(const double* obs, int n_traj, int entries, double* mean,
                                  double* sem) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= entries) return;
  double s = 0.0;
  for (int t = 0; t < n_traj; ++t) s += obs[(long)t * entries + e];
  const double mu = s / n_traj;
  double q = 0.0;
  for (int t = 0; t < n_traj; ++t) {
    double x = obs[(long)t * entries + e] - mu;
    q += x * x;
  }
  mean[e] = mu;
  sem[e] = n_traj > 1 ? sqrt(q / ((double)(n_traj - 1) * n_traj)) : 0.0;
}

size_t tjm_dyn_lds_bytes(int L) { return sizeof(int) * (size_t)(3 * L + 4); }

hipError_t tjm_blocks_per_cu(int mixed, int L, int* blocks) {
  if (mixed)
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, tjm_step_kernel<float>, TJM_NT,
                                                        tjm_dyn_lds_bytes(L));
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, tjm_step_kernel<double>, TJM_NT,
                                                      tjm_dyn_lds_bytes(L));
}

hipError_t tjm_launch_reset(int* counter, hipStream_t s) {
  hipLaunchKernelGGL(tjm_reset_kernel, dim3(1), dim3(1), 0, s, counter);
  return hipGetLastError();
}

hipError_t tjm_launch_step(const TjmParams& P, int k, int workers, hipStream_t s) {
  const size_t dyn = tjm_dyn_lds_bytes(P.L);
  if (k == 0) {
    if (P.mixed)
      hipLaunchKernelGGL(tjm_init_kernel<float>, dim3(workers), dim3(TJM_NT), dyn, s, P);
    else
      hipLaunchKernelGGL(tjm_init_kernel<double>, dim3(workers), dim3(TJM_NT), dyn, s, P);
  } else if (P.mixed) {
    hipLaunchKernelGGL(tjm_step_kernel<float>, dim3(workers), dim3(TJM_NT), dyn, s, P, k);
  } else {
    hipLaunchKernelGGL(tjm_step_kernel<double>, dim3(workers), dim3(TJM_NT), dyn, s, P, k);
  }
  return hipGetLastError();
}

hipError_t tjm_launch_reduce(const double* obs, int n_traj, int entries, double* mean,
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
  __shared__ alignas(16) char gl[GEMM_LDS_BYTES];
  blk_cgemm<T>(M, N, K, nb, sum != 0, cmat(A, lda, bsA, tA != 0, cA != 0),
               cmat(B, ldb, bsB, tB != 0, cB != 0), C, ldc, cs, acc != 0, gl);
}

__global__ __launch_bounds__(TJM_NT) void st_qr_kernel(int m, int n, zd* X, zd* Q, zd* R) {
  __shared__ BlkScratch S;
  __shared__ QrLds H;
  blk_qr(m, n, X, Q, R, H, S);
}

__global__ __launch_bounds__(TJM_NT) void st_svd_kernel(int m, int n, const zd* G, double discard,
    int cap, double deg_tol, int absorb, zd* left, zd* right, double* Sout, int* kout, zd* Wc, zd* Uc, zd* Tg) {
  __shared__ BlkScratch S;
  __shared__ SvdLds SL;
  __shared__ alignas(16) char gl[SVD_LDS_BYTES > GEMM_LDS_BYTES ? SVD_LDS_BYTES : GEMM_LDS_BYTES];
  int k = blk_svd(m, n, G, left, right, absorb != 0, discard, cap, deg_tol, Wc, Uc, Tg, SL, S, gl);
  if (threadIdx.x == 0) *kout = k;
  for (int j = threadIdx.x; j < k; j += TJM_NT) Sout[j] = SL.s[SL.order[j]];
}

struct DenseOp {
  const zd* H;
  int n;
  void* gl;
  TJM_DEV void apply(const zd* q, zd* y) {
    blk_cgemm<double>(n, 1, n, 1, true, cmat(H, n), cmat(q, 1), y, 1, 0, false, gl);
    tjm_sync();
  }
};

__global__ __launch_bounds__(TJM_NT) void st_expm_kernel(int n, const zd* H, zd* v, double t,
    int kmax, double tol, zd* Q, zd* w, int* iters) {
  __shared__ BlkScratch S;
  __shared__ LanczosLds Lz;
  __shared__ alignas(16) char gl[GEMM_LDS_BYTES];
  DenseOp op{H, n, gl};
  int it = blk_expm(op, v, n, t, kmax, tol, Q, w, Lz, S);
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

hipError_t tjm_launch_st_qr(int m, int n, double* X, double* Q, double* R) {
  hipLaunchKernelGGL(st_qr_kernel, dim3(1), dim3(TJM_NT), 0, 0, m, n, (zd*)X, (zd*)Q, (zd*)R);
  return hipGetLastError();
}

hipError_t tjm_launch_st_svd(int m, int n, const double* G, double discard, int cap, double deg_tol,
                             int absorb_left, double* left, double* right, double* S, int* k,
                             double* Wc, double* Uc, double* Tg) {
  hipLaunchKernelGGL(st_svd_kernel, dim3(1), dim3(TJM_NT), 0, 0, m, n, (const zd*)G, discard, cap,
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
