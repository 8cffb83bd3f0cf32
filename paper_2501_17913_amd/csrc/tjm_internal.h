// Host-side interface between the C ABI (tjm_api.cpp) and the kernels
// (tjm_kernels.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include "tjm.h"
#include "tjm_params.h"

size_t tjm_dyn_lds_bytes(int L);
hipError_t tjm_blocks_per_cu(int mixed, int L, int* blocks);
hipError_t tjm_launch_reset(int* counter, hipStream_t s);
// k = 0: F_0 and t = 0 observables; k >= 1: step function k
hipError_t tjm_launch_step(const TjmParams& P, int k, int workers, hipStream_t s);
// the same per contraction precision (tjm_step.hip, compiled once for each)
hipError_t tjm_blocks_per_cu_float(int L, int* blocks);
hipError_t tjm_blocks_per_cu_double(int L, int* blocks);
hipError_t tjm_launch_step_float(const TjmParams& P, int k, int workers, hipStream_t s);
hipError_t tjm_launch_step_double(const TjmParams& P, int k, int workers, hipStream_t s);
// the pooled server's resident kernel (whole trajectories from a work queue)
hipError_t tjm_launch_serve_float(const ServeDev& S, int workers, int L_max, hipStream_t s);
hipError_t tjm_launch_serve_double(const ServeDev& S, int workers, int L_max, hipStream_t s);
// mean / standard error over trajectories of obs[n_traj][entries], fixed order
hipError_t tjm_launch_reduce(const double* obs, int n_traj, long entries, double* mean,
                             double* sem, hipStream_t s);

hipError_t tjm_launch_st_cgemm(int mixed, int M, int N, int K, int nb, int sum_batches,
                               const double* A, int lda, long bsA, int transA, int conjA,
                               const double* B, int ldb, long bsB, int transB, int conjB,
                               double* C, int ldc, long csC, int accumulate);
hipError_t tjm_launch_st_qr(int m, int n, double* X, double* Q, double* R, double* V);
hipError_t tjm_launch_st_svd(int m, int n, const double* G, double discard, int cap, double deg_tol,
                             int absorb_left, double* left, double* right, double* S, int* k,
                             double* Wc, double* Uc, double* Tg, hipStream_t s);
hipError_t tjm_launch_st_expm(int n, const double* H, double* v, double t, int kmax, double tol,
                              double* Q, double* w, int* iters);
hipError_t tjm_launch_st_philox(int count, const uint32_t* ctr, uint32_t k0, uint32_t k1,
                                uint32_t* out);
hipError_t tjm_launch_st_copy(const void* src, void* dst, long n16, int blocks, hipStream_t s);

// Records msg as the message tjm_last_error(NULL) returns and returns st.
tjm_status tjm_fail_global(tjm_status st, const char* msg);

// Host-side helpers of tjm_api.cpp used by the server (tjm_server.cpp).
// A deep copy of a model's inputs (no run state); NULL if out of memory.
tjm_model* tjm_model_copy(const tjm_model* m);
int tjm_model_d(const tjm_model* m);
int tjm_model_L(const tjm_model* m);
int tjm_model_n_mpo_obs(const tjm_model* m);   // MPO observables registered (output columns after n_obs)
int tjm_model_Dmax(const tjm_model* m);        // largest MPO bond dimension
// Records msg as the model's last error and returns st.
tjm_status tjm_model_fail(tjm_model* m, tjm_status st, const char* msg);
int tjm_model_busy(const tjm_model* m);          // 1: a run is in progress
// Validates a run as tjm_run_begin does and returns the device memory it
// would hold and the resident workgroups it would use (opt->workers caps
// them).  Makes opt->device current.  Errors as tjm_run_begin, message on m.
tjm_status tjm_run_footprint(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                             const int* obs_site, const double* obs_op, const tjm_options* opt,
                             size_t* bytes, int* workers);

// Jobs of the pooled server (tjm_server.cpp), whose trajectories run whole in
// the resident work-queue kernel with the server's scratch pool.
// tjm_pool_plan: the scratch stride a job needs and the device bytes it
// holds besides scratch (validation as tjm_run_begin, no device call).
tjm_status tjm_pool_plan(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                         const int* obs_site, const double* obs_op, const tjm_options* opt, long* stride,
                         size_t* bytes);
// tjm_pool_prepare: allocates and uploads the job (scratch: `workers` slots
// of `stride` bytes at `scratch`) and its kernel parameters into d_slot,
// all on `stream` (the server's, which the job borrows and never destroys),
// waits for that stream, and returns the job handle and its parameters.
tjm_status tjm_pool_prepare(tjm_model* m, int n_traj, double dt, double T, int chi_max, int n_obs,
                            const int* obs_site, const double* obs_op, uint64_t seed, const tjm_options* opt,
                            char* scratch, long stride, int workers, TjmParams* d_slot, hipStream_t stream,
                            void** job, TjmParams* P);
// tjm_pool_finish: once every trajectory has finished, copies the mean, sem
// and statistics the serve kernel reduced the job into (no device work).
tjm_status tjm_pool_finish(tjm_model* m, void* job, double* mean, double* sem, tjm_stats* stats);
// tjm_pool_release: frees the job's device and host buffers; the server
// calls it while none of its resident kernels runs (freeing device memory
// waits for the whole device).
void tjm_pool_release(void* job);

