// The persistent TJM kernels of one contraction precision.
//
// This file is compiled twice, with TJM_TC = float (complex-FP32 matrix-core
// contractions, the mixed path) and TJM_TC = double (the FP64 path); each
// object defines the launchers of its own precision.
//
// tjm_step_kernel is persistent: a grid of resident workgroups pulls
// trajectory indices from a device work counter, so trajectories with more
// work (jumps, larger bonds, more Lanczos iterations) do not stall the
// others.  One launch applies one step function to every trajectory; the
// per-trajectory MPS lives in HBM between launches, the environments,
// Krylov basis and factorisation workspaces are per-workgroup scratch.
#include <dev_tjm.hpp>
#include "tjm_internal.h"

#ifndef TJM_TC
#error "compile with -DTJM_TC=float or -DTJM_TC=double"
#endif

typedef TJM_TC Tc;

template <typename T>
__global__ __launch_bounds__(TJM_NT, 2) void tjm_step_kernel(TjmParams P, int k) {
  extern __shared__ int dyn[];
  Tjm<T> t(P, dyn, (int)blockIdx.x);
  for (;;) {
    if (threadIdx.x == 0) tjm_lds.item = atomicAdd(P.counter, 1);
    __syncthreads();
    const int item = tjm_lds.item;
    __syncthreads();
    if (item >= P.n_traj) break;
    t.traj_step(item, k);
  }
}

// Psi(0) -> t = 0 observables and Phi = F_0 Psi(0), same work queue
template <typename T>
__global__ __launch_bounds__(TJM_NT, 2) void tjm_init_kernel(TjmParams P) {
  extern __shared__ int dyn[];
  Tjm<T> t(P, dyn, (int)blockIdx.x);
  for (;;) {
    if (threadIdx.x == 0) tjm_lds.item = atomicAdd(P.counter, 1);
    __syncthreads();
    const int item = tjm_lds.item;
    __syncthreads();
    if (item >= P.n_traj) break;
    t.traj_init(item);
  }
}

// The pooled server's resident kernel: whole trajectories of any admitted
// job, taken from the work queue of ServeDev (see tjm_params.h).  Each
// workgroup's scratch is slot blockIdx.x of the pool every job's
// parameters point to, so only one such kernel per pool may be resident.
template <typename T>
__global__ __launch_bounds__(TJM_NT, 2) void tjm_serve_kernel(ServeDev S) {
  extern __shared__ int dyn[];
  for (;;) {
    if (threadIdx.x == 0) {
      int got = -1;
      for (int idle = 0; idle < S.idle_spins;) {
        const unsigned h = __hip_atomic_load(S.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned t = __hip_atomic_load(&S.sh->tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
        if (h < t) {
          if (atomicCAS(S.head, h, h + 1) == h) { got = (int)h; break; }
          continue;                      // another workgroup took item h
        }
        if (__hip_atomic_load(&S.sh->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)) break;
        __builtin_amdgcn_s_sleep(127);
        ++idle;
      }
      tjm_lds.item = got;
    }
    __syncthreads();
    const int it = tjm_lds.item;
    __syncthreads();
    if (it < 0) break;
    const ServeItem w = S.items[it % S.cap];
    const TjmParams& P = S.params[w.job];
    Tjm<T> t(P, dyn, (int)blockIdx.x);
    // the job's buffers come uninitialised (admission launches no kernel:
    // the resident one holds every compute unit): clear what this
    // trajectory accumulates into or may leave unwritten
    {
      double* o = P.obs + (long)w.traj * (P.n_steps + 1) * P.n_obs;
      for (long e = threadIdx.x; e < (long)(P.n_steps + 1) * P.n_obs; e += TJM_NT) o[e] = 0.0;
      for (int i = threadIdx.x; i < TJM_NSTAT; i += TJM_NT) P.tstats[(long)w.traj * TJM_NSTAT + i] = 0ull;
      if (threadIdx.x == 0) P.tflags[w.traj] = 0;
      __syncthreads();
    }
    t.traj_init(w.traj);
    for (int k = 1; k <= P.n_steps; ++k) {
      t.traj_step(w.traj, k);
      if (threadIdx.x == 0)                // progress of the job, read by the host
        __hip_atomic_fetch_add(&S.steps[w.job], 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    // every thread's writes of the trajectory reach device scope before the
    // count: a fence orders only its own wavefront's stores, and the barrier
    // alone keeps them within the workgroup
    __threadfence();
    __syncthreads();
    // the workgroup that finishes a job's last trajectory reduces the job
    // (mean, standard error, statistics) into the host's buffers, so that
    // finishing a job needs no further device work
    if (threadIdx.x == 0) tjm_lds.pick = atomicAdd(&S.count[w.job], 1);
    __syncthreads();
    if (tjm_lds.pick == P.n_traj - 1) {
      __threadfence();
      if (threadIdx.x == 0) S.count[w.job] = 0;      // every other trajectory of the job has counted
      const long entries = (long)(P.n_steps + 1) * P.n_obs;
      for (long e = threadIdx.x; e < entries; e += TJM_NT)
        tjm_reduce_entry(P.obs, P.n_traj, entries, e, P.serve_mean, P.serve_sem);
      for (int i = threadIdx.x; i <= TJM_NSTAT; i += TJM_NT) {
        unsigned long long s = 0;
        if (i < TJM_NSTAT)
          for (int q = 0; q < P.n_traj; ++q) s += P.tstats[(long)q * TJM_NSTAT + i];
        else
          for (int q = 0; q < P.n_traj; ++q) s += P.tflags[q] != 0;
        P.serve_stats[i] = s;
      }
      __threadfence_system();            // each thread's results, before the done flag
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      __threadfence_system();
      __hip_atomic_store(&S.done[it % S.cap], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

#define TJM_CAT2(a, b) a##b
#define TJM_CAT(a, b) TJM_CAT2(a, b)
#define TJM_SUFFIX TJM_CAT(_, TJM_TC)

hipError_t TJM_CAT(tjm_blocks_per_cu, TJM_SUFFIX)(int L, int* blocks) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, tjm_step_kernel<Tc>, TJM_NT, tjm_dyn_lds_bytes(L));
}

hipError_t TJM_CAT(tjm_launch_step, TJM_SUFFIX)(const TjmParams& P, int k, int workers, hipStream_t s) {
  const size_t dyn = tjm_dyn_lds_bytes(P.L);
  if (k == 0)
    hipLaunchKernelGGL(tjm_init_kernel<Tc>, dim3(workers), dim3(TJM_NT), dyn, s, P);
  else
    hipLaunchKernelGGL(tjm_step_kernel<Tc>, dim3(workers), dim3(TJM_NT), dyn, s, P, k);
  return hipGetLastError();
}

hipError_t TJM_CAT(tjm_launch_serve, TJM_SUFFIX)(const ServeDev& S, int workers, int L_max, hipStream_t s) {
  hipLaunchKernelGGL(tjm_serve_kernel<Tc>, dim3(workers), dim3(TJM_NT), tjm_dyn_lds_bytes(L_max), s, S);
  return hipGetLastError();
}

