// Workgroup execution model of the TJM kernels on CDNA4 (gfx950).
//
// Every device routine in this library is written against the few names
// below: one workgroup of TJM_NT threads cooperates on one trajectory, split
// into 64-wide wavefronts.  Keeping the vocabulary this small keeps the
// contraction, factorisation and sweep code independent of launch details.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TJM_DEV __device__ __forceinline__
#define TJM_DEVNI __device__ __noinline__
#define TJM_SHARED __shared__

#ifndef TJM_NT
#define TJM_NT 256                  // threads per workgroup (4 wavefronts)
#endif
#define TJM_WAVE 64                 // CDNA wavefront width
#define TJM_NWAVE (TJM_NT / TJM_WAVE)

TJM_DEV int tjm_tid() { return (int)threadIdx.x; }
TJM_DEV int tjm_lane() { return (int)(threadIdx.x & (TJM_WAVE - 1)); }
TJM_DEV int tjm_wave() { return (int)(threadIdx.x / TJM_WAVE); }
TJM_DEV void tjm_sync() { __syncthreads(); }

// Butterfly exchange inside a wavefront.
TJM_DEV double tjm_shfl_xor(double v, int m) { return __shfl_xor(v, m, TJM_WAVE); }
TJM_DEV float tjm_shfl_xor(float v, int m) { return __shfl_xor(v, m, TJM_WAVE); }
TJM_DEV int tjm_shfl_xor(int v, int m) { return __shfl_xor(v, m, TJM_WAVE); }
// value held by lane `src` of this wavefront
TJM_DEV double tjm_shfl(double v, int src) { return __shfl(v, src, TJM_WAVE); }

TJM_DEV uint32_t tjm_mulhi(uint32_t a, uint32_t b) { return __umulhi(a, b); }

// constant-rate (100 MHz) device clock, for phase timing
TJM_DEV unsigned long long tjm_clock() { return (unsigned long long)wall_clock64(); }
