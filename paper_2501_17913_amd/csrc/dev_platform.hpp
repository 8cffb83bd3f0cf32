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

// Lane exchange inside rows of 16 lanes by a DPP move (the VALU reads the
// partner lane's register; no LDS crossbar, no address computation).  CTRL
// is the DPP control code: 0xB1 takes lane ^ 1 and 0x4E lane ^ 2 (quad
// permutations), 0x141 mirrors each half row (lane i of 8 takes 7 - i),
// 0x140 mirrors each row (i of 16 takes 15 - i).  Every lane of the row must
// be active.
template <int CTRL>
TJM_DEV double tjm_dpp(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over aligned groups of G consecutive lanes (G a power of two <= 64);
// every lane of a group receives the same bits (each step adds a lane's
// value and its partner's, and addition commutes), so decisions taken on
// the sum agree across the group.  Up to 16 lanes by DPP moves, beyond that
// by lane shuffles.
template <int G>
TJM_DEV double tjm_grp_sum(double v) {
  if constexpr (G >= 2) v += tjm_dpp<0xB1>(v);
  if constexpr (G >= 4) v += tjm_dpp<0x4E>(v);
  if constexpr (G >= 8) v += tjm_dpp<0x141>(v);
  if constexpr (G >= 16) v += tjm_dpp<0x140>(v);
  if constexpr (G >= 32) v += __shfl_xor(v, 16, TJM_WAVE);
  if constexpr (G >= 64) v += __shfl_xor(v, 32, TJM_WAVE);
  return v;
}

TJM_DEV uint32_t tjm_mulhi(uint32_t a, uint32_t b) { return __umulhi(a, b); }

// constant-rate (100 MHz) device clock, for phase timing
TJM_DEV unsigned long long tjm_clock() { return (unsigned long long)wall_clock64(); }
