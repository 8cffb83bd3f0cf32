// Run description shared by the host runtime and the device kernels.
// All pointers are device pointers; all complex arrays are interleaved
// (re, im) doubles unless a field says otherwise.
#pragma once
#include <stdint.h>

// One nonzero of a local MPO block, seen from an output row: the source
// virtual channel w, the source physical index s (s1*d+s2 for two sites)
// and the value.
struct MixEnt {
  int w;
  int s;
  double re, im;
};

struct TjmParams {
  // sizes and options
  int L, d, Dmax;
  int n_traj, n_steps;
  int chi_max, chi_cap, krylov_max;
  int n_jump, n_obs;                 // n_obs: output columns (site observables, then MPO observables)
  int n_site_obs, n_mpo_obs;         // site observables are columns 0..n_site_obs-1
  int record_bonds;
  int order;                         // 2: Strang-split schedule with sampling layer; 1: first-order splitting
  int tile_mode;                     // contraction tile choices (bit 0: no wide tiles in H_eff products; bit 1: small
                                     // products in 16 x 8 wavefront blocks; bit 2: wide tiles in the other products)
  int mixed;                         // 1: complex-FP32 contractions
  int certify;                       // 1: QR moves with a no-truncation certificate in post-jump sweeps
  double dt, krylov_tol, svd_discard, deg_tol;
  uint64_t seed;
  uint32_t traj_base;                // global id of trajectory 0 of this run

  // model tables
  const int* mpoD;                   // [L+1] MPO bond dimensions
  const int* mixL_ptr;               // [L][Dmax*d+1]      rows w'*d+s'  -> (w, s)
  const MixEnt* mixL;
  const int* mixR_ptr;               // [L][Dmax*d+1]      rows w*d+s'   -> (w', s)
  const MixEnt* mixR;
  const int* mix2_ptr;               // [L-1][Dmax*d*d+1]  rows w''*d*d+s1'*d+s2' -> (w, s1*d+s2)
  const MixEnt* mix2;
  // structured effective Hamiltonians (structured = 1): per site s and class
  // c (0 = left, 1 = right) the channels of that class and the CSR mixing
  // rows (batch b, s_out) -> (0, s_in, value); local terms [s][dp][dp]
  int structured;
  const int* s1_ptr;                 // [L][2][Dmax*d+1]
  const int* s1_chan;                // [L][2][Dmax]
  const int* s1_n;                   // [L][2]
  const double* s1_loc;              // [L][d][d] complex
  const int* s2_ptr;                 // [L-1][2][Dmax*d*d+1]
  const int* s2_chan;                // [L-1][2][Dmax]
  const int* s2_n;                   // [L-1][2]
  const double* s2_loc;              // [L-1][d*d][d*d] complex
  const int* env_st;                 // [L+1] identity channel of L_b (left-canonical left part)
  const int* env_en;                 // [L+1] identity channel of R_b (right-canonical right part)
  const int* lr_chan;                // [L+1][Dmax] the other channels of bond b
  const int* lr_n;                   // [L+1]
  // MPO observables q < n_mpo_obs (column n_site_obs + q): bond dimensions
  // and right-environment mixing rows in the layout of mixR_ptr
  int oDmax;
  const int* oD;                     // [n_mpo_obs][L+1]
  const int* omixR_ptr;              // [n_mpo_obs][L][oDmax*d+1], entries in mixR
  const double* Dhalf;               // [L][d][d] complex: D_l[dt/2]
  const double* Dfull;               // [L][d][d] complex: D_l[dt]
  const double* jump_op;             // [n_jump][d][d] complex
  const double* jump_rate;           // [n_jump]
  const int* jump_site;              // [n_jump]
  const int* jptr;                   // [L+1] CSR: jumps of site s are jidx[jptr[s]..jptr[s+1])
  const int* jidx;
  const int* optr;                   // [L+1] CSR of observables per site
  const int* oidx;
  const double* obs_op;              // [n_obs][d][d] complex
  const double* init_sites;          // [L][d] complex product state
  int init_mps;                      // 1: Psi(0) is the MPS below instead of init_sites
  const double* init_tensors;        // Psi(0) site tensors in the trajectory layout (site_off), complex
  const int* init_bonds;             // [L+1] bonds of Psi(0)

  // layout of one trajectory MPS (complex doubles)
  const long* site_off;              // [L+1]
  long mps_cap;
  const int* bond_cap;               // [L+1]

  // per-trajectory state
  double* mps;                       // [n_traj][mps_cap] complex
  int* bonds;                        // [n_traj][L+1]
  double* obs;                       // [n_traj][n_steps+1][n_obs]
  int* jlog;                         // [n_traj][2*n_steps]
  int* blog;                         // [n_traj][n_steps][L+1] (if record_bonds)
  unsigned long long* tstats;        // [n_traj][TJM_NSTAT]
  int* tflags;                       // [n_traj] nonzero: numerical failure

  // per-worker scratch (byte offsets inside one worker's block)
  char* scratch;
  long scratch_stride;
  long off_env, env_cap;             // (L+2) slots of env_cap complex (T_c)
  long off_smps;                     // mps_cap complex doubles
  long off_Q, vec_cap;               // krylov_max vectors of vec_cap complex doubles
  long off_w, off_v;                 // vec_cap complex doubles each
  long off_T1, t_cap;                // stage buffer, t_cap complex (T_c)
  long off_X, off_Y, off_Z, off_C, mat_cap;   // mat_cap complex doubles each
  long off_wts;                      // n_jump doubles
  long off_oenv, oenv_cap;           // MPO observables: two FP64 environments of oenv_cap complex
  long off_ot, ot_cap;               //   and their FP64 stage buffer of ot_cap complex

  int* counter;                      // work queue head
  // server jobs only (null otherwise): where the workgroup that finishes the
  // job's last trajectory writes its mean and standard error
  // [n_steps+1][n_obs] and its summed statistics [TJM_NSTAT] plus the count
  // of failed trajectories (host-coherent memory)
  double* serve_mean;
  double* serve_sem;
  unsigned long long* serve_stats;
};

// indices of the per-trajectory statistics
enum {
  TJM_ST_CMAC_MFMA = 0,   // complex multiply-adds issued to the matrix cores
  TJM_ST_CMAC_MIX = 1,    // complex multiply-adds of the MPO mixing stage
  TJM_ST_KRYLOV = 2,      // Lanczos iterations
  TJM_ST_EXPM = 3,        // Lanczos exponentials
  TJM_ST_ONE_SITE = 4,    // 1TDVP bond updates
  TJM_ST_TWO_SITE = 5,    // 2TDVP bond updates
  TJM_ST_FACT = 6,        // QR + SVD factorisations
  TJM_ST_JUMPS = 7,       // jumps applied
  // device-clock ticks (100 MHz) spent by the trajectory's workgroup in:
  TJM_ST_T_TOTAL = 8,     //   the whole step function
  TJM_ST_T_CONTRACT = 9,  //   effective-Hamiltonian and environment contractions
  TJM_ST_T_JUMP = 10,     //   jump processes (dissipation, sweeps, measurement), their factorisations included
  TJM_ST_T_SVD = 11,      //   SVD factorisations
  TJM_ST_T_QR = 12,       //   QR / LQ factorisations
  TJM_ST_T_EXPM = 13,     //   Lanczos exponentials (including their contractions)
  TJM_ST_T_ABSORB = 14,   //   bond-matrix absorption and two-site products
  TJM_ST_T_GEMM = 15,     //   matrix-core products of the effective Hamiltonians (part of contractions)
  TJM_NSTAT = 16
};

// Work queue of the pooled server: one resident kernel per contraction
// precision runs whole trajectories (F_0 .. F_n) of any admitted job.  The
// host appends items to a ring in host-coherent memory and then raises
// `tail`; workgroups take items in order through the device counter `head`
// and mark each finished item in `done` (host-coherent).  A workgroup that
// finds no item for `idle_spins` sleeps (about 8k cycles each), or sees
// `stop`, exits, so the kernel always ends on its own.
struct ServeItem {
  int job;                           // index into params
  int traj;                          // trajectory of that job
};

struct ServeShared {                 // host-coherent, written by the host
  unsigned tail;                     // items appended so far
  int stop;                          // 1: exit as soon as the queue is empty
};

struct ServeDev {
  const TjmParams* params;           // [max_jobs] device copies of the jobs' parameters
  const ServeItem* items;            // [cap] ring (host-coherent)
  int* done;                         // [cap] 1 once item i % cap has finished (host-coherent)
  unsigned long long* steps;         // [max_jobs] step functions finished per job slot (host-coherent)
  int* count;                        // [max_jobs] trajectories finished per job slot (device; zero
                                     // between jobs: the workgroup that finishes a job resets it)
  ServeShared* sh;                   // host-coherent
  unsigned* head;                    // device counter: items taken
  int cap;
  int idle_spins;
};

