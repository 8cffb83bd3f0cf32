/*
 * tjm.h - tensor jump method (TJM) on one MI355X GPU: C ABI.
 *
 * The library runs the per-trajectory TJM of arXiv:2501.17913 (Sec. "Tensor
 * jump method"): a sampling MPS Phi evolved by the step functions
 * F_0 = J D[dt/2], F_j = J D[dt] U[dt], and sampled through
 * F_n = J D[dt/2] U[dt] (Eqs. TimeEvolutionFunctions, SimulationStep), with
 *   U  dynamic TDVP (Sec. "Dynamic TDVP"),
 *   D  the exact dissipative contraction (Eq. DissipativeMPO),
 *   J  the stochastic jump process (Sec. "Stochastic jump process"),
 * averaged over N trajectories (Eq. TJMExpVal).  Inputs follow the
 * paper's list in Sec. "Algorithm / Initialization": the initial state, the
 * Hamiltonian as an MPO, single-site jump operators with rates, dt, T,
 * chi_max and N.
 *
 * Conventions
 *  - Complex arrays are interleaved (re, im) doubles.
 *  - An MPO site tensor is W_l[s_out][s_in][w_{l-1}][w_l] (Methods, MPO
 *    section: O = sum W^{s,s'} |s><s'|); an operator matrix is op[s_out][s_in].
 *  - The basis is (|0>, |1>); sites and jump/observable indices are 0-based.
 *  - Every pointer argument is a HOST pointer.  The library copies all
 *    inputs before returning; outputs are written into caller-allocated host
 *    buffers.  A model handle owns its device memory until tjm_destroy.
 *  - Functions return a tjm_status and never throw; tjm_last_error gives a
 *    message for the last failing call on that handle.
 *  - A model handle is not thread-safe.
 *  - Only local dimension d = 2 is supported (TJM_E_UNSUPPORTED otherwise).
 *
 * Random numbers: each jump process draws two uniforms in [0,1) from
 * Philox4x32-10 (Salmon et al., SC'11) with key (seed lo, seed hi) and
 * counter (traj_base + trajectory, step, branch, 0); branch 0 is the jump
 * process of the sampling MPS (step 0 = F_0), branch 1 the sampling layer.
 * Results therefore do not depend on how trajectories are scheduled.
 */
#ifndef TJM_H
#define TJM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tjm_model tjm_model;

typedef enum {
  TJM_OK = 0,
  TJM_E_INVAL = 1,        /* invalid argument (message says which)            */
  TJM_E_NOMEM = 2,        /* device or host allocation failed                 */
  TJM_E_DEVICE = 3,       /* HIP runtime error / no usable GPU                */
  TJM_E_NUMERIC = 4,      /* non-finite norm in some trajectory               */
  TJM_E_UNSUPPORTED = 5,  /* valid request outside what is implemented        */
  TJM_E_BUSY = 6          /* call out of order (e.g. advance without begin)   */
} tjm_status;

typedef enum {
  TJM_PREC_FP64 = 0,      /* complex128 everywhere                            */
  TJM_PREC_MIXED = 1      /* complex64 contractions on FP32 matrix cores with
                             FP32 accumulation; MPS, Krylov basis,
                             re-orthogonalisation, small exponentials,
                             QR/SVD, jump probabilities and observables FP64 */
} tjm_precision;

typedef struct {
  int precision;          /* tjm_precision, default TJM_PREC_FP64             */
  int chi_cap;            /* hard bond cap of SVD truncation; <= 0 means
                             chi_max; at most 64                              */
  double svd_discard;     /* keep the smallest k with discarded weight
                             sum_{i>=k} s_i^2 <= svd_discard * sum s_i^2;
                             default 1e-12                                    */
  int krylov_max;         /* Lanczos iterations per exponential, 1..32;
                             default 30                                       */
  double krylov_tol;      /* stop when beta_j |[exp(-itT)]_{j,0}| <= tol;
                             <= 0 selects 1e-12 (FP64) or 1e-6 (mixed, the
                             accuracy of its FP32 contractions)              */
  double deg_tol;         /* multiplet tolerance at the cap, default 1e-12    */
  int workers;            /* resident workgroups; <= 0: automatic             */
  int record_bonds;       /* 1: keep bond dimensions after every U[dt]        */
  uint32_t traj_base;     /* global id of trajectory 0 of this run            */
  int device;             /* HIP device ordinal                               */
  int certify_sweeps;     /* normalisation sweeps after a jump: 1 = QR moves
                             where a bound on the smallest singular value
                             proves the SVD would truncate nothing (same state,
                             other gauge), SVD otherwise; 0 = SVD at every
                             bond; < 0 (default) = 1 for TJM_PREC_MIXED and 0
                             for TJM_PREC_FP64                                */
  int sweep_jumps;        /* must be 1 (the default): the jump process runs
                             its sweeps in the printed order (QR sweep for
                             delta p, LQ sweep for the weights, QR moves to
                             the jump site); any other value is rejected
                             with TJM_E_UNSUPPORTED                           */
  int generic_heff;       /* 0 (default): effective Hamiltonians of
                             nearest-neighbour MPOs as two single products
                             (left and right environment) plus a local term,
                             using the identity channels of canonical
                             environments; 1: always the generic contraction
                             L x W x M x R through a (D chi d chi)
                             intermediate.  Same operator, other rounding.  */
  int graph;              /* 1: tjm_run_advance captures its launches (work
                             queue reset and step kernel of every step) in
                             one HIP graph and replays it once, with no host
                             synchronisation between steps (the statistics
                             then split the replay's duration equally over
                             its steps); 0 (default): launches one step at a
                             time and waits for each.  Same kernels, same
                             results                                          */
  int trotter_order;      /* 2 (default): the Strang-split schedule of Eq.
                             (TimeEvolutionFunctions) with the sampling layer
                             D[dt/2]; 1: the first-order splitting of Sec.
                             "Higher-order Trotterization" (the paper's
                             baseline): no F_0, every step F_k = J D[dt] U[dt]
                             with the main draws of step k, observables
                             measured on its result; jump_log then holds the
                             step-k jump at 2k-1 and -1 at 0 and 2k         */
  int tile_mode;          /* tile choices of the contractions, 0..7 (default
                             0); every choice gives the same results, only
                             the speed differs (tjm_autotune picks one per
                             workload).  Bit 0: the effective-Hamiltonian
                             products keep the default 64 x 32 tile instead
                             of the wide 64 x 128 / 128 x 64 (f32) or 64 x 64
                             (f64) ones; bit 1: products below 32 x 16 run in
                             16 x 8 wavefront blocks instead of 32 x 16;
                             bit 2: the environment updates and generic
                             products take the wide tiles too               */
} tjm_options;

typedef struct {
  int n_traj, n_steps, steps_done, workers;
  double init_kernel_ms;          /* duration of the F_0 launch               */
  double step_kernel_ms_total;    /* sum of all step-kernel durations         */
  double step_kernel_ms_last;     /* duration of the most recent step launch  */
  int step_launches;              /* launches counted in the total            */
  unsigned long long cmac_mfma;   /* complex MACs issued to matrix cores      */
  unsigned long long cmac_mix;    /* complex MACs of the MPO mixing stage     */
  unsigned long long krylov_iters, expm_calls;
  unsigned long long one_site, two_site, factorizations, jumps;
  size_t device_bytes;            /* device memory held by the run            */
  /* workgroup-seconds summed over trajectories, by phase: [0] whole step
   * functions, [1] contractions (effective Hamiltonians, environments),
   * [2] jump processes (dissipation, sweeps, measurement, with their
   * factorisations), [3] SVDs, [4] QR/LQ, [5] Lanczos exponentials
   * including their contractions, [6] bond-matrix absorption and two-site
   * products, [7] the matrix-core products inside the effective
   * Hamiltonians (part of [1]).  Phases overlap where stated.             */
  double phase_s[8];
  int failed_traj;                /* trajectories flagged with a non-finite
                                     norm so far (tjm_run_end then returns
                                     TJM_E_NUMERIC)                           */
  unsigned long long cmac_env;    /* unused (0)                               */
} tjm_stats;

/* Fills *opt with the defaults listed above. */
void tjm_default_options(tjm_options *opt);

/*
 * Creates a model: chain length L >= 1, local dimension d (must be 2), the
 * Hamiltonian H0 as an MPO and the jump operators (Eq. Lindblad).
 *   mpo_bond  L+1 MPO bond dimensions, mpo_bond[0] = mpo_bond[L] = 1, each
 *             in 1..8
 *   mpo       concatenation over l of W_l[d][d][mpo_bond[l]][mpo_bond[l+1]]
 *             (complex); H0 must be Hermitian (not checked)
 *   n_jump    number of jump operators (>= 0)
 *   jump_site site of each jump operator (0..L-1)
 *   jump_op   n_jump complex d x d matrices L_m^{[l]}[s_out][s_in]
 *   rate      gamma_m, finite and >= 0
 * The initial state defaults to |0...0>.
 * Errors: TJM_E_INVAL (sizes, boundary bonds, sites, non-finite values,
 * negative rates), TJM_E_UNSUPPORTED (d != 2).  On error *out is NULL.
 */
tjm_status tjm_create(tjm_model **out, int L, int d, const int *mpo_bond, const double *mpo,
                      int n_jump, const int *jump_site, const double *jump_op, const double *rate);

/*
 * Sets the initial state Psi(0) to the product state with site vectors
 * site_vec[l][s] (L x d complex); each must be nonzero and finite.  The state
 * is normalised by the library.
 */
tjm_status tjm_set_initial_product(tjm_model *m, const double *site_vec);

/*
 * Sets Psi(0) to a general MPS (Sec. "Algorithm / Initialization": the
 * initial state is given as an MPS):
 *   bond     L+1 bond dimensions, bond[0] = bond[L] = 1, 1 <= bond[l] <= 64
 *   tensors  the site tensors M_l[s][a][b] (s < d, a < bond[l], b < bond[l+1],
 *            the paper's layout), concatenated over l, interleaved complex
 * Any gauge and any nonzero norm: each trajectory starts from the state
 * brought to right-canonical form by an LQ sweep from the right end and
 * normalised.  A run rejects (TJM_E_INVAL) an MPS with a bond above
 * min(chi_cap, d^l, d^(L-l)).  Errors: TJM_E_INVAL (NULL, bonds, non-finite
 * entries).  The library copies the input.
 */
tjm_status tjm_set_initial_mps(tjm_model *m, const int *bond, const double *tensors);

/*
 * Registers an MPO observable O with the model (Eq. TJMExpVal with O stored
 * as an MPO; Methods, "Resources required for calculating expectation
 * values").  mpo_bond and mpo have the layout of tjm_create; O must be
 * Hermitian (the real part of <Psi|O|Psi> is reported).  Every later run
 * reports the registered MPO observables after its n_obs site observables,
 * in registration order: the output rows of mean, sem and per_traj_obs are
 * n_obs + (number registered) wide.  Each is measured on the same states
 * as the site observables (Psi(0), then Psi_k after the sampling layer),
 * by an MPS-MPO-MPS contraction from the right end in FP64 on both
 * precision paths (L environment updates per observable and step).
 * *index (may be NULL) receives its position among the MPO observables.
 * Errors: TJM_E_INVAL (as tjm_create for the MPO; more than 64
 * observables), TJM_E_BUSY while a run is in progress.  The library copies
 * the input.
 */
tjm_status tjm_add_mpo_observable(tjm_model *m, const int *mpo_bond, const double *mpo, int *index);

/* Removes every registered MPO observable (TJM_E_BUSY during a run). */
tjm_status tjm_clear_mpo_observables(tjm_model *m);

/*
 * One whole run (Sec. "Algorithm"): N = n_traj trajectories from t = 0 to
 * T = n dt (n = T/dt must be an integer within 1e-9), chi_max the bond
 * dimension at which dynamic TDVP switches to 1TDVP, and single-site
 * observables (obs_site[i], obs_op[i] complex d x d).  Outputs:
 *   mean  [(n+1)][n_out]  trajectory average of <Psi_i(t_k)|O|Psi_i(t_k)>
 *                         (real part), t_k = k dt, k = 0..n (Eq. TJMExpVal);
 *                         n_out = n_obs + the MPO observables registered
 *                         with tjm_add_mpo_observable
 *   sem   [(n+1)][n_out]  standard error of that mean, or NULL
 * opt may be NULL (defaults).  Errors: TJM_E_INVAL for bad arguments,
 * TJM_E_NUMERIC if a trajectory's norm became non-finite, TJM_E_NOMEM /
 * TJM_E_DEVICE from the GPU.
 */
tjm_status tjm_run(tjm_model *m, int n_traj, double dt, double T, int chi_max,
                   int n_obs, const int *obs_site, const double *obs_op,
                   uint64_t seed, const tjm_options *opt, double *mean, double *sem);

/*
 * As tjm_run, additionally returning per-trajectory records (each pointer may
 * be NULL):
 *   per_traj_obs [n_traj][n+1][n_out]
 *   jump_log     [n_traj][2n]: index m of the applied jump operator or -1,
 *                in the order F_0, then (sampling layer k, main step k) for
 *                k = 1..n (no main step at k = n)
 *   bond_log     [n_traj][n][L+1]: bond dimensions after U[dt] of step k
 *                (requires opt->record_bonds = 1)
 */
tjm_status tjm_run_traces(tjm_model *m, int n_traj, double dt, double T, int chi_max,
                          int n_obs, const int *obs_site, const double *obs_op,
                          uint64_t seed, const tjm_options *opt, double *mean, double *sem,
                          double *per_traj_obs, int32_t *jump_log, int32_t *bond_log);

/*
 * The same run in three calls, so that a caller can time steps with all
 * inputs resident on the GPU.  tjm_run_begin validates, uploads and applies
 * F_0 to every trajectory (and measures t = 0); tjm_run_advance applies the
 * next `steps` step functions to every trajectory (one kernel launch per
 * step) and waits for them; tjm_run_end reduces and copies the outputs (any
 * pointer may be NULL) and releases the run.  TJM_E_BUSY if called out of
 * order or past step n.
 */
tjm_status tjm_run_begin(tjm_model *m, int n_traj, double dt, double T, int chi_max,
                         int n_obs, const int *obs_site, const double *obs_op,
                         uint64_t seed, const tjm_options *opt);
tjm_status tjm_run_advance(tjm_model *m, int steps);
tjm_status tjm_run_end(tjm_model *m, double *mean, double *sem, double *per_traj_obs,
                       int32_t *jump_log, int32_t *bond_log);

/*
 * Copies the per-trajectory records of the run in progress as they stand
 * after the steps applied so far (layouts as tjm_run_traces; entries of
 * later steps are zero; any pointer may be NULL).  The run continues.
 * TJM_E_BUSY without a run in progress, TJM_E_INVAL for bond_log without
 * record_bonds.
 */
tjm_status tjm_run_read(tjm_model *m, double *per_traj_obs, int32_t *jump_log, int32_t *bond_log);

/* Kernel timings and algorithmic counters of the current or last run. */
tjm_status tjm_get_stats(const tjm_model *m, tjm_stats *out);

/*
 * Autotuning of the launch configuration (tile_mode and resident workers)
 * for one workload.  Every candidate gives the same results, so the tuner
 * compares candidates on identical work: each trial is a separate run of a
 * copy of m with the caller's arguments, seed and options (record_bonds and
 * graph off) on min(n_traj, resident workgroups of one full launch)
 * trajectories; it applies warm_steps untimed step functions, then times
 * timed_steps with HIP events (step-kernel time per trajectory-step).  The
 * candidates are the tile modes that can matter at chi_max (bits 0 and 2
 * only change products of 48 or more rows, so below chi_max = 48 only bit 1
 * is tried), at automatic workers; then, for the best tile mode, one
 * workgroup per compute unit instead of the occupancy limit.
 *
 * Results are cached per key (device architecture and compute units,
 * precision, chain length rounded up to a power of two, chi_max, largest MPO
 * bond, site dimension, trial trajectories, trotter_order): in the process,
 * and, if cache_path is not NULL, in that text file (one line per result,
 * "key tile_mode workers us_per_traj_step"; appended after tuning).  The
 * file's last line for the key, else this process's result for it, is
 * returned without any trial.
 *
 * *tuned receives *base (NULL: defaults) with tile_mode and workers
 * replaced.  warm_steps >= 0, timed_steps >= 1, and their sum at most the
 * run's step count (otherwise TJM_E_INVAL).  m is not changed (its last
 * error is set on failure); it must not have a run in progress
 * (TJM_E_BUSY).  Unreadable cache files are ignored; an unwritable one is
 * not an error (rep->cache_written = 0).
 */
typedef struct {
  int cached;                      /* 1: from the cache, nothing timed          */
  int trials;                      /* trial runs timed                          */
  int trial_traj;                  /* trajectories per trial run                */
  int tile_mode, workers;          /* the choice (as in *tuned)                 */
  int cache_written;               /* 1: the result was appended to cache_path  */
  double us_per_traj_step;         /* step-kernel time of the choice per
                                      trajectory-step, microseconds            */
  double default_us_per_traj_step; /* the same for tile_mode 0 at automatic
                                      workers (0 when cached)                  */
  char key[192];                   /* cache key, NUL-terminated                 */
} tjm_tune_report;

/* Called after each trial (in the caller's thread): its 0-based number, the
 * candidate and its time per trajectory-step in microseconds. */
typedef void (*tjm_tune_progress)(int trial, int tile_mode, int workers, double us_per_traj_step, void *ctx);

tjm_status tjm_autotune(tjm_model *m, int n_traj, double dt, double T, int chi_max,
                        int n_obs, const int *obs_site, const double *obs_op, uint64_t seed,
                        const tjm_options *base, int warm_steps, int timed_steps,
                        const char *cache_path, tjm_tune_progress progress, void *progress_ctx,
                        tjm_options *tuned, tjm_tune_report *rep);

/* Message of the last failing call on m (m may be NULL: last create error). */
const char *tjm_last_error(const tjm_model *m);

/* Releases the model and any run it holds; NULL is ignored. */
void tjm_destroy(tjm_model *m);

/*
 * Serving.  A server executes independent jobs, each one whole run as
 * tjm_run defines it (Sec. "Algorithm"), on one GPU as they are submitted,
 * with continuous batching at the level of trajectories.  Trajectories of
 * different jobs never interact (Eq. TJMExpVal averages within a job), so
 * each precision has one work queue served by a resident kernel whose
 * workgroups run (job, trajectory) items whole, F_0 to F_n, in admission
 * order: the trajectories of a job admitted while others run start as soon
 * as workgroups free up, next to theirs.  Results are bit-identical to
 * tjm_run with the same arguments.
 *
 * Device memory: each admitted job holds its own buffers (tables, MPSs,
 * outputs); the workgroups' scratch is a pool per queue, shaped for the
 * largest chain and bond dimension it serves (and at least the shape
 * given to tjm_server_reserve, budget permitting).  A job larger than the
 * current pool of its precision waits until that queue has drained; a new
 * queue then opens with a pool shaped for every waiting job of that
 * precision that fits the budget.  Admission is first come, first served:
 * the oldest waiting job is admitted once its buffers, and any new pool it
 * needs, fit into the budget not held by admitted jobs and pools; no
 * younger job overtakes it.  Up to 256 jobs per queue are in flight, and up
 * to 2^20 of their trajectories.  The server functions are thread-safe; a
 * model handle passed to tjm_submit is only read during that call (the
 * server keeps a copy).  tjm_options.graph and workers do not apply to
 * server jobs (the resident kernel has no per-step launches, and its
 * workgroup count is the pool's).
 */
typedef struct tjm_server tjm_server;

/* Arguments of one job: those of tjm_run.  The server copies them. */
typedef struct {
  int n_traj;
  double dt;
  double T;
  int chi_max;
  int n_obs;
  const int *obs_site;      /* n_obs sites                                   */
  const double *obs_op;     /* n_obs complex d x d matrices                  */
  uint64_t seed;
  const tjm_options *opt;   /* NULL: defaults; opt->device is replaced by the
                               server's device; workers and graph are not
                               used                                          */
} tjm_run_args;

/* What tjm_wait reports about a finished job. */
typedef struct {
  double latency_s;         /* submission to completion (steady clock)       */
  double queue_s;           /* submission to start                           */
  double run_s;             /* start to completion                           */
  double start_s, end_s;    /* start and completion on the same steady clock
                               (seconds from an arbitrary origin, comparable
                               between jobs of one process)                 */
  int n_traj, n_steps;
  size_t device_bytes;      /* the job's own device buffers (tables, MPSs,
                               outputs) it was admitted with                */
  tjm_stats stats;          /* counters and kernel timings of its run        */
  size_t pool_bytes;        /* scratch pool of its precision while it ran    */
} tjm_job_report;

/*
 * Creates a server on HIP device `device` with a device-memory budget
 * (bytes; 0 selects 85% of the memory free at creation) and starts its
 * dispatcher thread.  Errors: TJM_E_INVAL (NULL, device ordinal),
 * TJM_E_DEVICE (no GPU), TJM_E_NOMEM.
 */
tjm_status tjm_server_create(tjm_server **out, int device, size_t hbm_budget_bytes);

/*
 * Queues one job and returns its id in *job without waiting for it.  The
 * arguments are validated as tjm_run validates them (TJM_E_INVAL,
 * TJM_E_UNSUPPORTED; also more than 2^20 trajectories) and the job is
 * sized; a job whose buffers and a pool of its own shape exceed the whole
 * budget is refused with TJM_E_NOMEM.  TJM_E_BUSY once the server is being
 * destroyed.
 */
tjm_status tjm_submit(tjm_server *s, const tjm_model *m, const tjm_run_args *args, uint64_t *job);

/*
 * Shape hint for the scratch pools: every pool of args->opt's precision
 * that opens from now on is shaped to serve at least a job of this model
 * and these arguments (its chain length and its per-workgroup scratch),
 * where the budget allows it at the time the pool opens; otherwise the pool
 * is shaped as if no hint had been given.  Serving a stream whose largest
 * request shape is known, this spares the drain and reshape that a larger
 * request arriving after a smaller one would otherwise cost.  Several calls
 * combine (the largest of each).  Nothing is allocated or queued.  The
 * resident kernel's LDS grows with the pool's chain length, so a reserved
 * chain longer than the jobs need can lower the workgroups resident per
 * compute unit (on gfx950: two up to 198 sites, one beyond).  Errors:
 * those of tjm_submit's validation, and TJM_E_NOMEM if the shape alone (a
 * job's buffers and its pool) exceeds the budget.
 */
tjm_status tjm_server_reserve(tjm_server *s, const tjm_model *m, const tjm_run_args *args);

/* *done = 1 if the job has finished (successfully or not), else 0.
 * TJM_E_INVAL for an unknown or already collected job. */
tjm_status tjm_poll(tjm_server *s, uint64_t job, int *done);

/* Progress of a job: *traj_done = its trajectories finished so far and
 * *steps_done = its step functions F_k (k >= 1) finished so far over all of
 * its trajectories (n_traj and n_traj * n once it has finished
 * successfully; 0 while it waits for admission).  TJM_E_INVAL for NULL, an
 * unknown or an already collected job. */
tjm_status tjm_job_progress(tjm_server *s, uint64_t job, int *traj_done, unsigned long long *steps_done);

/*
 * Blocks until the job has finished, then writes its outputs into
 * caller-allocated buffers (each may be NULL): mean and sem as in tjm_run,
 * [(n+1)][n_out] each (n_out as in tjm_run), and the report.  Returns the job's own status (the
 * outputs are written only for TJM_OK) and releases the job: its id is
 * unknown afterwards (TJM_E_INVAL).  TJM_E_BUSY if another call is already
 * waiting for the same job.
 */
tjm_status tjm_wait(tjm_server *s, uint64_t job, double *mean, double *sem, tjm_job_report *report);

/* Message of the last failing server call made by the calling thread. */
const char *tjm_server_last_error(void);

/*
 * Stops the server: jobs not yet started are dropped, running jobs are
 * finished, then every resource is released.  No other call on s may be in
 * progress or follow.  NULL is ignored.
 */
void tjm_server_destroy(tjm_server *s);

#ifdef __cplusplus
}
#endif

#endif /* TJM_H */
