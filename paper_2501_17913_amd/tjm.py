"""ctypes binding of libtjm.so (include/tjm.h, include/tjm_selftest.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Importing this module fails loudly if libtjm.so has not been
built (python -m paper_2501_17913_amd.build).
"""
import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtjm.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError("libtjm.so is not built: run python -m paper_2501_17913_amd.build")
lib = C.CDLL(_LIB_PATH)

OK, E_INVAL, E_NOMEM, E_DEVICE, E_NUMERIC, E_UNSUPPORTED, E_BUSY = range(7)
PREC_FP64, PREC_MIXED = 0, 1
STATUS_NAMES = {0: "OK", 1: "E_INVAL", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_NUMERIC",
                5: "E_UNSUPPORTED", 6: "E_BUSY"}

EXPORTED = [
    "tjm_default_options", "tjm_create", "tjm_set_initial_product", "tjm_set_initial_mps",
    "tjm_add_mpo_observable", "tjm_clear_mpo_observables", "tjm_run",
    "tjm_run_traces",
    "tjm_run_begin", "tjm_run_advance", "tjm_run_end", "tjm_run_read", "tjm_get_stats", "tjm_autotune",
    "tjm_last_error",
    "tjm_destroy", "tjm_selftest_cgemm", "tjm_selftest_qr", "tjm_selftest_svd", "tjm_svd_noalloc",
    "tjm_selftest_expm", "tjm_selftest_philox", "tjm_selftest_copy",
    "tjm_server_create", "tjm_submit", "tjm_server_reserve", "tjm_poll", "tjm_job_progress", "tjm_wait", "tjm_server_last_error",
    "tjm_server_destroy",
]


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("chi_cap", C.c_int), ("svd_discard", C.c_double),
                ("krylov_max", C.c_int), ("krylov_tol", C.c_double), ("deg_tol", C.c_double),
                ("workers", C.c_int), ("record_bonds", C.c_int), ("traj_base", C.c_uint32),
                ("device", C.c_int), ("certify_sweeps", C.c_int), ("sweep_jumps", C.c_int),
                ("generic_heff", C.c_int), ("graph", C.c_int), ("trotter_order", C.c_int),
                ("tile_mode", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("n_traj", C.c_int), ("n_steps", C.c_int), ("steps_done", C.c_int), ("workers", C.c_int),
                ("init_kernel_ms", C.c_double), ("step_kernel_ms_total", C.c_double),
                ("step_kernel_ms_last", C.c_double), ("step_launches", C.c_int),
                ("cmac_mfma", C.c_ulonglong), ("cmac_mix", C.c_ulonglong),
                ("krylov_iters", C.c_ulonglong), ("expm_calls", C.c_ulonglong),
                ("one_site", C.c_ulonglong), ("two_site", C.c_ulonglong),
                ("factorizations", C.c_ulonglong), ("jumps", C.c_ulonglong),
                ("device_bytes", C.c_size_t), ("phase_s", C.c_double * 8), ("failed_traj", C.c_int),
                ("cmac_env", C.c_ulonglong)]

    PHASES = ("total", "contract", "jump", "svd", "qr", "expm", "absorb", "gemm")

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "phase_s"}
        d["phase_s"] = {k: self.phase_s[i] for i, k in enumerate(self.PHASES)}
        return d


class TuneReport(C.Structure):
    _fields_ = [("cached", C.c_int), ("trials", C.c_int), ("trial_traj", C.c_int), ("tile_mode", C.c_int),
                ("workers", C.c_int), ("cache_written", C.c_int), ("us_per_traj_step", C.c_double),
                ("default_us_per_traj_step", C.c_double), ("key", C.c_char * 192)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["key"] = self.key.decode()
        return d


class RunArgs(C.Structure):
    _fields_ = [("n_traj", C.c_int), ("dt", C.c_double), ("T", C.c_double), ("chi_max", C.c_int),
                ("n_obs", C.c_int), ("obs_site", C.POINTER(C.c_int)), ("obs_op", C.POINTER(C.c_double)),
                ("seed", C.c_uint64), ("opt", C.POINTER(Options))]


class JobReport(C.Structure):
    _fields_ = [("latency_s", C.c_double), ("queue_s", C.c_double), ("run_s", C.c_double),
                ("start_s", C.c_double), ("end_s", C.c_double), ("n_traj", C.c_int), ("n_steps", C.c_int), ("device_bytes", C.c_size_t),
                ("stats", Stats), ("pool_bytes", C.c_size_t)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "stats"}
        d["stats"] = self.stats.as_dict()
        return d


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)
_up = C.POINTER(C.c_uint32)
_vp = C.c_void_p

lib.tjm_default_options.argtypes = [C.POINTER(Options)]
lib.tjm_default_options.restype = None
lib.tjm_create.argtypes = [C.POINTER(_vp), C.c_int, C.c_int, _ip, _dp, C.c_int, _ip, _dp, _dp]
lib.tjm_create.restype = C.c_int
lib.tjm_set_initial_product.argtypes = [_vp, _dp]
lib.tjm_set_initial_product.restype = C.c_int
lib.tjm_set_initial_mps.argtypes = [_vp, _ip, _dp]
lib.tjm_set_initial_mps.restype = C.c_int
lib.tjm_add_mpo_observable.argtypes = [_vp, _ip, _dp, _ip]
lib.tjm_add_mpo_observable.restype = C.c_int
lib.tjm_clear_mpo_observables.argtypes = [_vp]
lib.tjm_clear_mpo_observables.restype = C.c_int
lib.tjm_run.argtypes = [_vp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, _ip, _dp, C.c_uint64,
                        C.POINTER(Options), _dp, _dp]
lib.tjm_run.restype = C.c_int
lib.tjm_run_traces.argtypes = lib.tjm_run.argtypes + [_dp, _ip, _ip]
lib.tjm_run_traces.restype = C.c_int
lib.tjm_run_begin.argtypes = [_vp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, _ip, _dp, C.c_uint64,
                              C.POINTER(Options)]
lib.tjm_run_begin.restype = C.c_int
lib.tjm_run_advance.argtypes = [_vp, C.c_int]
lib.tjm_run_advance.restype = C.c_int
lib.tjm_run_end.argtypes = [_vp, _dp, _dp, _dp, _ip, _ip]
lib.tjm_run_end.restype = C.c_int
lib.tjm_run_read.argtypes = [_vp, _dp, _ip, _ip]
lib.tjm_run_read.restype = C.c_int
lib.tjm_get_stats.argtypes = [_vp, C.POINTER(Stats)]
lib.tjm_get_stats.restype = C.c_int
TuneProgress = C.CFUNCTYPE(None, C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p)
lib.tjm_autotune.argtypes = [_vp, C.c_int, C.c_double, C.c_double, C.c_int, C.c_int, _ip, _dp, C.c_uint64,
                             C.POINTER(Options), C.c_int, C.c_int, C.c_char_p, TuneProgress, C.c_void_p,
                             C.POINTER(Options), C.POINTER(TuneReport)]
lib.tjm_autotune.restype = C.c_int
lib.tjm_last_error.argtypes = [_vp]
lib.tjm_last_error.restype = C.c_char_p
lib.tjm_destroy.argtypes = [_vp]
lib.tjm_destroy.restype = None
lib.tjm_selftest_cgemm.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                   _dp, C.c_int, C.c_long, C.c_int, C.c_int,
                                   _dp, C.c_int, C.c_long, C.c_int, C.c_int,
                                   _dp, C.c_int, C.c_long, C.c_int, C.c_long, C.c_long, C.c_long]
lib.tjm_selftest_cgemm.restype = C.c_int
lib.tjm_selftest_qr.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp]
lib.tjm_selftest_qr.restype = C.c_int
lib.tjm_selftest_svd.argtypes = [C.c_int, C.c_int, _dp, C.c_double, C.c_int, C.c_double, C.c_int,
                                 _dp, _dp, _dp, _ip]
lib.tjm_selftest_svd.restype = C.c_int
lib.tjm_svd_noalloc.argtypes = [C.c_int, C.c_int, _vp, C.c_double, C.c_int, C.c_double, C.c_int,
                                _vp, _vp, _vp, _vp, _vp]
lib.tjm_svd_noalloc.restype = C.c_int
lib.tjm_selftest_expm.argtypes = [C.c_int, _dp, _dp, C.c_double, C.c_int, C.c_double, _dp, _ip]
lib.tjm_selftest_expm.restype = C.c_int
lib.tjm_selftest_philox.argtypes = [C.c_int, _up, C.c_uint32, C.c_uint32, _up]
lib.tjm_selftest_philox.restype = C.c_int
lib.tjm_selftest_copy.argtypes = [C.c_long, C.c_int, _dp]
lib.tjm_selftest_copy.restype = C.c_int
lib.tjm_server_create.argtypes = [C.POINTER(_vp), C.c_int, C.c_size_t]
lib.tjm_server_create.restype = C.c_int
lib.tjm_submit.argtypes = [_vp, _vp, C.POINTER(RunArgs), C.POINTER(C.c_uint64)]
lib.tjm_submit.restype = C.c_int
lib.tjm_server_reserve.argtypes = [_vp, _vp, C.POINTER(RunArgs)]
lib.tjm_server_reserve.restype = C.c_int
lib.tjm_poll.argtypes = [_vp, C.c_uint64, _ip]
lib.tjm_poll.restype = C.c_int
lib.tjm_job_progress.argtypes = [_vp, C.c_uint64, _ip, C.POINTER(C.c_ulonglong)]
lib.tjm_job_progress.restype = C.c_int
lib.tjm_wait.argtypes = [_vp, C.c_uint64, _dp, _dp, C.POINTER(JobReport)]
lib.tjm_wait.restype = C.c_int
lib.tjm_server_last_error.argtypes = []
lib.tjm_server_last_error.restype = C.c_char_p
lib.tjm_server_destroy.argtypes = [_vp]
lib.tjm_server_destroy.restype = None


class TjmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def _dptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _iptr(a):
    return None if a is None else a.ctypes.data_as(_ip)


def default_options(**kw):
    o = Options()
    lib.tjm_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Model:
    """A TJM model: chain length, Hamiltonian MPO, jump operators (tjm_create)."""

    def __init__(self, L, mpo, jump_sites, jump_ops, rates, d=2):
        mpo = [_c128(W) for W in mpo]
        bonds = np.array([1] + [W.shape[3] for W in mpo], dtype=np.int32)
        if len(mpo) != L:
            raise ValueError("need one MPO tensor per site")
        flat = np.concatenate([W.reshape(-1) for W in mpo]) if mpo else np.zeros(1, np.complex128)
        self._flat = flat
        js = np.ascontiguousarray(jump_sites, dtype=np.int32)
        jo = _c128(np.asarray(jump_ops).reshape(-1)) if len(js) else np.zeros(1, np.complex128)
        rt = np.ascontiguousarray(rates, dtype=np.float64) if len(js) else np.zeros(1)
        h = _vp()
        st = lib.tjm_create(C.byref(h), int(L), int(d), _iptr(bonds), flat.view(np.float64).ctypes.data_as(_dp),
                            int(len(js)), _iptr(js), jo.view(np.float64).ctypes.data_as(_dp), _dptr(rt))
        if st != OK:
            raise TjmError(st, lib.tjm_last_error(None).decode())
        self.h = h
        self.L = L
        self.d = d
        self.n_mpo_obs = 0

    def add_mpo_observable(self, mpo):
        """Registers an MPO observable (site tensors W[s_out, s_in, w_l, w_r],
        the layout of the Hamiltonian); runs report it after the site
        observables, in registration order.  Returns its column offset among
        the MPO observables."""
        mpo = [_c128(W) for W in mpo]
        if len(mpo) != self.L:
            raise ValueError("need one MPO tensor per site")
        bonds = np.array([1] + [W.shape[3] for W in mpo], dtype=np.int32)
        if any(W.ndim != 4 or W.shape[2] != bonds[l] for l, W in enumerate(mpo)):
            raise ValueError("site tensors must be (d, d, w_left, w_right) with matching neighbouring bonds")
        flat = np.concatenate([W.reshape(-1) for W in mpo])
        idx = C.c_int()
        self._check(lib.tjm_add_mpo_observable(self.h, _iptr(bonds), flat.view(np.float64).ctypes.data_as(_dp),
                                               C.byref(idx)))
        self.n_mpo_obs += 1
        return idx.value

    def clear_mpo_observables(self):
        self._check(lib.tjm_clear_mpo_observables(self.h))
        self.n_mpo_obs = 0

    def _check(self, st):
        if st != OK:
            raise TjmError(st, lib.tjm_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib.tjm_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def set_initial_product(self, site_vecs):
        v = _c128(site_vecs).reshape(-1)
        self._check(lib.tjm_set_initial_product(self.h, v.view(np.float64).ctypes.data_as(_dp)))

    def set_initial_mps(self, tensors):
        """Psi(0) as an MPS: tensors[l] has shape (d, bond[l], bond[l+1])."""
        ts = [_c128(t) for t in tensors]
        if len(ts) != self.L:
            raise ValueError("need one tensor per site")
        bond = np.array([1] + [t.shape[2] for t in ts], dtype=np.int32)
        flat = np.concatenate([t.reshape(-1) for t in ts])
        self._check(lib.tjm_set_initial_mps(self.h, _iptr(bond), flat.view(np.float64).ctypes.data_as(_dp)))

    @staticmethod
    def _obs(observables):
        sites = np.ascontiguousarray([s for s, _ in observables], dtype=np.int32)
        ops = _c128(np.array([o for _, o in observables]).reshape(-1)) if observables else np.zeros(1, np.complex128)
        return sites, ops

    def run(self, n_traj, dt, T, chi_max, observables, seed, options=None, traces=False):
        """Whole run; returns dict with mean, sem (and per_traj, jumps, bonds)."""
        opt = options or default_options()
        n = max(int(round(T / dt)), 0) if dt > 0 and T > 0 else 0
        sites, ops = self._obs(observables)
        no = len(observables) + self.n_mpo_obs
        mean = np.zeros((n + 1, no))
        sem = np.zeros((n + 1, no))
        out = {"mean": mean, "sem": sem}
        if traces:
            per = np.zeros((n_traj, n + 1, no))
            jl = np.zeros((n_traj, 2 * n), dtype=np.int32)
            bl = np.zeros((n_traj, n, self.L + 1), dtype=np.int32) if opt.record_bonds else None
            st = lib.tjm_run_traces(self.h, n_traj, dt, T, chi_max, len(observables), _iptr(sites),
                                    ops.view(np.float64).ctypes.data_as(_dp), C.c_uint64(seed), C.byref(opt),
                                    _dptr(mean), _dptr(sem), _dptr(per), _iptr(jl), _iptr(bl))
            out.update(per_traj=per, jumps=jl, bonds=bl)
        else:
            st = lib.tjm_run(self.h, n_traj, dt, T, chi_max, len(observables), _iptr(sites),
                             ops.view(np.float64).ctypes.data_as(_dp), C.c_uint64(seed), C.byref(opt),
                             _dptr(mean), _dptr(sem))
        self._check(st)
        out["stats"] = self.stats()
        return out

    def begin(self, n_traj, dt, T, chi_max, observables, seed, options=None):
        opt = options or default_options()
        sites, ops = self._obs(observables)
        self._n = max(int(round(T / dt)), 0) if dt > 0 and T > 0 else 0
        self._no = len(observables) + self.n_mpo_obs
        self._nt = n_traj
        self._rec = bool(opt.record_bonds)
        self._check(lib.tjm_run_begin(self.h, n_traj, dt, T, chi_max, len(observables), _iptr(sites),
                                      ops.view(np.float64).ctypes.data_as(_dp), C.c_uint64(seed), C.byref(opt)))

    def advance(self, steps):
        self._check(lib.tjm_run_advance(self.h, int(steps)))

    def end(self, traces=False):
        n, no, nt = self._n, self._no, self._nt
        mean = np.zeros((n + 1, no))
        sem = np.zeros((n + 1, no))
        per = np.zeros((nt, n + 1, no)) if traces else None
        jl = np.zeros((nt, 2 * n), dtype=np.int32) if traces else None
        bl = np.zeros((nt, n, self.L + 1), dtype=np.int32) if (traces and self._rec) else None
        self._check(lib.tjm_run_end(self.h, _dptr(mean), _dptr(sem), _dptr(per), _iptr(jl), _iptr(bl)))
        return {"mean": mean, "sem": sem, "per_traj": per, "jumps": jl, "bonds": bl}

    def read(self):
        """Per-trajectory records of the run in progress (tjm_run_read)."""
        n, no, nt = self._n, self._no, self._nt
        per = np.zeros((nt, n + 1, no))
        jl = np.zeros((nt, 2 * n), dtype=np.int32)
        bl = np.zeros((nt, n, self.L + 1), dtype=np.int32) if self._rec else None
        self._check(lib.tjm_run_read(self.h, _dptr(per), _iptr(jl), _iptr(bl)))
        return {"per_traj": per, "jumps": jl, "bonds": bl}

    def autotune(self, n_traj, dt, T, chi_max, observables, seed, options=None, warm_steps=3, timed_steps=2,
                 cache_path=None, progress=None):
        """tjm_autotune: (tuned Options, report dict) for this run.  progress,
        if given, is called as progress(trial, tile_mode, workers, us) after
        each trial."""
        sites, ops = self._obs(observables)
        tuned = Options()
        rep = TuneReport()
        base = C.byref(options) if options is not None else None
        cp = cache_path.encode() if cache_path else None
        cb = TuneProgress((lambda i, tm, w, us, _ctx: progress(i, tm, w, us)) if progress else 0)
        self._check(lib.tjm_autotune(self.h, n_traj, dt, T, chi_max, len(observables), _iptr(sites), _dptr(ops),
                                     seed, base, int(warm_steps), int(timed_steps), cp, cb, None,
                                     C.byref(tuned), C.byref(rep)))
        return tuned, rep.as_dict()

    def stats(self):
        s = Stats()
        self._check(lib.tjm_get_stats(self.h, C.byref(s)))
        return s.as_dict()


class Server:
    """Serving front end (tjm_server_create / tjm_submit / tjm_poll / tjm_wait)."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        h = _vp()
        self._sc(lib.tjm_server_create(C.byref(h), int(device), C.c_size_t(int(hbm_budget_bytes))))
        self.h = h
        self._jobs = {}

    @staticmethod
    def _sc(st):
        if st != OK:
            raise TjmError(st, lib.tjm_server_last_error().decode())

    @staticmethod
    def _args(n_traj, dt, T, chi_max, observables, seed, options):
        sites, ops = Model._obs(observables)
        opsd = ops.view(np.float64)
        a = RunArgs(n_traj=n_traj, dt=dt, T=T, chi_max=chi_max, n_obs=len(observables),
                    obs_site=_iptr(sites), obs_op=opsd.ctypes.data_as(_dp), seed=seed,
                    opt=C.pointer(options) if options is not None else None)
        return a, (sites, opsd)          # the arrays must outlive the call

    def submit(self, model, n_traj, dt, T, chi_max, observables, seed, options=None):
        """Queues one run of `model`; returns the job id."""
        a, keep = self._args(n_traj, dt, T, chi_max, observables, seed, options)
        job = C.c_uint64()
        self._sc(lib.tjm_submit(self.h, model.h, C.byref(a), C.byref(job)))
        del keep
        n = max(int(round(T / dt)), 0) if dt > 0 and T > 0 else 0
        self._jobs[job.value] = (n, len(observables) + model.n_mpo_obs)
        return job.value

    def reserve(self, model, n_traj, dt, T, chi_max, observables, options=None):
        """tjm_server_reserve: pools of the options' precision that open from
        now on serve at least a job of this shape, budget permitting."""
        a, keep = self._args(n_traj, dt, T, chi_max, observables, 0, options)
        self._sc(lib.tjm_server_reserve(self.h, model.h, C.byref(a)))
        del keep

    def poll(self, job):
        done = C.c_int()
        self._sc(lib.tjm_poll(self.h, C.c_uint64(job), C.byref(done)))
        return bool(done.value)

    def progress(self, job):
        """(trajectories, step functions) of the job finished so far (tjm_job_progress)."""
        n = C.c_int()
        k = C.c_ulonglong()
        self._sc(lib.tjm_job_progress(self.h, C.c_uint64(job), C.byref(n), C.byref(k)))
        return n.value, k.value

    def wait(self, job):
        """Blocks until the job ends; returns dict with mean, sem and report."""
        n, no = self._jobs.pop(job, (0, 0))
        mean = np.zeros((n + 1, no))
        sem = np.zeros((n + 1, no))
        rep = JobReport()
        self._sc(lib.tjm_wait(self.h, C.c_uint64(job), _dptr(mean), _dptr(sem), C.byref(rep)))
        return {"mean": mean, "sem": sem, "report": rep.as_dict()}

    def close(self):
        if getattr(self, "h", None):
            lib.tjm_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


# ---------------------------------------------------------------------------
# self-test wrappers (one workgroup of the device building blocks)
# ---------------------------------------------------------------------------

def _st(status):
    if status != OK:
        raise TjmError(status, lib.tjm_last_error(None).decode())


def selftest_cgemm(precision, M, N, K, A, B, C0=None, nb=1, sum_batches=True, lda=None, ldb=None, ldc=None,
                   bsA=0, bsB=0, csC=0, transA=False, conjA=False, transB=False, conjB=False, accumulate=False):
    A = _c128(A).reshape(-1)
    B = _c128(B).reshape(-1)
    if C0 is None:
        C0 = np.zeros(max(1, (M * N) if sum_batches else nb * M * N), np.complex128)
    Cb = _c128(C0).reshape(-1).copy()
    lda = lda if lda is not None else (M if transA else K)
    ldb = ldb if ldb is not None else (K if transB else N)
    ldc = ldc if ldc is not None else N
    _st(lib.tjm_selftest_cgemm(precision, M, N, K, nb, int(sum_batches),
                               A.view(np.float64).ctypes.data_as(_dp), lda, bsA, int(transA), int(conjA),
                               B.view(np.float64).ctypes.data_as(_dp), ldb, bsB, int(transB), int(conjB),
                               Cb.view(np.float64).ctypes.data_as(_dp), ldc, csC, int(accumulate),
                               A.size, B.size, Cb.size))
    return Cb


def selftest_qr(X):
    X = _c128(X)
    m, n = X.shape
    k = min(m, n)
    Q = np.zeros((m, k), np.complex128)
    R = np.zeros((k, n), np.complex128)
    _st(lib.tjm_selftest_qr(m, n, X.view(np.float64).ctypes.data_as(_dp),
                            Q.view(np.float64).ctypes.data_as(_dp), R.view(np.float64).ctypes.data_as(_dp)))
    return Q, R


def selftest_svd(G, discard=1e-12, cap=1 << 30, deg_tol=1e-12, absorb_left=False):
    G = _c128(G)
    m, n = G.shape
    nc = min(m, n)
    left = np.zeros(m * max(m, n), np.complex128)
    right = np.zeros(max(m, n) * n, np.complex128)
    S = np.zeros(max(m, n))
    k = C.c_int(0)
    _st(lib.tjm_selftest_svd(m, n, G.view(np.float64).ctypes.data_as(_dp), discard, min(cap, 1 << 30), deg_tol,
                             int(absorb_left), left.view(np.float64).ctypes.data_as(_dp),
                             right.view(np.float64).ctypes.data_as(_dp), _dptr(S), C.byref(k)))
    kk = k.value
    return left[:m * kk].reshape(m, kk), S[:kk], right[:kk * n].reshape(kk, n)


def selftest_expm(H, v, t, krylov_max=30, tol=1e-12):
    H = _c128(H)
    v = _c128(v)
    n = v.size
    out = np.zeros(n, np.complex128)
    it = C.c_int(0)
    _st(lib.tjm_selftest_expm(n, H.view(np.float64).ctypes.data_as(_dp), v.view(np.float64).ctypes.data_as(_dp),
                              t, krylov_max, tol, out.view(np.float64).ctypes.data_as(_dp), C.byref(it)))
    return out, it.value


def selftest_philox(counters, k0, k1):
    c = np.ascontiguousarray(counters, dtype=np.uint32).reshape(-1, 4)
    out = np.zeros_like(c)
    _st(lib.tjm_selftest_philox(c.shape[0], c.ctypes.data_as(_up), k0, k1, out.ctypes.data_as(_up)))
    return out


def selftest_copy(n_bytes, reps=5):
    """Mean duration (ms) of a plain streaming copy of n_bytes on the device."""
    ms = C.c_double(0.0)
    _st(lib.tjm_selftest_copy(int(n_bytes), int(reps), C.byref(ms)))
    return ms.value
