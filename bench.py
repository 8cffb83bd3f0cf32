"""Throughput of the TJM step on one MI355X.

One *step* is one step function F_k of the sampling MPS applied to every
trajectory of the batch (dynamic TDVP, both dissipation/jump branches,
observables): one launch of the persistent TJM kernel.  The workload is the
XXX chain L=100, chi_max=64, 4096 trajectories, dt=0.1, T=5 (50 steps),
Neel initial state, relaxation + dephasing at gamma=0.1 on every site,
mixed precision (complex-FP32 matrix-core contractions, FP64 factorisations).

Timed region: the K steps that follow W untimed warmup steps of the same run
(F_0 and uploads happen before; inputs are resident in HBM).  value =
trajectories x K / wall seconds.  The default window (W=5, K=20: steps
6..25) is where the bulk bonds reach chi_max=64 and stay there.  The FP64
path is timed on the same steps for trajectory ids 0..511 (fp64_path), and
the observables of those ids on both paths are compared step by step
(error_vs_fp64: largest difference over trajectories whose jump logs agree,
the number whose jump logs differ, how many exceed 2e-4 and through which
step all stay within it, and the largest difference of the ensemble means,
also in FP64 standard errors).

roofline.traffic (HBM bytes per launch of the step kernel) comes from the
FETCH_SIZE / WRITE_SIZE counter summary in profiles/, scaled by the same
counters read for a plain copy of known size (--copy-calibration), and is
reported only while the kernel sources still hash to the profiled ones.

Prints ONE JSON line.
"""
import hashlib
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "C2": dict(L=40, chi_max=32, n_traj=1024, T=5.0, init="neel"),
    "C3": dict(L=100, chi_max=64, n_traj=4096, T=5.0, init="neel"),
    "C4": dict(L=1000, chi_max=16, n_traj=512, T=2.0, init="zero"),
}
PEAK_TFLOPS = {"mixed": 157.3, "fp64": 78.6}     # MI355X dense FP32 / FP64 matrix peaks
SEED = 0x250117913
CSRC = os.path.join(ROOT, "paper_2501_17913_amd", "csrc")
TRAFFIC = os.path.join(ROOT, "profiles", "tjm_step_kernel_C3_traffic.json")


def kernel_sha():
    """Hash of the device sources: counters taken from other sources are stale."""
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hpp", ".hip", ".h")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def traffic_per_launch(workload, precision, W, K):
    """Calibrated HBM bytes per step launch from the committed counter
    summary, or None if it does not cover these sources and this window."""
    try:
        with open(TRAFFIC) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("kernel_sha") != kernel_sha() or t.get("workload") != workload or t.get("precision") != precision
            or t.get("warmup") != W or t.get("steps") != K):
        return None
    fetch = sum(t["fetch_kib"]) / len(t["fetch_kib"]) * t["fetch_scale"]
    write = sum(t["write_kib"]) / len(t["write_kib"]) * t["write_scale"]
    return 1024.0 * (fetch + write)


def _oracle_sample(args):
    """One process of the CPU baseline: the oracle's own routines timed on a
    random right-canonical MPS of the workload's chain with every bond at
    min(2^b, 2^(L-b), chi_max) (the saturated regime of the timed steps)."""
    L, chi, budget, seed = args
    import numpy as np
    from oracle import model as om, mps_tjm
    rng = np.random.default_rng(seed)
    bonds = [min(2 ** b, 2 ** (L - b), chi) for b in range(L + 1)]
    # every site a random isometry (rows orthonormal over (s, b)): a
    # right-canonical state of norm 1 however long the chain, where a product
    # of unnormalised random tensors would overflow
    psi = []
    for l in range(L):
        a, b = bonds[l], bonds[l + 1]
        g = rng.normal(size=(2 * b, a)) + 1j * rng.normal(size=(2 * b, a))
        q, _ = np.linalg.qr(g)                       # 2b x a, orthonormal columns
        psi.append(q.conj().T.reshape(a, 2, b).transpose(1, 0, 2).copy())
    Ws = om.xxx_mpo(L, 1.0, 0.5)
    jumps = om.relax_dephase_jumps(L, 0.1, 0.1)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    opt = mps_tjm.Options(chi_max=chi)
    stats = mps_tjm.Stats()
    tau = 0.05
    # right environments of the whole chain, as U[dt] rebuilds them
    t0 = time.perf_counter()
    one = np.ones((1, 1, 1), dtype=np.complex128)
    Renv = [None] * (L + 1)
    Renv[L] = one
    for s in range(L - 1, 0, -1):
        Renv[s] = mps_tjm.right_update(Renv[s + 1], psi[s], Ws[s])
    t_env = time.perf_counter() - t0
    # one-site updates (forward Lanczos, QR, environment, backward bond
    # evolution, absorption) of bulk sites, left to right, within the budget
    Lenv = mps_tjm.left_update(one, psi[0], Ws[0])
    for s in range(1, L // 4):
        Lenv = mps_tjm.left_update(Lenv, psi[s], Ws[s])
    s, done = L // 4, 0
    t0 = time.perf_counter()
    while s < L - L // 4 and time.perf_counter() - t0 < budget:
        Le, W, Re = Lenv, Ws[s], Renv[s + 1]
        psi[s] = mps_tjm.expm_krylov(lambda v: mps_tjm.h1_apply(Le, W, Re, v), psi[s], tau, 30, 1e-12, stats)
        A, Cm = mps_tjm.qr_left(psi[s])
        psi[s] = A
        Lenv = mps_tjm.left_update(Lenv, A, Ws[s])
        Cm = mps_tjm.expm_krylov(lambda v: mps_tjm.h0_apply(Lenv, Re, v), Cm, -tau, 30, 1e-12, stats)
        psi[s + 1] = mps_tjm.absorb_right(Cm, psi[s + 1])
        s += 1
        done += 1
    t_site = (time.perf_counter() - t0) / max(done, 1)
    # a jump process without a jump (QR sweep for delta p, LQ sweep back) and
    # the measurement of every observable
    mps_tjm.canonicalize(psi)
    Dh = [om.local_dissipator(jumps, q, tau) for q in range(L)]
    t0 = time.perf_counter()
    mps_tjm.dissipate(psi, Dh)
    mps_tjm.jump_process(psi, jumps, 1.0, 0.5, opt)
    t_jump = time.perf_counter() - t0
    # the measurement: a fixed part (the transfer environments of the whole
    # chain) plus one contraction per observable; timed without observables
    # and with four of bulk sites
    t0 = time.perf_counter()
    mps_tjm.expectation_values(psi, [])
    t_fix = time.perf_counter() - t0
    mid = L // 2
    t0 = time.perf_counter()
    mps_tjm.expectation_values(psi, [(mid, om.Z), (mid + 1, om.Z), (mid, om.X), (mid + 1, om.X)])
    per_obs = max(time.perf_counter() - t0 - t_fix, 0.0) / 4.0
    t_obs = t_fix + len(obs) * per_obs
    step = t_env + 2 * (L - 1) * t_site + 2 * t_jump + t_obs
    return {"updates": done, "t_site": t_site, "t_env": t_env, "t_jump": t_jump, "t_obs": t_obs, "t_step": step}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(L, chi, budget=8.0):
    """The oracle as it stands on the host cores, one process per core with
    single-threaded BLAS (one trajectory per thread, as in the paper's
    runs).  A full saturated step of the FP64 NumPy oracle takes minutes, so
    each process times a bounded sample of one (see _oracle_sample) and the
    rate is the sum over processes of 1 / (estimated seconds per
    trajectory-step)."""
    cores = max(1, min(os.cpu_count() or 1, 16))
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"
    res = []
    with mp.get_context("spawn").Pool(cores) as pool:
        for r in pool.imap_unordered(_oracle_sample, [(L, chi, budget, 1000 + t) for t in range(cores)]):
            res.append(r)
            print("  cpu baseline: %d of %d processes done" % (len(res), cores), file=sys.stderr, flush=True)
    rate = sum(1.0 / r["t_step"] for r in res)
    med = sorted(res, key=lambda r: r["t_step"])[len(res) // 2]
    return {"value": rate, "unit": "trajectory-steps/s", "cores": cores, "kind": "oracle", "cpu": cpu_model(),
            "sample": "per process: the FP64 NumPy oracle's routines on a random right-canonical MPS of the "
                      "L=%d chain with every bond at min(2^b, 2^(L-b), %d), the saturated regime of the timed "
                      "steps: the right-environment rebuild, one-site TDVP updates of bulk sites for %.0f s "
                      "(Lanczos forward, QR, environment update, backward bond evolution, absorption), one jump "
                      "process without a jump, and the measurement without observables and with 4 of bulk sites "
                      "(a fixed part plus a contraction per observable); seconds per trajectory-step = rebuild "
                      "+ 2(L-1) updates + 2 jump processes + measurement of all 2L observables"
                      % (L, chi, budget),
            "median_process": {k: round(v, 4) if isinstance(v, float) else v for k, v in med.items()}}


def copy_calibration(tjm, n_bytes=1 << 30, reps=5):
    ms = tjm.selftest_copy(n_bytes, reps)
    return {"copy_bytes": n_bytes, "reps": reps, "avg_ms": ms, "GB/s": 2 * n_bytes / (ms * 1e-3) / 1e9}


def xxx_job(tjm, models, L, init):
    """The XXX chain of the workloads (J=1, g=0.5, gamma=0.1) from the Neel
    state or |0...0>."""
    mpo, s, o, r = models.xxx_model(L, 1.0, 0.5, 0.1)
    m = tjm.Model(L, mpo, s, o, r)
    m.set_initial_product(models.neel(L) if init == "neel" else models.product_state([0] * L))
    return m


def autotune(tjm, models, L, init, chi, N, T, prec, warm, timed, cache):
    """tjm_autotune for the workload: (tile_mode, workers, report)."""
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
    m = xxx_job(tjm, models, L, init)
    t0 = time.perf_counter()
    def progress(i, tm, w, us):
        print("  autotune trial %d: tile_mode %d workers %d: %.1f us per trajectory-step (%.1fs)"
              % (i, tm, w, us, time.perf_counter() - t0), file=sys.stderr, flush=True)

    tuned, rep = m.autotune(N, 0.1, T, chi, models.zx_observables(L), SEED, tjm.default_options(precision=prec),
                            warm_steps=warm, timed_steps=timed, cache_path=cache, progress=progress)
    m.close()
    rep["tune_wall_s"] = time.perf_counter() - t0
    print("  autotune: tile_mode %d workers %d (%s, %d trials, %.1fs)"
          % (tuned.tile_mode, tuned.workers, "cached" if rep["cached"] else "tuned", rep["trials"],
             rep["tune_wall_s"]), file=sys.stderr, flush=True)
    return tuned.tile_mode, tuned.workers, rep


def measure(tjm, models, L, init, chi, N, T, prec, warmup, K, workers, read_ids=0, deadline=None, tile_mode=0):
    """Run one job on the GPU; time steps warmup+1 .. warmup+K.  With
    read_ids, the records of trajectories 0..read_ids-1 after the window are
    returned too.  With a deadline (perf_counter seconds), the job stops
    early once it is passed and the result says so (partial)."""
    dt = 0.1
    m = xxx_job(tjm, models, L, init)
    opt = tjm.default_options(precision=prec, workers=workers, tile_mode=tile_mode)
    name = "mixed" if prec == tjm.PREC_MIXED else "fp64"
    tb = time.perf_counter()
    m.begin(N, dt, T, chi, models.zx_observables(L), SEED, opt)
    print("  %s F_0 done at %.1fs" % (name, time.perf_counter() - tb), file=sys.stderr, flush=True)
    for k in range(warmup):
        m.advance(1)
        print("  %s warmup step %d of %d done at %.1fs" % (name, k + 1, warmup, time.perf_counter() - tb),
              file=sys.stderr, flush=True)
        if deadline and time.perf_counter() > deadline:
            m.close()
            return {"partial": True, "steps_done": k + 1}
    s0 = m.stats()
    t0 = time.perf_counter()
    for k in range(K):                # each advance returns after its launch has finished
        m.advance(1)
        print("  %s step %d of %d done at %.1fs" % (name, warmup + k + 1, warmup + K, time.perf_counter() - t0),
              file=sys.stderr, flush=True)
        if deadline and k + 1 < K and time.perf_counter() > deadline:
            m.close()
            return {"partial": True, "steps_done": warmup + k + 1}
    wall = time.perf_counter() - t0
    s1 = m.stats()
    rec = None
    if read_ids:
        r = m.read()
        last = warmup + K
        rec = {"per_traj": r["per_traj"][:read_ids, :last + 1], "jumps": r["jumps"][:read_ids, :2 * last + 1]}
    m.close()                         # the rest of the job is not needed for timing
    if s1["failed_traj"]:
        raise RuntimeError("%d trajectories hit a non-finite norm" % s1["failed_traj"])
    launches = s1["step_launches"] - s0["step_launches"]
    kern_ms = s1["step_kernel_ms_total"] - s0["step_kernel_ms_total"]
    cmac = s1["cmac_mfma"] - s0["cmac_mfma"]
    flops_per_launch = 8.0 * cmac / launches
    avg_ms = kern_ms / launches
    phases = {k: s1["phase_s"][k] - s0["phase_s"][k] for k in s1["phase_s"]}
    tot = phases["total"] or 1.0
    return {
        "partial": False, "value": N * K / wall, "wall": wall, "avg_ms": avg_ms, "flops_per_launch": flops_per_launch,
        "achieved_tflops": flops_per_launch / (avg_ms * 1e-3) / 1e12, "workers": s1["workers"],
        "counts": {k: s1[k] - s0[k] for k in ("krylov_iters", "expm_calls", "one_site", "two_site",
                                              "factorizations", "jumps", "cmac_mix")},
        "phase_frac": {k: round(v / tot, 4) for k, v in phases.items() if k != "total"},
        "records": rec,
    }


def compare(a, b, tol=2e-4):
    """Mixed (a) against FP64 (b) records of the same trajectory ids.

    Per trajectory: those whose jump logs differ are counted (a decision
    within the FP32 error of its threshold sends the trajectory elsewhere);
    over the rest, the largest and mean absolute difference of the
    observables, how many exceed tol at some step, and the last step through
    which every one of them stays within tol (in the truncated regime the
    dynamics amplify any difference, FP32 rounding included, step by step).
    Ensemble: the largest difference of the trajectory means over all ids,
    absolute and in units of the FP64 standard error of the mean."""
    same = np.all(a["jumps"] == b["jumps"], axis=1)
    d = np.abs(a["per_traj"] - b["per_traj"])[same]            # traj x step x obs
    out = {"trajectories": int(len(same)), "flipped": int((~same).sum()),
           "max_abs": float(d.max()) if d.size else None, "mean_abs": float(d.mean()) if d.size else None,
           "steps": int(a["per_traj"].shape[1] - 1), "tol": tol}
    if d.size:
        per_step = d.max(axis=(0, 2))
        bad = np.nonzero(per_step > tol)[0]
        out["over_tol"] = int((d.max(axis=(1, 2)) > tol).sum())
        out["within_tol_through_step"] = int(bad[0] - 1) if bad.size else out["steps"]
    n = a["per_traj"].shape[0]
    if n > 1:
        dm = np.abs(a["per_traj"].mean(axis=0) - b["per_traj"].mean(axis=0))
        sem = b["per_traj"].std(axis=0, ddof=1) / np.sqrt(n)
        pos = sem > 0
        out["ensemble_max_abs"] = float(dm.max())
        out["ensemble_max_over_sem"] = float((dm[pos] / sem[pos]).max()) if pos.any() else None
    return out


def serving(tjm, models, K, precision, reserve=True):
    """The first K requests of the serving stream, submitted at their arrival
    times to one tjm_server; latency = submission to completion.  With
    reserve, the server's pools are shaped for the largest request shape
    among them (tjm_server_reserve) before the first arrival."""
    from tests import inputs
    reqs = inputs.serving_stream(K)
    prec = tjm.PREC_MIXED if precision == "mixed" else tjm.PREC_FP64
    built = []
    for q in reqs:                       # host-side model tables, before the clock starts
        mpo, s, o, r = models.xxx_model(q["L"], 1.0, q["g"], q["gamma"])
        m = tjm.Model(q["L"], mpo, s, o, r)
        m.set_initial_product(models.neel(q["L"]))
        built.append(m)
    srv = tjm.Server(0)
    Lr = max(q["L"] for q in reqs)
    chir = max(q["chi_max"] for q in reqs)
    if reserve:                          # the largest request shape of the K requests
        mpo, s, o, r = models.xxx_model(Lr, 1.0, 0.5, 0.1)
        hint = tjm.Model(Lr, mpo, s, o, r)
        srv.reserve(hint, 64, 0.1, 0.1, chir, models.zx_observables(Lr), tjm.default_options(precision=prec))
        hint.close()
    t0 = time.perf_counter()
    ids = []
    for q, m in zip(reqs, built):
        delay = t0 + q["t"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        ids.append(srv.submit(m, q["n_traj"], q["dt"], q["T"], q["chi_max"], models.zx_observables(q["L"]),
                              q["seed"], tjm.default_options(precision=prec)))
    reps = []
    pending = set(range(len(ids)))
    total = sum(q["n_traj"] * q["n_steps"] for q in reqs)
    finished = {i: 0 for i in pending}
    reported, t_rep = 0, time.perf_counter()
    while pending:                        # progress as step functions and jobs finish, in any order
        for i in sorted(pending):
            if srv.poll(ids[i]):
                finished[i] = reqs[i]["n_traj"] * reqs[i]["n_steps"]
                reps.append((i, srv.wait(ids[i])["report"]))
                pending.discard(i)
                print("  request %d done (%d of %d) at %.1fs" % (i, len(reps), len(ids), time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
            else:
                finished[i] = srv.progress(ids[i])[1]
        done = sum(finished.values())
        # every 5% of all trajectory-steps, or any finished after 20 s without a line
        if done >= reported + total // 20 or (done > reported and time.perf_counter() - t_rep > 20.0):
            reported, t_rep = done, time.perf_counter()
            print("  %d of %d trajectory-steps finished at %.1fs" % (done, total, time.perf_counter() - t0),
                  file=sys.stderr, flush=True)
        time.sleep(0.01)
    makespan = time.perf_counter() - t0
    srv.close()
    for m in built:
        m.close()
    reps.sort()
    lat = np.array([r["latency_s"] for _, r in reps])
    steps = sum(r["n_traj"] * r["n_steps"] for _, r in reps)
    span = max(reqs[-1]["t"], 1e-9)
    flop = sum(8.0 * r["stats"]["cmac_mfma"] for _, r in reps)
    return {
        "metric": "p50/p99 latency of the serving stream (first %d requests)" % K,
        "value": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "unit": "s",
        "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "dtype": "c64-mfma+f64" if prec else "f64",
        "requests": K, "reserved_shape": {"L": Lr, "chi_max": chir} if reserve else None,
        "offered_rate_per_s": K / span, "makespan_s": makespan,
        "offered_traj_steps_per_s": steps / span, "achieved_traj_steps_per_s": steps / makespan,
        "mean_queue_s": float(np.mean([r["queue_s"] for _, r in reps])),
        "mean_run_s": float(np.mean([r["run_s"] for _, r in reps])),
        "per_request": {"latency_s": [round(r["latency_s"], 3) for _, r in reps],
                        "queue_s": [round(r["queue_s"], 3) for _, r in reps],
                        "run_s": [round(r["run_s"], 3) for _, r in reps]},
        "traj_steps_per_s": steps / makespan, "achieved_tflops": flop / makespan / 1e12,
        "config": {"workload": "serving stream: Poisson arrivals (mean 0.05 s), XXX chains L~U{20..200}, "
                               "chi_max in {16,32,64}, gamma~U[0.01,0.2], g~U[0,1], N~U{64..512}, "
                               "T~U[1,5], Neel; numpy default_rng(5); %s" % precision,
                   "requests": [{k: q[k] for k in ("L", "chi_max", "n_traj", "n_steps")} for q in reqs]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps before the timed ones")
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--n-traj", type=int, default=None)
    ap.add_argument("--workers", type=int, default=0)
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=8.0, help="seconds of sampled oracle updates per process")
    ap.add_argument("--budget", type=float, default=520.0,
                    help="seconds after which the FP64 comparison is cut short (reported as partial)")
    ap.add_argument("--fp64-traj", type=int, default=512, help="trajectory ids of the FP64 comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy kernel used to calibrate the traffic counters")
    ap.add_argument("--no-reserve", action="store_true",
                    help="serving: no pool shape reserved for the stream's largest request")
    ap.add_argument("--serving", type=int, default=0, metavar="K",
                    help="instead: latency of the first K requests of the serving stream")
    ap.add_argument("--tune", action="store_true",
                    help="autotune tile_mode and workers for the workload first (tjm_autotune) and time with them")
    ap.add_argument("--tune-warm", type=int, default=3, help="untimed steps of each autotuner trial")
    ap.add_argument("--tune-steps", type=int, default=2, help="timed steps of each autotuner trial")
    ap.add_argument("--tune-cache", default=os.path.join(os.path.expanduser("~"), ".cache", "paper_2501_17913_amd",
                                                          "autotune.txt"),
                    help="autotuner cache file ('' for none)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from paper_2501_17913_amd import models, tjm

    if args.copy_calibration:
        print(json.dumps(copy_calibration(tjm)), flush=True)
        return

    if args.serving > 0:
        print(json.dumps(serving(tjm, models, args.serving, args.precision, not args.no_reserve)), flush=True)
        return

    w = dict(WORKLOADS[args.workload])
    if args.n_traj:
        w["n_traj"] = args.n_traj
    L, chi, N, T, init = w["L"], w["chi_max"], w["n_traj"], w["T"], w["init"]
    n = int(round(T / 0.1))
    K, W = args.steps, args.warmup
    if W + K > n or K < 1:
        print("warmup + steps must be within the %d steps of the job" % n, file=sys.stderr)
        sys.exit(2)
    prec = tjm.PREC_MIXED if args.precision == "mixed" else tjm.PREC_FP64
    t_start = time.perf_counter()
    nf = min(N, args.fp64_traj)
    compare_ids = nf if prec == tjm.PREC_MIXED and not args.no_fp64_compare else 0
    workers, tile_mode, tune = args.workers, 0, None
    if args.tune:
        tile_mode, workers, tune = autotune(tjm, models, L, init, chi, N, T, prec, args.tune_warm, args.tune_steps,
                                            args.tune_cache or None)
    head = measure(tjm, models, L, init, chi, N, T, prec, W, K, workers, read_ids=compare_ids, tile_mode=tile_mode)
    peak = PEAK_TFLOPS[args.precision]
    out = {
        "metric": "trajectory-steps/s at L=%d chi=%d (mixed vs FP64 path)" % (L, chi),
        "value": head["value"],
        "unit": "trajectory-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1e3 * head["wall"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64-mfma+f64" if prec == tjm.PREC_MIXED else "f64",
        "data": "synthetic",
        "config": {"workload": "XXX chain L=%d J=1 g=0.5 (X field), sigma- and Z jumps gamma=0.1 on every "
                               "site, %s initial state, chi_max=%d, dt=0.1, T=%g, %d trajectories, %s; "
                               "timed steps %d..%d of the %d-step job"
                               % (L, "Neel" if init == "neel" else "|0...0>", chi, T, N, args.precision, W + 1,
                                  W + K, n),
                   "L": L, "chi_max": chi, "n_traj": N, "dt": 0.1, "T": T, "init": init,
                   "precision": args.precision},
        "roofline": {"bound": "mfma", "achieved": head["achieved_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": head["achieved_tflops"] / peak,
                     "traffic": traffic_per_launch(args.workload, args.precision, W, K),
                     "kernel": "tjm_step_kernel<%s>" % ("float" if prec == tjm.PREC_MIXED else "double"),
                     "avg_launch_ms": head["avg_ms"], "algorithmic_flop_per_launch": head["flops_per_launch"]},
        "workers": head["workers"],
        "tile_mode": tile_mode,
        "counts": head["counts"],
        "phase_frac": head["phase_frac"],
    }
    if tune is not None:
        out["autotune"] = tune
    if compare_ids:
        # leave room for the CPU baseline after it
        deadline = t_start + args.budget - (0 if args.no_cpu_baseline else args.cpu_budget + 60.0)
        f = measure(tjm, models, L, init, chi, nf, T, tjm.PREC_FP64, W, K, workers, read_ids=nf, deadline=deadline,
                    tile_mode=tile_mode)
        if f["partial"]:
            out["fp64_path"] = {"value": None, "n_traj": nf, "partial": True, "steps_done": f["steps_done"],
                                "reason": "stopped at the bench time budget (--budget %g s)" % args.budget}
        else:
            out["fp64_path"] = {"value": f["value"], "n_traj": nf, "ms_per_step": 1e3 * f["wall"] / K,
                                "achieved_tflops": f["achieved_tflops"], "peak": PEAK_TFLOPS["fp64"],
                                "frac": f["achieved_tflops"] / PEAK_TFLOPS["fp64"],
                                "per_trajectory_speedup_of_mixed": (head["value"] / N) / (f["value"] / nf),
                                "phase_frac": f["phase_frac"]}
            out["error_vs_fp64"] = compare(head["records"], f["records"])
            out["error_vs_fp64"]["ids"] = "0..%d" % (nf - 1)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, chi, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
