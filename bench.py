"""Throughput of the TJM step on one MI355X.

One *step* is one step function F_k of the sampling MPS applied to every
trajectory of the batch (dynamic TDVP, both dissipation/jump branches,
observables): one launch of the persistent TJM kernel.  The workload is the
XXX chain L=100, chi_max=64, 4096 trajectories, dt=0.1, T=5 (50 steps),
Neel initial state, relaxation + dephasing at gamma=0.1 on every site,
mixed precision (complex-FP32 matrix-core contractions, FP64 factorisations).

Timed region: the K steps that follow W untimed warmup steps of the same run
(F_0 and uploads happen before; inputs are resident in HBM).  value =
trajectories x K / wall seconds.  The FP64 path is timed on the same steps
for trajectory ids 0..511 (fp64_path).

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
    "C2": dict(L=40, chi_max=32, n_traj=1024, T=5.0),
    "C3": dict(L=100, chi_max=64, n_traj=4096, T=5.0),
    "C4": dict(L=1000, chi_max=16, n_traj=512, T=2.0),
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


def _oracle_worker(args):
    L, chi, steps, traj = args
    from oracle import model as om, mps_tjm
    Ws = om.xxx_mpo(L, 1.0, 0.5)
    jumps = om.relax_dephase_jumps(L, 0.1, 0.1)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, [l % 2 for l in range(L)])
    t0 = time.time()
    mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, steps, obs, SEED, traj,
                           mps_tjm.Options(chi_max=chi))
    return steps, time.time() - t0


def cpu_baseline(L, chi, steps=5):
    """The oracle as it stands on the host cores, one trajectory per process
    (trajectory ids 0..cores-1), each run for the first `steps` steps of the
    job; rate = sum over processes of steps / seconds."""
    cores = max(1, min(os.cpu_count() or 1, 16))
    for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[v] = "1"                     # one core per trajectory, as in the paper's runs
    res = []
    with mp.get_context("spawn").Pool(cores) as pool:
        for r in pool.imap_unordered(_oracle_worker, [(L, chi, steps, t) for t in range(cores)]):
            res.append(r)
            print("  cpu baseline: %d of %d trajectories done" % (len(res), cores), file=sys.stderr, flush=True)
    rate = sum(n / el for n, el in res)
    return {"value": rate, "unit": "trajectory-steps/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 NumPy MPS-TJM of the same chain and seed, trajectory ids 0..%d (one per core), "
                      "steps 1..%d from the Neel state, each run from F_0" % (cores - 1, steps)}


def copy_calibration(tjm, n_bytes=1 << 30, reps=5):
    ms = tjm.selftest_copy(n_bytes, reps)
    return {"copy_bytes": n_bytes, "reps": reps, "avg_ms": ms, "GB/s": 2 * n_bytes / (ms * 1e-3) / 1e9}


def measure(tjm, models, L, chi, N, T, prec, warmup, K, workers):
    """Run one job on the GPU; time steps warmup+1 .. warmup+K."""
    dt = 0.1
    n = int(round(T / dt))
    mpo, s, o, r = models.xxx_model(L, 1.0, 0.5, 0.1)
    m = tjm.Model(L, mpo, s, o, r)
    m.set_initial_product(models.neel(L))
    opt = tjm.default_options(precision=prec, workers=workers)
    m.begin(N, dt, T, chi, models.zx_observables(L), SEED, opt)
    for k in range(warmup):
        m.advance(1)
        print("  warmup step %d of %d done" % (k + 1, warmup), file=sys.stderr, flush=True)
    s0 = m.stats()
    t0 = time.perf_counter()
    for k in range(K):                # each advance returns after its launch has finished
        m.advance(1)
        print("  %s step %d of %d done at %.1fs" % ("mixed" if prec == tjm.PREC_MIXED else "fp64", warmup + k + 1,
                                                    warmup + K, time.perf_counter() - t0), file=sys.stderr, flush=True)
    wall = time.perf_counter() - t0
    s1 = m.stats()
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
        "value": N * K / wall, "wall": wall, "avg_ms": avg_ms, "flops_per_launch": flops_per_launch,
        "achieved_tflops": flops_per_launch / (avg_ms * 1e-3) / 1e12, "workers": s1["workers"],
        "counts": {k: s1[k] - s0[k] for k in ("krylov_iters", "expm_calls", "one_site", "two_site",
                                              "factorizations", "jumps", "cmac_mix")},
        "phase_frac": {k: round(v / tot, 4) for k, v in phases.items() if k != "total"},
    }


def serving(tjm, models, K, precision):
    """The first K requests of the serving stream, submitted at their arrival
    times to one tjm_server; latency = submission to completion."""
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
    while pending:                        # progress as jobs finish, in any order
        for i in sorted(pending):
            if srv.poll(ids[i]):
                reps.append((i, srv.wait(ids[i])["report"]))
                pending.discard(i)
                print("  request %d done (%d of %d) at %.1fs" % (i, len(reps), len(ids), time.perf_counter() - t0),
                      file=sys.stderr, flush=True)
        time.sleep(0.01)
    makespan = time.perf_counter() - t0
    srv.close()
    for m in built:
        m.close()
    reps.sort()
    lat = np.array([r["latency_s"] for _, r in reps])
    steps = sum(r["n_traj"] * r["n_steps"] for _, r in reps)
    flop = sum(8.0 * r["stats"]["cmac_mfma"] for _, r in reps)
    return {
        "metric": "p50/p99 latency of the serving stream (first %d requests)" % K,
        "value": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)), "unit": "s",
        "higher_is_better": False, "n_gpus": 1, "data": "synthetic", "dtype": "c64-mfma+f64" if prec else "f64",
        "requests": K, "offered_rate_per_s": K / reqs[-1]["t"], "makespan_s": makespan,
        "mean_queue_s": float(np.mean([r["queue_s"] for _, r in reps])),
        "mean_run_s": float(np.mean([r["run_s"] for _, r in reps])),
        "traj_steps_per_s": steps / makespan, "achieved_tflops": flop / makespan / 1e12,
        "config": {"workload": "serving stream: Poisson arrivals (mean 0.05 s), XXX chains L~U{20..200}, "
                               "chi_max in {16,32,64}, gamma~U[0.01,0.2], g~U[0,1], N~U{64..512}, "
                               "T~U[1,5], Neel; numpy default_rng(5); %s" % precision,
                   "requests": [{k: q[k] for k in ("L", "chi_max", "n_traj", "n_steps")} for q in reqs]},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=6, help="timed steps")
    ap.add_argument("--warmup", type=int, default=0, help="untimed steps before the timed ones")
    ap.add_argument("--workload", default="C3", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--n-traj", type=int, default=None)
    ap.add_argument("--workers", type=int, default=0)
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=5, help="steps per trajectory of the CPU oracle sample")
    ap.add_argument("--fp64-traj", type=int, default=512, help="trajectory ids of the FP64 comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run the plain copy kernel used to calibrate the traffic counters")
    ap.add_argument("--serving", type=int, default=0, metavar="K",
                    help="instead: latency of the first K requests of the serving stream")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    from paper_2501_17913_amd import models, tjm

    if args.copy_calibration:
        print(json.dumps(copy_calibration(tjm)), flush=True)
        return

    if args.serving > 0:
        print(json.dumps(serving(tjm, models, args.serving, args.precision)), flush=True)
        return

    w = dict(WORKLOADS[args.workload])
    if args.n_traj:
        w["n_traj"] = args.n_traj
    L, chi, N, T = w["L"], w["chi_max"], w["n_traj"], w["T"]
    n = int(round(T / 0.1))
    K, W = args.steps, args.warmup
    if W + K > n or K < 1:
        print("warmup + steps must be within the %d steps of the job" % n, file=sys.stderr)
        sys.exit(2)
    prec = tjm.PREC_MIXED if args.precision == "mixed" else tjm.PREC_FP64
    head = measure(tjm, models, L, chi, N, T, prec, W, K, args.workers)
    peak = PEAK_TFLOPS[args.precision]
    out = {
        "metric": "trajectory-steps/s at L=100 chi=64 (mixed vs FP64 path)",
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
                               "site, Neel initial state, chi_max=%d, dt=0.1, T=%g, %d trajectories, %s; "
                               "timed steps %d..%d of the %d-step job"
                               % (L, chi, T, N, args.precision, W + 1, W + K, n),
                   "L": L, "chi_max": chi, "n_traj": N, "dt": 0.1, "T": T, "precision": args.precision},
        "roofline": {"bound": "mfma", "achieved": head["achieved_tflops"], "peak": peak, "unit": "TFLOP/s",
                     "frac": head["achieved_tflops"] / peak,
                     "traffic": traffic_per_launch(args.workload, args.precision, W, K),
                     "kernel": "tjm_step_kernel<%s>" % ("float" if prec == tjm.PREC_MIXED else "double"),
                     "avg_launch_ms": head["avg_ms"], "algorithmic_flop_per_launch": head["flops_per_launch"]},
        "workers": head["workers"],
        "counts": head["counts"],
        "phase_frac": head["phase_frac"],
    }
    if prec == tjm.PREC_MIXED and not args.no_fp64_compare:
        nf = min(N, args.fp64_traj)
        f = measure(tjm, models, L, chi, nf, T, tjm.PREC_FP64, W, K, args.workers)
        out["fp64_path"] = {"value": f["value"], "n_traj": nf, "ms_per_step": 1e3 * f["wall"] / K,
                            "achieved_tflops": f["achieved_tflops"], "peak": PEAK_TFLOPS["fp64"],
                            "mixed_speedup": head["value"] / f["value"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(L, chi, min(args.cpu_steps, n))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
