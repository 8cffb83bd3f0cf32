"""The serving front end (tjm_server_create / tjm_submit / tjm_poll /
tjm_wait) through the C ABI: jobs of different models, sizes and precisions
run concurrently on one GPU and return exactly what tjm_run returns for the
same arguments; a small FP64 job also matches the CPU oracle trajectory by
trajectory.  Admission: a budget that holds one job at a time still runs
every job, in submission order; a job above the budget is refused."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2501_17913_amd import models, tjm  # noqa: E402
from oracle import model as om, mps_tjm  # noqa: E402
from tests import inputs  # noqa: E402


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _model(L, g, gamma, init="neel"):
    mpo, s, o, r = models.xxx_model(L, 1.0, g, gamma)
    m = tjm.Model(L, mpo, s, o, r)
    m.set_initial_product(models.product_state(inputs.init_bits(L, init)))
    return m


JOBS = [  # (L, chi_max, n_traj, steps, g, gamma, precision, seed)
    (6, 8, 40, 6, 0.5, 0.1, tjm.PREC_FP64, inputs.SEED + 81),
    (12, 16, 300, 4, 0.3, 0.05, tjm.PREC_MIXED, inputs.SEED + 82),
    (5, 4, 16, 8, 0.6, 0.1, tjm.PREC_FP64, inputs.SEED + 83),
    (20, 16, 700, 3, 0.8, 0.2, tjm.PREC_MIXED, inputs.SEED + 84),
    (8, 8, 64, 5, 0.5, 0.1, tjm.PREC_MIXED, inputs.SEED + 85),
]


def _submit_all(srv, jobs):
    ids = []
    for (L, chi, N, n, g, gamma, prec, seed) in jobs:
        m = _model(L, g, gamma)
        ids.append(srv.submit(m, N, 0.1, n * 0.1, chi, models.zx_observables(L), seed,
                              tjm.default_options(precision=prec)))
        m.close()            # the server holds its own copy of the model
    return ids


def _direct(job):
    (L, chi, N, n, g, gamma, prec, seed) = job
    m = _model(L, g, gamma)
    out = m.run(N, 0.1, n * 0.1, chi, models.zx_observables(L), seed, tjm.default_options(precision=prec))
    m.close()
    return out


def test_server_jobs_equal_direct_runs():
    log("server: %d concurrent jobs" % len(JOBS))
    srv = tjm.Server(0)
    ids = _submit_all(srv, JOBS)
    res = {}
    for i in reversed(range(len(ids))):        # collected out of order
        res[i] = srv.wait(ids[i])
        with pytest.raises(tjm.TjmError) as e:   # released once collected
            srv.poll(ids[i])
        assert e.value.status == tjm.E_INVAL
    srv.close()
    for i, job in enumerate(JOBS):
        ref = _direct(job)
        r = res[i]
        log("job", i, job[:4], "latency %.3f s" % r["report"]["latency_s"])
        assert r["mean"].shape == ref["mean"].shape
        assert np.array_equal(r["mean"], ref["mean"]) and np.array_equal(r["sem"], ref["sem"])
        rep = r["report"]
        assert rep["n_traj"] == job[2] and rep["n_steps"] == job[3]
        assert 0.0 <= rep["queue_s"] <= rep["latency_s"] and rep["run_s"] > 0.0
        assert rep["stats"]["steps_done"] == job[3] and rep["stats"]["failed_traj"] == 0
        assert rep["device_bytes"] >= rep["stats"]["device_bytes"]


def test_server_small_fp64_job_matches_oracle():
    L, chi, N, n, g, gamma, _, seed = JOBS[2]
    srv = tjm.Server(0)
    job = srv.submit(_model(L, g, gamma), N, 0.1, n * 0.1, chi, models.zx_observables(L), seed,
                     tjm.default_options())
    out = srv.wait(job)
    srv.close()
    Ws = om.xxx_mpo(L, 1.0, g)
    jumps = om.relax_dephase_jumps(L, gamma, gamma)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, inputs.init_bits(L, "neel"))
    per = np.array([mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, n, obs, seed, t,
                                           mps_tjm.Options(chi_max=chi)) for t in range(N)])
    assert np.abs(out["mean"] - per.mean(axis=0)).max() < 1e-10
    sem = per.std(axis=0, ddof=1) / np.sqrt(N)
    assert np.abs(out["sem"] - sem).max() < 1e-10


def test_server_budget_admits_one_job_at_a_time():
    # one chain shape and precision, so that every job uses the same scratch
    # pool whatever the server reshapes (a smaller pool would leave room for
    # more buffers than the first pass measured)
    jobs = [(8, 8, 40, 6, 0.5, 0.1, tjm.PREC_FP64, inputs.SEED + 86),
            (8, 8, 120, 4, 0.3, 0.05, tjm.PREC_FP64, inputs.SEED + 87),
            (8, 8, 16, 8, 0.6, 0.1, tjm.PREC_FP64, inputs.SEED + 88)]
    sizes, pools = [], {}
    srv = tjm.Server(0)
    for job in jobs:       # learn each job's buffers and its precision's pool from a first pass
        rep = srv.wait(_submit_all(srv, [job])[0])["report"]
        sizes.append(rep["device_bytes"])
        pools[job[6]] = max(pools.get(job[6], 0), rep["pool_bytes"])
    srv.close()
    # the pools, plus never room for the buffers of two jobs at once
    budget = sum(pools.values()) + max(sizes) + min(sizes) // 2
    srv = tjm.Server(0, budget)
    ids = _submit_all(srv, jobs)
    reps = [srv.wait(j) for j in ids]
    srv.close()
    for job, r in zip(jobs, reps):
        assert np.array_equal(r["mean"], _direct(job)["mean"])
    t = [(r["report"]["start_s"], r["report"]["end_s"]) for r in reps]
    # first come, first served and no overlap: each starts after the previous ended
    for a, b in zip(t, t[1:]):
        assert b[0] >= a[1]
    # a job above the whole budget is refused at submission
    srv = tjm.Server(0, min(sizes) // 4)
    with pytest.raises(tjm.TjmError) as e:
        _submit_all(srv, [jobs[0]])
    assert e.value.status == tjm.E_NOMEM
    srv.close()


def test_server_rejects_bad_jobs_and_reports_failures():
    srv = tjm.Server(0)
    m = _model(6, 0.5, 0.1)
    with pytest.raises(tjm.TjmError) as e:
        srv.submit(m, 4, 0.1, 0.25, 8, models.zx_observables(6), 1)      # T/dt not an integer
    assert e.value.status == tjm.E_INVAL
    with pytest.raises(tjm.TjmError) as e:
        srv.submit(m, 4, 0.1, 0.2, 8, models.zx_observables(6), 1, tjm.default_options(chi_cap=128))
    assert e.value.status == tjm.E_UNSUPPORTED
    with pytest.raises(tjm.TjmError) as e:     # more trajectories than the work ring holds
        srv.submit(m, (1 << 20) + 1, 0.1, 0.2, 8, models.zx_observables(6), 1)
    assert e.value.status == tjm.E_UNSUPPORTED
    with pytest.raises(tjm.TjmError) as e:
        srv.wait(12345)
    assert e.value.status == tjm.E_INVAL
    job = srv.submit(m, 4, 0.1, 0.2, 8, models.zx_observables(6), 1)
    while not srv.poll(job):
        pass
    assert srv.wait(job)["report"]["n_steps"] == 2
    # jobs still queued or uncollected at shutdown are released with the server
    for _ in range(3):
        srv.submit(m, 64, 0.1, 0.3, 8, models.zx_observables(6), 2)
    srv.close()
    m.close()


def test_server_admits_trajectories_of_new_jobs_while_others_run():
    # continuous batching: a long job runs in the resident kernel (fewer
    # trajectories than its workgroups, many steps each); jobs of other chain
    # lengths and bond dimensions that arrive while it runs take the idle
    # workgroups of the same kernel and finish long before it; each equals
    # its own direct run
    long_job = (24, 32, 300, 24, 0.5, 0.1, tjm.PREC_MIXED, inputs.SEED + 91)
    short_jobs = [(7, 8, 48, 4, 0.4, 0.1, tjm.PREC_MIXED, inputs.SEED + 92),
                  (16, 16, 96, 3, 0.6, 0.05, tjm.PREC_MIXED, inputs.SEED + 93)]
    srv = tjm.Server(0)
    first = _submit_all(srv, [long_job])[0]
    import time
    time.sleep(0.2)
    later = _submit_all(srv, short_jobs)
    # per-job progress: trajectories and step functions finished so far,
    # never decreasing, all of them once the job is done
    seen = []
    while not srv.poll(first):
        seen.append(srv.progress(first))
        time.sleep(0.05)
    n_steps = long_job[3]
    assert all(0 <= a[0] <= b[0] <= long_job[2] and 0 <= a[1] <= b[1] <= long_job[2] * n_steps
               and a[0] * n_steps <= a[1] for a, b in zip(seen, seen[1:]))
    assert any(0 < s[1] < long_job[2] * n_steps for s in seen)
    assert srv.progress(first) == (long_job[2], long_job[2] * n_steps)
    reps = [srv.wait(j) for j in later]
    lrep = srv.wait(first)
    with pytest.raises(tjm.TjmError):
        srv.progress(first)                # collected
    srv.close()
    for job, r in zip(short_jobs, reps):
        log("short job", job[:4], "start %.3f end %.3f (long job ends %.3f)"
            % (r["report"]["start_s"], r["report"]["end_s"], lrep["report"]["end_s"]))
        assert r["report"]["start_s"] < lrep["report"]["end_s"]
        # and is finished and released while the long job still runs (its
        # release does not wait for the resident kernel)
        assert r["report"]["end_s"] < lrep["report"]["end_s"]
        assert np.array_equal(r["mean"], _direct(job)["mean"])
    assert np.array_equal(lrep["mean"], _direct(long_job)["mean"])


def test_server_reserve_shapes_the_first_pool():
    # a larger job arriving while a smaller one runs would wait for the
    # smaller one's queue to drain; with the larger shape reserved, the first
    # pool already serves it and it starts at once, in the same kernel
    first = (24, 32, 1500, 6, 0.5, 0.1, tjm.PREC_MIXED, inputs.SEED + 94)
    larger = (40, 32, 32, 2, 0.6, 0.05, tjm.PREC_MIXED, inputs.SEED + 95)
    opt = tjm.default_options(precision=tjm.PREC_MIXED)
    srv = tjm.Server(0)
    hint = _model(40, 0.6, 0.05)
    with pytest.raises(tjm.TjmError) as e:      # validated as a submission is
        srv.reserve(hint, 32, 0.1, 0.25, 32, models.zx_observables(40), opt)
    assert e.value.status == tjm.E_INVAL
    srv.reserve(hint, 32, 0.1, 0.2, 32, models.zx_observables(40), opt)
    hint.close()
    a = _submit_all(srv, [first])[0]
    import time
    time.sleep(0.2)
    b = _submit_all(srv, [larger])[0]
    rb = srv.wait(b)
    ra = srv.wait(a)
    srv.close()
    log("reserved: first start %.3f end %.3f, larger start %.3f end %.3f" % (
        ra["report"]["start_s"], ra["report"]["end_s"], rb["report"]["start_s"], rb["report"]["end_s"]))
    assert rb["report"]["pool_bytes"] == ra["report"]["pool_bytes"]
    assert rb["report"]["start_s"] < ra["report"]["end_s"]
    assert rb["report"]["queue_s"] < 1.0
    assert np.array_equal(rb["mean"], _direct(larger)["mean"])
    # a reserved shape beyond the whole budget is refused
    srv = tjm.Server(0, 1 << 20)
    m = _model(40, 0.6, 0.05)
    with pytest.raises(tjm.TjmError) as e:
        srv.reserve(m, 32, 0.1, 0.2, 32, models.zx_observables(40), opt)
    assert e.value.status == tjm.E_NOMEM
    m.close()
    srv.close()
