"""The HIP TJM against the CPU oracle, through the C ABI.

Per trajectory (same Philox streams on both sides): identical jump logs and
bond dimensions, site observables within 1e-10 on the FP64 path; within
2e-4 on the mixed path for trajectories whose jump logs agree.  Ensembles:
the C1 workload against exact Lindblad dynamics.  Large launch shapes: the
full trajectory counts and chain lengths of the measured workloads, a few
steps, with sampled trajectories recomputed by the oracle one by one, plus
properties that hold at any size."""
import sys
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2501_17913_amd import models, tjm  # noqa: E402
from oracle import lindblad, model as om, mps_tjm  # noqa: E402
from tests import inputs  # noqa: E402
from tests.oracle_pool import oracle_trajectories  # noqa: E402


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_run(L, chi, init, n, N, g, gamma, seed, prec=tjm.PREC_FP64, J=1.0, traces=True, **kw):
    mpo, s, o, r = models.xxx_model(L, J, g, gamma)
    m = tjm.Model(L, mpo, s, o, r)
    m.set_initial_product(models.product_state(inputs.init_bits(L, init)))
    opt = tjm.default_options(precision=prec, record_bonds=1 if traces else 0, **kw)
    out = m.run(N, 0.1, n * 0.1, chi, models.zx_observables(L), seed, opt, traces=traces)
    m.close()
    return out


def oracle_traj(L, chi, init, n, g, gamma, seed, traj, J=1.0):
    Ws = om.xxx_mpo(L, J, g)
    jumps = om.relax_dephase_jumps(L, gamma, gamma)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, inputs.init_bits(L, init))
    rec = {}
    out = mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, n, obs, seed, traj,
                                 mps_tjm.Options(chi_max=chi), rec)
    return out, [m for (_, _, m) in rec['jumps']], np.array(rec['bonds'])


@pytest.mark.parametrize("case", inputs.small_cases(), ids=lambda c: "L%d_chi%d_%s" % (c[0], c[1], c[2]))
def test_fp64_per_trajectory_parity(case):
    L, chi, init, n, N, g, gamma = case
    seed = inputs.SEED + L
    log("fp64 parity", case)
    res = gpu_run(L, chi, init, n, N, g, gamma, seed)
    worst = 0.0
    for t in range(N):
        ref, jl, bl = oracle_traj(L, chi, init, n, g, gamma, seed, t)
        assert list(res['jumps'][t]) == jl, (t, list(res['jumps'][t]), jl)
        assert np.array_equal(res['bonds'][t], bl), t
        worst = max(worst, np.abs(res['per_traj'][t] - ref).max())
    log("  max |gpu - oracle| =", worst)
    assert worst < 1e-10
    # trajectory average and its standard error are those of the records
    per = res['per_traj']
    assert np.abs(res['mean'] - per.mean(0)).max() < 1e-13
    if N > 1:
        assert np.abs(res['sem'] - per.std(0, ddof=1) / np.sqrt(N)).max() < 1e-13


@pytest.mark.parametrize("case", [inputs.small_cases()[4], inputs.small_cases()[5]],
                         ids=lambda c: "L%d_chi%d" % (c[0], c[1]))
def test_fp64_certified_sweeps_parity(case):
    # Post-jump normalisation sweeps with QR moves where a bound proves the
    # SVD would discard nothing: the same states in another gauge, so the
    # same jumps and bonds; observables agree to the conditioning of 1TDVP
    # on bonds with Schmidt values near the discard threshold.
    L, chi, init, n, N, g, gamma = case
    seed = inputs.SEED + L
    res = gpu_run(L, chi, init, n, N, g, gamma, seed, certify_sweeps=1)
    worst = 0.0
    for t in range(N):
        ref, jl, bl = oracle_traj(L, chi, init, n, g, gamma, seed, t)
        assert list(res['jumps'][t]) == jl
        assert np.array_equal(res['bonds'][t], bl)
        worst = max(worst, np.abs(res['per_traj'][t] - ref).max())
    log("  certified sweeps: max |gpu - oracle| =", worst)
    assert worst < 1e-8


@pytest.mark.parametrize("prec", [tjm.PREC_FP64, tjm.PREC_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("case", [inputs.small_cases()[2], inputs.small_cases()[5]],
                         ids=lambda c: "L%d_chi%d" % (c[0], c[1]))
def test_generic_effective_hamiltonian_parity(case, prec):
    # the generic three-stage contraction L x W x M x R (any MPO), which the
    # nearest-neighbour XXX chain otherwise replaces by the structured products
    L, chi, init, n, N, g, gamma = case
    seed = inputs.SEED + L
    res = gpu_run(L, chi, init, n, N, g, gamma, seed, prec=prec, generic_heff=1)
    worst, flips = 0.0, 0
    for t in range(N):
        ref, jl, bl = oracle_traj(L, chi, init, n, g, gamma, seed, t)
        if prec == tjm.PREC_FP64:
            assert list(res['jumps'][t]) == jl
            assert np.array_equal(res['bonds'][t], bl)
        if list(res['jumps'][t]) != jl:
            flips += 1
            continue
        worst = max(worst, np.abs(res['per_traj'][t] - ref).max())
    log("  generic contraction: max |gpu - oracle| =", worst, "flipped", flips)
    assert flips <= max(1, N // 8)
    assert worst < (1e-10 if prec == tjm.PREC_FP64 else 2e-4)


@pytest.mark.parametrize("case", [inputs.small_cases()[3], inputs.small_cases()[5]],
                         ids=lambda c: "L%d_chi%d" % (c[0], c[1]))
def test_mixed_precision_per_trajectory_parity(case):
    L, chi, init, n, N, g, gamma = case
    seed = inputs.SEED + L
    log("mixed parity", case)
    res = gpu_run(L, chi, init, n, N, g, gamma, seed, prec=tjm.PREC_MIXED)
    worst, flips = 0.0, 0
    for t in range(N):
        ref, jl, bl = oracle_traj(L, chi, init, n, g, gamma, seed, t)
        if list(res['jumps'][t]) != jl:
            flips += 1
            continue
        worst = max(worst, np.abs(res['per_traj'][t] - ref).max())
    log("  max |mixed - oracle| =", worst, "flipped trajectories", flips)
    assert flips <= max(1, N // 8)
    assert worst < 2e-4


def test_c1_ensemble_matches_exact_lindblad_and_oracle():
    w = inputs.workload("C1")
    L, n = w["L"], int(round(w["T"] / w["dt"]))
    log("C1 ensemble", w)
    res = gpu_run(L, w["chi_max"], w["init"], n, w["n_traj"], w["g"], w["gamma"], w["seed"])
    H = om.xxx_dense(L, w["J"], w["g"])
    jumps = om.relax_dephase_jumps(L, w["gamma"], w["gamma"])
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    psi0 = om.product_dense(om.product_site_vectors(L, inputs.init_bits(L, w["init"])))
    t0 = time.time()
    exact = lindblad.evolve_observables(H, jumps, psi0, w["dt"], n, obs)
    log("  exact Lindblad (4096-entry density matrix) in %.1fs" % (time.time() - t0))
    dev = np.abs(res['mean'] - exact)
    se = res['sem']
    assert np.mean(dev <= 3 * se + 2e-3) >= 0.99
    assert np.all(dev <= 5 * se + 2e-3)
    for t in (0, 57, 199):
        ref, jl, _ = oracle_traj(L, w["chi_max"], w["init"], n, w["g"], w["gamma"], w["seed"], t)
        assert list(res['jumps'][t]) == jl
        assert np.abs(res['per_traj'][t] - ref).max() < 1e-10


def _large(name, steps, prec, sample):
    w = inputs.workload(name)
    L = w["L"]
    log("large launch", name, "steps", steps, "precision", prec, "sampled", sample)
    t0 = time.time()
    res = gpu_run(L, w["chi_max"], w["init"], steps, w["n_traj"], w["g"], w["gamma"], w["seed"], prec=prec)
    log("  gpu %.1fs" % (time.time() - t0), {k: res['stats'][k] for k in ('jumps', 'krylov_iters', 'two_site', 'one_site')})
    per = res['per_traj']
    # properties that hold at any size
    assert np.all(np.isfinite(per)) and np.all(np.abs(per) <= 1 + 1e-9)
    assert np.all(res['bonds'] <= w["chi_max"]) and np.all(res['bonds'][:, :, 0] == 1)
    assert np.all(res['bonds'][:, :, -1] == 1)
    assert np.all((res['jumps'] >= -1) & (res['jumps'] < 2 * L))
    tol = 1e-10 if prec == tjm.PREC_FP64 else 2e-4
    t1 = time.time()
    ref = oracle_trajectories(L, w["chi_max"], w["init"], steps, w["g"], w["gamma"], w["seed"], sample)
    log("  oracle: %d sampled trajectories in %.1fs" % (len(sample), time.time() - t1))
    flips, worst = 0, 0.0
    for t in sample:
        out, jl, bl = ref[t]
        if prec == tjm.PREC_FP64:
            assert list(res['jumps'][t]) == jl
            assert np.array_equal(res['bonds'][t], bl)
        if list(res['jumps'][t]) != jl:
            flips += 1                    # mixed path: a decision within the FP32 error of its threshold
            continue
        worst = max(worst, float(np.abs(per[t] - out).max()))
    log("  sampled: max |gpu - oracle| = %.3e, %d of %d flipped" % (worst, flips, len(sample)))
    assert flips <= max(1, len(sample) // 8)
    assert worst < tol


def test_c2_launch_fp64_sampled_trajectories():
    _large("C2", 3, tjm.PREC_FP64, (0, 511, 1023))


def test_c3_launch_mixed_sampled_trajectories():
    _large("C3", 2, tjm.PREC_MIXED, (0, 1, 2, 3, 1024, 2047, 3000, 4095))


def test_fp64_general_initial_mps_parity():
    # Psi(0) a random MPS, unnormalised and in no particular gauge, with one
    # rank-deficient bond (b_3 > d b_2 is allowed and kept, as the oracle keeps it)
    L, chi, n, N, g, gamma = 6, 8, 6, 8, 0.5, 0.15
    seed = inputs.SEED + 61
    rng = np.random.default_rng(61)
    bonds = [1, 2, 2, 5, 4, 2, 1]
    psi0 = [rng.normal(size=(2, bonds[l], bonds[l + 1])) + 1j * rng.normal(size=(2, bonds[l], bonds[l + 1]))
            for l in range(L)]
    mpo, s_, o_, r_ = models.xxx_model(L, 1.0, g, gamma)
    m = tjm.Model(L, mpo, s_, o_, r_)
    m.set_initial_mps(psi0)
    opt = tjm.default_options(precision=tjm.PREC_FP64, record_bonds=1)
    res = m.run(N, 0.1, n * 0.1, chi, models.zx_observables(L), seed, opt, traces=True)
    m.close()
    Ws = om.xxx_mpo(L, 1.0, g)
    jumps = om.relax_dephase_jumps(L, gamma, gamma)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    worst = 0.0
    for t in range(N):
        rec = {}
        ref = mps_tjm.run_trajectory(Ws, jumps, psi0, 0.1, n, obs, seed, t, mps_tjm.Options(chi_max=chi), rec)
        assert list(res['jumps'][t]) == [j for (_, _, j) in rec['jumps']]
        assert np.array_equal(res['bonds'][t], np.array(rec['bonds']))
        worst = max(worst, np.abs(res['per_traj'][t] - ref).max())
    log("  general initial MPS: max |gpu - oracle| =", worst)
    assert worst < 1e-10


@pytest.mark.skip(reason="the transfer-environment jump path (sweep_jumps=0) faulted the device once "
                         "in the mixed L6 chi8 case and its cause was never found; the path has been removed "
                         "and sweep_jumps=0 is rejected with TJM_E_UNSUPPORTED")
@pytest.mark.parametrize("case", [inputs.small_cases()[4], inputs.small_cases()[6]],
                         ids=lambda c: "L%d_chi%d" % (c[0], c[1]))
def test_fp64_environment_jump_path_parity(case):
    # delta p, the jump weights and sampled observables from transfer-matrix
    # environments: the same decisions and bond dimensions as the sweeps
    L, chi, init, n, N, g, gamma = case
    seed = inputs.SEED + L
    res = gpu_run(L, chi, init, n, N, g, gamma, seed, sweep_jumps=0)
    for t in range(N):
        ref, jl, bl = oracle_traj(L, chi, init, n, g, gamma, seed, t)
        assert list(res['jumps'][t]) == jl
        assert np.array_equal(res['bonds'][t], bl)
        assert np.abs(res['per_traj'][t] - ref).max() < 1e-10


def test_graph_captured_steps_equal_direct_launches():
    # the same run with its step launches captured in HIP graphs (one graph
    # for the whole run, and one per call of a session advanced in uneven
    # pieces with host work between the replays) equals the step-by-step
    # launches bit for bit (FP64)
    L, chi, init, n, N, g, gamma = inputs.small_cases()[5]
    seed = inputs.SEED + 500
    ref = gpu_run(L, chi, init, n, N, g, gamma, seed)
    whole = gpu_run(L, chi, init, n, N, g, gamma, seed, graph=1)
    mpo, s_, o_, r_ = models.xxx_model(L, 1.0, g, gamma)
    m = tjm.Model(L, mpo, s_, o_, r_)
    m.set_initial_product(models.product_state(inputs.init_bits(L, init)))
    m.begin(N, 0.1, n * 0.1, chi, models.zx_observables(L), seed,
            tjm.default_options(precision=tjm.PREC_FP64, record_bonds=1, graph=1))
    done = 0
    for piece in (1, 3, 2, n):
        piece = min(piece, n - done)
        if piece <= 0:
            break
        m.advance(piece)
        done += piece
        mid = m.read()                   # host work between the replays
        assert np.array_equal(mid["jumps"][:, :2 * done], ref["jumps"][:, :2 * done])
    parts = m.end(traces=True)
    stats = m.stats()
    m.close()
    assert stats["step_launches"] == n
    for res in (whole, parts):
        assert np.array_equal(res["per_traj"], ref["per_traj"])
        assert np.array_equal(res["jumps"], ref["jumps"])
        assert np.array_equal(res["bonds"], ref["bonds"])
        assert np.array_equal(res["mean"], ref["mean"])


def test_degenerate_runs():
    """Edge cases of the method and the interface, each against the oracle:
    no jump operators at all, gamma = 0 (delta p = 0: never a jump), one
    step, one trajectory, no observables."""
    L, chi, g = 5, 4, 0.6
    Ws = om.xxx_mpo(L, 1.0, g)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, inputs.init_bits(L, "neel"))
    seed = inputs.SEED + 71
    # no jump operators: the paper's method reduces to TDVP with renormalisation
    m = tjm.Model(L, models.xxx_mpo(L, 1.0, g), [], [], [])
    m.set_initial_product(models.neel(L))
    res = m.run(3, 0.1, 0.4, chi, models.zx_observables(L), seed, tjm.default_options(record_bonds=1), traces=True)
    m.close()
    assert np.all(res['jumps'] == -1)
    for t in range(3):
        ref = mps_tjm.run_trajectory(Ws, [], mps_tjm.product_mps(sv), 0.1, 4, obs, seed, t, mps_tjm.Options(chi_max=chi))
        assert np.abs(res['per_traj'][t] - ref).max() < 1e-10
    # gamma = 0 with jump operators present: identical to the run without them
    mpo, s_, o_, r_ = models.xxx_model(L, 1.0, g, 0.0)
    m = tjm.Model(L, mpo, s_, o_, r_)
    m.set_initial_product(models.neel(L))
    res0 = m.run(3, 0.1, 0.4, chi, models.zx_observables(L), seed, tjm.default_options(record_bonds=1), traces=True)
    assert np.all(res0['jumps'] == -1)
    assert np.abs(res0['per_traj'] - res['per_traj']).max() < 1e-12
    # one step, one trajectory, and a run without observables
    res1 = m.run(1, 0.1, 0.1, chi, models.zx_observables(L), seed, tjm.default_options(), traces=True)
    assert res1['per_traj'].shape == (1, 2, 2 * L)
    assert np.abs(res1['per_traj'][0] - res0['per_traj'][0][:2]).max() < 1e-12
    out = m.run(2, 0.1, 0.2, chi, [], seed, tjm.default_options())
    assert out['mean'].shape == (3, 0)
    m.close()


def test_c4_launch_mixed_sampled_trajectory():
    # the long chain (L = 1000, chi 16): every trajectory, one step, one
    # trajectory recomputed by the oracle, properties of all of them
    _large("C4", 1, tjm.PREC_MIXED, (0,))
