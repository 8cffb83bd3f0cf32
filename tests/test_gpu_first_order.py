"""The first-order splitting of Sec. "Higher-order Trotterization"
(tjm_options.trotter_order = 1: no F_0, F_k = J D[dt] U[dt] measured on its
result) through the C ABI against the oracle's first-order schedule, per
trajectory with the same Philox streams, and a one-spin ensemble against
the exact average of that schedule."""
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


@pytest.mark.parametrize("prec", [tjm.PREC_FP64, tjm.PREC_MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("L,chi,init", [(6, 8, "zero"), (9, 8, "neel"), (12, 16, "neel")])
def test_first_order_per_trajectory(L, chi, init, prec):
    g, gamma, n, N = 0.5, 0.1, 8, 8
    seed = inputs.SEED + 700 + L
    mpo, s, o, r = models.xxx_model(L, 1.0, g, gamma)
    m = tjm.Model(L, mpo, s, o, r)
    m.set_initial_product(models.product_state(inputs.init_bits(L, init)))
    m.add_mpo_observable(mpo)                       # energy as well
    opt = tjm.default_options(precision=prec, record_bonds=1, trotter_order=1)
    res = m.run(N, 0.1, n * 0.1, chi, models.zx_observables(L), seed, opt, traces=True)
    m.close()
    Ws = om.xxx_mpo(L, 1.0, g)
    jumps = om.relax_dephase_jumps(L, gamma, gamma)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, inputs.init_bits(L, init))
    worst, flips, njump = 0.0, 0, 0
    for t in range(N):
        rec = {}
        ref = mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, n, obs, seed, t,
                                     mps_tjm.Options(chi_max=chi), rec, mpo_observables=[Ws], order=1)
        jl = np.full(2 * n, -1)
        for (k, _, x) in rec['jumps']:
            jl[2 * k - 1] = x
        njump += int(np.sum(jl >= 0))
        if prec == tjm.PREC_FP64:
            assert np.array_equal(res['jumps'][t], jl), (t, res['jumps'][t], jl)
            assert np.array_equal(res['bonds'][t], np.array(rec['bonds']))
        if not np.array_equal(res['jumps'][t], jl):
            flips += 1
            continue
        worst = max(worst, np.abs(res['per_traj'][t] - ref).max())
    log("  first order: max |gpu - oracle| =", worst, "flipped", flips, "jumps", njump)
    assert flips <= 1
    assert worst < (1e-10 if prec == tjm.PREC_FP64 else 2e-4)
    assert np.all(res['jumps'][:, 0] == -1) and np.all(res['jumps'][:, 2:-1:2] == -1)


def test_first_order_one_spin_ensemble():
    # sigma_minus damping with an X field on one spin: the trajectory average
    # of the first-order schedule, from the distribution of the last reset
    # to |0> (each jump resets), against the GPU ensemble
    import scipy.linalg as sla
    g, gam, dt, n, N = 1.0, 0.8, 0.1, 20, 20000
    psi0 = np.array([np.cos(0.3), np.sin(0.3)], dtype=complex)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Zm = np.diag([1.0, -1.0]).astype(complex)
    sm = np.array([[0, 1], [0, 0]], dtype=complex)
    U = sla.expm(1j * g * X * dt)
    D = sla.expm(-0.5 * dt * gam * sm.conj().T @ sm)
    zero = np.array([1.0, 0.0], dtype=complex)
    ez = lambda v: np.real(np.vdot(v, Zm @ v)) / np.real(np.vdot(v, v))
    dist, ref = [(1.0, psi0)], [ez(psi0)]
    for k in range(n):
        nd, reset = [], 0.0
        for (p, v) in dist:
            w = D @ (U @ v)
            p0 = np.real(np.vdot(w, w))
            nd.append((p * p0, w / np.sqrt(p0)))
            reset += p * (1 - p0)
        dist = nd + [(reset, zero)]
        ref.append(sum(p * ez(v) for p, v in dist))
    mpo = models.xxx_mpo(1, 1.0, g)
    m = tjm.Model(1, mpo, np.array([0], np.int32), np.array([models.LOWER]), np.array([gam]))
    m.set_initial_product(psi0.reshape(1, 2))
    res = m.run(N, dt, n * dt, 2, [(0, models.PAULI_Z)], inputs.SEED + 1, tjm.default_options(trotter_order=1))
    m.close()
    dev = np.abs(res['mean'][:, 0] - np.array(ref))
    log("  one spin first order: max dev", dev.max(), "max se", res['sem'].max())
    assert np.all(dev <= 4 * res['sem'][:, 0] + 1e-12)
