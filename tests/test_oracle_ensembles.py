"""P6: trajectory ensembles of the oracle against exact Lindblad dynamics.

The TJM mean converges to the solution of Eq. (Lindblad) as N grows
(Eq. MCWFConvergence, Sec. "Convergence"), up to the O(dt^2) global
splitting error of the second-order schedule (Sec. "Higher-order
Trotterization").  Criterion per (time, observable) entry: at least 99%
within 3 standard errors plus a 2e-3 time-step allowance, and all within 5
standard errors plus the allowance.
"""
import os

import numpy as np
import pytest

from oracle import dense_tjm, lindblad, model, mps_tjm

BIAS = 2e-3
SEED = 0x250117913


def _check(samples, exact):
    N = samples.shape[0]
    m = samples.mean(0)
    se = samples.std(0, ddof=1) / np.sqrt(N)
    dev = np.abs(m - exact)
    assert np.mean(dev <= 3 * se + BIAS) >= 0.99
    assert np.all(dev <= 5 * se + BIAS)


def _setup(L, bits, gam=0.1, J=1.0, g=0.5):
    H = model.xxx_dense(L, J, g)
    Ws = model.xxx_mpo(L, J, g)
    jumps = model.relax_dephase_jumps(L, gam, gam)
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    sv = model.product_site_vectors(L, bits)
    return H, Ws, jumps, obs, sv


@pytest.mark.parametrize("bits", [[0, 0, 0, 0], [0, 1, 0, 1]])
def test_dense_tjm_ensemble_matches_lindblad(bits):
    L, dt, n, N = 4, 0.1, 20, 600
    H, _, jumps, obs, sv = _setup(L, bits)
    exact = lindblad.evolve_observables(H, jumps, model.product_dense(sv), dt, n, obs)
    S = np.array([dense_tjm.run_trajectory(H, jumps, model.product_dense(sv), dt, n, obs, SEED, t)
                  for t in range(N)])
    _check(S, exact)


def test_mps_tjm_ensemble_matches_lindblad():
    L, dt, n, N = 4, 0.1, 15, 200
    H, Ws, jumps, obs, sv = _setup(L, model.neel_bits(L))
    exact = lindblad.evolve_observables(H, jumps, model.product_dense(sv), dt, n, obs)
    opt = mps_tjm.Options(chi_max=4)
    S = np.array([mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), dt, n, obs, SEED, t, opt)
                  for t in range(N)])
    _check(S, exact)


def test_dense_tjm_ensemble_relaxation_excitation_domain_wall():
    # the noise and initial state of the 30-site comparison, on a chain the
    # exact integrator reaches: sigma_-/sigma_+ at 0.1, XXX with J = h = 1
    # (Z field), domain wall.  Jumps here are rare events (about one per
    # site in 50 steps), so the ensemble is large enough to sample them.
    L, dt, n, N = 5, 0.1, 12, 1500
    H = model.xxx_dense(L, 1.0, 0.0, 1.0)
    jumps = model.relax_excite_jumps(L, 0.1, 0.1)
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    psi0 = model.product_dense(model.product_site_vectors(L, model.domain_wall_bits(L)))
    exact = lindblad.evolve_observables(H, jumps, psi0, dt, n, obs)
    S = np.array([dense_tjm.run_trajectory(H, jumps, psi0, dt, n, obs, SEED, t) for t in range(N)])
    _check(S, exact)


def test_textbook_mcwf_ensemble_matches_lindblad():
    # first-order MCWF (Sec. "Monte Carlo wave function method") at small dt
    L, dt, n, N = 3, 0.01, 100, 500
    H, _, jumps, obs, sv = _setup(L, [1, 0, 1], gam=0.2)
    exact = lindblad.evolve_observables(H, jumps, model.product_dense(sv), dt * 10, n // 10, obs)
    rng = np.random.default_rng(17)
    S = np.array([dense_tjm.run_mcwf_textbook(H, jumps, model.product_dense(sv), dt, n, obs, rng)[::10]
                  for _ in range(N)])
    m = S.mean(0)
    se = S.std(0, ddof=1) / np.sqrt(N)
    dev = np.abs(m - exact)
    # first order: allow a larger O(dt) bias
    assert np.mean(dev <= 3 * se + 5e-3) >= 0.99 and np.all(dev <= 5 * se + 5e-3)


def test_monte_carlo_error_shrinks_as_inverse_sqrt_n():
    # Sec. "Convergence": sigma ~ C / sqrt(N), independent of L.
    L, dt, n = 3, 0.1, 10
    H, _, jumps, obs, sv = _setup(L, [0, 1, 0], gam=0.2)
    exact = lindblad.evolve_observables(H, jumps, model.product_dense(sv), dt, n, obs)
    S = np.array([dense_tjm.run_trajectory(H, jumps, model.product_dense(sv), dt, n, obs, 3, t)
                  for t in range(1600)])
    errs = []
    for N in (25, 400):
        batches = S[: (1600 // N) * N].reshape(-1, N, *S.shape[1:]).mean(1)
        errs.append(np.sqrt(np.mean((batches[:, -1, :] - exact[-1]) ** 2)))
    # 16x more trajectories: error ratio ~4 (bias << sampling error here)
    assert 2.5 < errs[0] / errs[1] < 6.5


@pytest.mark.skipif(os.environ.get("TJM_SLOW") != "1", reason="set TJM_SLOW=1 (minutes)")
def test_c1_workload_mps_ensemble_matches_lindblad():
    # XXX L=6, J=1, g=0.5, sigma_- and Z at gamma=0.1, |0..0>, chi_max=8,
    # dt=0.1, T=2, 200 trajectories; 4096-entry density matrix for the exact side.
    L, dt, n, N = 6, 0.1, 20, 200
    H, Ws, jumps, obs, sv = _setup(L, model.zero_bits(L))
    exact = lindblad.evolve_observables(H, jumps, model.product_dense(sv), dt, n, obs)
    opt = mps_tjm.Options(chi_max=8)
    S = np.array([mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), dt, n, obs, SEED, t, opt)
                  for t in range(N)])
    _check(S, exact)
