"""The TJM schedule on dense state vectors (oracle O2) and the textbook
first-order MCWF (oracle O2').

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

O2 runs exactly the schedule of Eq. (TimeEvolutionFunctions) / Sec.
"Algorithm" with the same draws as the MPS oracle, but with U[dt] =
expm(-i H0 dt) exact, D[tau] the Kronecker product of the local dissipators
(Eq. DissipativeMPO) and no truncation.  Where TDVP is exact (H0 = 0, or
chains of one or two sites) it must agree with the MPS oracle trajectory by
trajectory.

O2' is the MCWF of Sec. "Monte Carlo wave function method": the first-order
jump probability delta p_m = dt gamma_m <L_m^dag L_m> evaluated on the state
at time t, jumps applied to the pre-evolved state.  It is only a statistical
cross-check against the exact Lindblad solution.
"""
import numpy as np
import scipy.linalg as sla

from . import model, philox


def _kron_all(mats):
    out = np.array([[1.0 + 0j]])
    for m in mats:
        out = np.kron(out, m)
    return out


def _jump(psi, full_jumps, eps, r):
    """J_eps on a dense vector (Sec. "Stochastic jump process", R6, R8)."""
    norm2 = np.real(np.vdot(psi, psi))
    dp = max(0.0, 1.0 - norm2)
    if eps >= dp:
        return psi / np.sqrt(norm2), -1
    w = np.array([g * np.real(np.vdot(Lm @ psi, Lm @ psi)) for (Lm, g) in full_jumps])
    cum = np.cumsum(w)
    W = cum[-1] if len(cum) else 0.0
    if not W > 1e-300:
        return psi / np.sqrt(norm2), -1
    m = int(np.argmax(cum > r * W)) if np.any(cum > r * W) else int(np.nonzero(w)[0][-1])
    psi = full_jumps[m][0] @ psi
    return psi / np.linalg.norm(psi), m


def run_trajectory(H, jumps, psi0, dt, n_steps, observables, seed, traj, record=None, dense_observables=(),
                   order=2):
    """Dense-vector TJM: the schedule of the MPS oracle with exact
    propagators.  order = 2 is Eq. (TimeEvolutionFunctions); order = 1 the
    first-order splitting of Sec. "Higher-order Trotterization" (F_k =
    J D[dt] U[dt], no F_0, measured after each step)."""
    L = int(round(np.log2(H.shape[0])))
    U = sla.expm(-1j * H * dt)
    Dh = _kron_all([model.local_dissipator(jumps, s, 0.5 * dt) for s in range(L)])
    Df = _kron_all([model.local_dissipator(jumps, s, dt) for s in range(L)])
    full = [(model.site_op_dense(op, s, L), g) for (s, op, g) in jumps]
    obs = [model.site_op_dense(op, s, L) for (s, op) in observables] + list(dense_observables)

    def measure(p):
        return [np.real(np.vdot(p, O @ p)) for O in obs]

    phi = psi0 / np.linalg.norm(psi0)
    out = np.zeros((n_steps + 1, len(obs)))
    out[0] = measure(phi)
    jlog = []
    if order == 1:
        for k in range(1, n_steps + 1):
            eps, r = philox.draws(seed, traj, k, philox.BRANCH_MAIN)
            phi, m = _jump(Df @ (U @ phi), full, eps, r)
            jlog.append((k, philox.BRANCH_MAIN, m))
            out[k] = measure(phi)
        if record is not None:
            record['jumps'] = jlog
        return out
    eps, r = philox.draws(seed, traj, 0, philox.BRANCH_MAIN)
    phi, m = _jump(Dh @ phi, full, eps, r)
    jlog.append((0, philox.BRANCH_MAIN, m))
    for k in range(1, n_steps + 1):
        x = U @ phi
        eps, r = philox.draws(seed, traj, k, philox.BRANCH_SAMPLE)
        y, m = _jump(Dh @ x, full, eps, r)
        jlog.append((k, philox.BRANCH_SAMPLE, m))
        out[k] = measure(y)
        if k < n_steps:
            eps, r = philox.draws(seed, traj, k, philox.BRANCH_MAIN)
            phi, m = _jump(Df @ x, full, eps, r)
            jlog.append((k, philox.BRANCH_MAIN, m))
    if record is not None:
        record['jumps'] = jlog
    return out


def run_mcwf_textbook(H, jumps, psi0, dt, n_steps, observables, rng):
    """First-order MCWF: dp_m = dt gamma_m <L_m^dag L_m>_psi(t); without a jump
    psi <- exp(-i H_eff dt) psi normalised, H_eff = H0 - i/2 sum gamma L^dag L
    (Eqs. EffectiveHamiltonian, NonHermitianHamiltonian); with a jump
    psi <- L_m psi(t) normalised (the pre-evolved state)."""
    L = int(round(np.log2(H.shape[0])))
    full = [(model.site_op_dense(op, s, L), g) for (s, op, g) in jumps]
    Heff = H.astype(np.complex128).copy()
    for Lm, g in full:
        Heff -= 0.5j * g * Lm.conj().T @ Lm
    Ueff = sla.expm(-1j * Heff * dt)
    obs = [model.site_op_dense(op, s, L) for (s, op) in observables]
    psi = psi0 / np.linalg.norm(psi0)
    out = np.zeros((n_steps + 1, len(obs)))
    out[0] = [np.real(np.vdot(psi, O @ psi)) for O in obs]
    for k in range(1, n_steps + 1):
        dpm = np.array([dt * g * np.real(np.vdot(Lm @ psi, Lm @ psi)) for (Lm, g) in full])
        dp = dpm.sum()
        if rng.random() >= dp:
            psi = Ueff @ psi
            psi = psi / np.linalg.norm(psi)
        else:
            m = int(np.searchsorted(np.cumsum(dpm), rng.random() * dp, side='right'))
            m = min(m, len(full) - 1)
            psi = full[m][0] @ psi
            psi = psi / np.linalg.norm(psi)
        out[k] = [np.real(np.vdot(psi, O @ psi)) for O in obs]
    return out
