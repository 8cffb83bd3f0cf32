"""Exact Lindblad integration for small chains (L <= 8).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Implements Eq. (Lindblad):
    d rho/dt = -i[H0, rho] + sum_m gamma_m (L_m rho L_m^dag - 1/2 {L_m^dag L_m, rho})
by vectorising rho row-major, vec(A rho B) = (A kron B^T) vec(rho), so the
generator is

    Lv = -i (H kron I - I kron H^T)
         + sum_m gamma_m (L kron conj(L) - 1/2 L^dag L kron I - 1/2 I kron (L^dag L)^T)

and rho(t + dt) = expm(Lv dt) rho(t) (dense for 4^L <= 4096, otherwise
scipy.sparse.linalg.expm_multiply).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import model


def _full_jump(op, site, L):
    return model.site_op_dense(op, site, L)


def liouvillian(H, full_jumps, sparse=False):
    """full_jumps: list of (dense L_m on the whole chain, gamma_m)."""
    dim = H.shape[0]
    if sparse:
        I = sp.identity(dim, dtype=np.complex128, format='csr')
        Hs = sp.csr_matrix(H)
        Lv = -1j * (sp.kron(Hs, I) - sp.kron(I, Hs.T))
        for Lm, g in full_jumps:
            Ls = sp.csr_matrix(Lm)
            LdL = Ls.conj().T @ Ls
            Lv = Lv + g * (sp.kron(Ls, Ls.conj()) - 0.5 * sp.kron(LdL, I)
                           - 0.5 * sp.kron(I, LdL.T))
        return sp.csr_matrix(Lv)
    I = np.eye(dim, dtype=np.complex128)
    Lv = -1j * (np.kron(H, I) - np.kron(I, H.T))
    for Lm, g in full_jumps:
        LdL = Lm.conj().T @ Lm
        Lv += g * (np.kron(Lm, Lm.conj()) - 0.5 * np.kron(LdL, I) - 0.5 * np.kron(I, LdL.T))
    return Lv


def evolve_observables(H, jumps, psi0, dt, n_steps, observables):
    """Exact <O>(k dt) = Tr(rho(k dt) O) for k = 0..n_steps.

    jumps: list of (site, 2x2 op, rate); observables: list of (site, 2x2 op).
    Returns real array [n_steps+1, n_obs]."""
    dim = H.shape[0]
    L = int(round(np.log2(dim)))
    full = [(_full_jump(op, s, L), g) for (s, op, g) in jumps]
    obs = [model.site_op_dense(op, s, L) for (s, op) in observables]
    rho = np.outer(psi0, psi0.conj())
    rho = rho / np.trace(rho)
    vec = rho.reshape(-1)
    sparse = dim * dim > 4096
    Lv = liouvillian(H, full, sparse=sparse)
    prop = None if sparse else sla.expm(Lv * dt)
    out = np.zeros((n_steps + 1, len(obs)))
    for k in range(n_steps + 1):
        r = vec.reshape(dim, dim)
        out[k] = [np.real(np.trace(r @ O)) for O in obs]
        if k == n_steps:
            break
        vec = spla.expm_multiply(Lv * dt, vec) if sparse else prop @ vec
    return out


def rk4_observables(H, jumps, psi0, dt, n_steps, observables, substeps=200):
    """Second, independent integrator: classical RK4 on the matrix form of
    Eq. (Lindblad) (no vectorisation), used only to cross-check the above."""
    dim = H.shape[0]
    L = int(round(np.log2(dim)))
    full = [(_full_jump(op, s, L), g) for (s, op, g) in jumps]
    obs = [model.site_op_dense(op, s, L) for (s, op) in observables]

    def rhs(r):
        out = -1j * (H @ r - r @ H)
        for Lm, g in full:
            LdL = Lm.conj().T @ Lm
            out += g * (Lm @ r @ Lm.conj().T - 0.5 * (LdL @ r + r @ LdL))
        return out

    rho = np.outer(psi0, psi0.conj())
    h = dt / substeps
    out = np.zeros((n_steps + 1, len(obs)))
    for k in range(n_steps + 1):
        out[k] = [np.real(np.trace(rho @ O)) for O in obs]
        if k == n_steps:
            break
        for _ in range(substeps):
            k1 = rhs(rho)
            k2 = rhs(rho + 0.5 * h * k1)
            k3 = rhs(rho + 0.5 * h * k2)
            k4 = rhs(rho + h * k3)
            rho = rho + (h / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return out
