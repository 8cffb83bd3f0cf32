"""Inputs of the C ABI: Hamiltonians as MPOs, jump sets, observables and
product states, in the layouts of include/tjm.h.

An MPO site tensor is W[s_out, s_in, w_left, w_right] (Methods, MPO section of
arXiv:2501.17913); operators are [s_out, s_in] in the basis (|0>, |1>) with
Z = diag(1, -1) and sigma_minus = |0><1| (Sec. "Benchmarking").
"""
import numpy as np

PAULI_X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
PAULI_Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
PAULI_Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
IDENT = np.eye(2, dtype=np.complex128)
LOWER = np.array([[0, 1], [0, 0]], dtype=np.complex128)    # sigma_minus
RAISE = np.array([[0, 0], [1, 0]], dtype=np.complex128)    # sigma_plus


def _finite_state_mpo(L, blocks, D):
    """MPO of a finite-state machine: `blocks` maps (w_left, w_right) -> 2x2
    operator of the bulk tensor; the first site keeps channel D-1 on its left,
    the last site channel 0 on its right."""
    bulk = np.zeros((2, 2, D, D), dtype=np.complex128)
    for (a, b), op in blocks.items():
        bulk[:, :, a, b] = op
    if L == 1:
        return [bulk[:, :, D - 1:D, 0:1].copy()]
    return [bulk[:, :, D - 1:D, :].copy()] + [bulk.copy() for _ in range(L - 2)] + [bulk[:, :, :, 0:1].copy()]


def xxx_mpo(L, J=1.0, hx=0.0, hz=0.0):
    """H0 = -J sum (X X + Y Y + Z Z) - hx sum X - hz sum Z (open chain), D = 5.

    Channel 4 carries 'identity so far', channels 1..3 a pending X/Y/Z, channel
    0 'Hamiltonian complete'."""
    blocks = {(0, 0): IDENT, (1, 0): PAULI_X, (2, 0): PAULI_Y, (3, 0): PAULI_Z,
              (4, 0): -hx * PAULI_X - hz * PAULI_Z,
              (4, 1): -J * PAULI_X, (4, 2): -J * PAULI_Y, (4, 3): -J * PAULI_Z, (4, 4): IDENT}
    return _finite_state_mpo(L, blocks, 5)


def tfim_mpo(L, J=1.0, g=1.0):
    """H0 = -J sum Z Z - g sum X (Sec. "Benchmarking"), D = 3."""
    blocks = {(0, 0): IDENT, (1, 0): PAULI_Z, (2, 0): -g * PAULI_X, (2, 1): -J * PAULI_Z, (2, 2): IDENT}
    return _finite_state_mpo(L, blocks, 3)


def relaxation_dephasing(L, gamma_minus, gamma_z):
    """sigma_minus and Z on every site, site-major (sites, ops, rates)."""
    sites, ops, rates = [], [], []
    for l in range(L):
        sites += [l, l]
        ops += [LOWER, PAULI_Z]
        rates += [gamma_minus, gamma_z]
    return np.array(sites, dtype=np.int32), np.array(ops), np.array(rates, dtype=np.float64)


def relaxation_excitation(L, gamma_minus, gamma_plus):
    """sigma_minus and sigma_plus on every site, site-major (the jump set of
    the 30-site comparison, Sec. "New frontiers")."""
    sites, ops, rates = [], [], []
    for l in range(L):
        sites += [l, l]
        ops += [LOWER, RAISE]
        rates += [gamma_minus, gamma_plus]
    return np.array(sites, dtype=np.int32), np.array(ops), np.array(rates, dtype=np.float64)


def zx_observables(L):
    """<Z_l> for every site, then <X_l> for every site."""
    return [(l, PAULI_Z) for l in range(L)] + [(l, PAULI_X) for l in range(L)]


def product_state(bits):
    v = np.zeros((len(bits), 2), dtype=np.complex128)
    v[np.arange(len(bits)), bits] = 1.0
    return v


def neel(L):
    """|0101...>: site 1 (index 0) in |0>."""
    return product_state([l % 2 for l in range(L)])


def domain_wall(L):
    """Domain wall of the 30-site comparison: site l (1-based) in |0> for
    l < L/2 and in |1> from L/2 on."""
    return product_state([0 if l + 1 < L / 2 else 1 for l in range(L)])


def all_zero(L):
    return product_state([0] * L)


def xxx_model(L, J=1.0, g=0.5, gamma=0.1):
    """The workload chain: XXX with transverse (X) field g, sigma_minus and Z
    jumps at rate gamma on every site.  Returns (mpo, sites, ops, rates)."""
    s, o, r = relaxation_dephasing(L, gamma, gamma)
    return xxx_mpo(L, J, g), s, o, r


def domain_wall_model(L, J=1.0, h=1.0, gamma=0.1):
    """The 30-site comparison chain (Sec. "New frontiers"): XXX with a Z
    field h, sigma_minus and sigma_plus at rate gamma on every site.  Returns
    (mpo, sites, ops, rates); the initial state is domain_wall(L)."""
    s, o, r = relaxation_excitation(L, gamma, gamma)
    return xxx_mpo(L, J, 0.0, h), s, o, r
