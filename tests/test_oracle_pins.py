"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names what pins it: a published known-answer vector, a closed form
derived from Eq. (Lindblad), an invariant the paper states, a special case
that reduces to a textbook routine, or brute force on tiny inputs.  None of
them re-types the oracle's own formula.
"""
import os

import numpy as np
import scipy.linalg as sla
import pytest

from oracle import dense_tjm, lindblad, model, mps_tjm, philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------
# Philox4x32-10: published known-answer vectors (Salmon et al., SC'11)
# --------------------------------------------------------------------------

def _kat_rows():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    return rows


def test_philox_known_answers():
    rows = _kat_rows()
    assert len(rows) == 3
    for r in rows:
        assert philox.philox4x32_10(r[0:4], r[4:6]) == r[6:10]


def test_philox_draws_are_53bit_uniforms():
    seen = set()
    for t in range(200):
        e, r = philox.draws(0x250117913, t, 3, 1)
        assert 0.0 <= e < 1.0 and 0.0 <= r < 1.0
        assert float(e * 2 ** 53).is_integer()
        seen.add(e)
    assert len(seen) == 200
    # the two streams (main / sample) and steps are distinct counters
    assert philox.draws(5, 0, 1, 0) != philox.draws(5, 0, 1, 1)
    assert philox.draws(5, 0, 1, 0) != philox.draws(5, 0, 2, 0)
    # mean of many draws near 1/2 (4 sigma for N=4000 uniforms)
    xs = [philox.draws(11, t, 0, 0)[0] for t in range(4000)]
    assert abs(np.mean(xs) - 0.5) < 4 * np.sqrt(1 / 12 / 4000)


# --------------------------------------------------------------------------
# Models
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L", [1, 2, 3, 5])
def test_xxx_mpo_matches_kronecker_sum(L):
    for (J, hx, hz) in [(1.0, 0.5, 0.0), (0.7, 0.0, 0.3), (0.0, 1.0, 0.0)]:
        Hm = model.mpo_to_dense(model.xxx_mpo(L, J, hx, hz))
        Hd = model.xxx_dense(L, J, hx, hz)
        assert np.abs(Hm - Hd).max() < 1e-13
        assert np.abs(Hd - Hd.conj().T).max() == 0.0


def test_xxx_two_site_spectrum_closed_form():
    # -J sigma.sigma on two spins: triplet energy -J, singlet +3J.
    H = model.xxx_dense(2, 1.3)
    ev = np.sort(np.linalg.eigvalsh(H))
    assert np.allclose(ev, [-1.3, -1.3, -1.3, 3.9], atol=1e-13)


@pytest.mark.parametrize("L", [2, 4])
def test_tfim_mpo_matches_kronecker_sum(L):
    Hm = model.mpo_to_dense(model.tfim_mpo(L, 1.0, 0.8))
    assert np.abs(Hm - model.tfim_dense(L, 1.0, 0.8)).max() < 1e-13


def test_local_dissipator_closed_form():
    # sigma_-^dag sigma_- = |1><1|, Z^dag Z = I: D = diag(e^{-t gz/2}, e^{-t(gm+gz)/2})
    jumps = model.relax_dephase_jumps(1, 0.3, 0.7)
    D = model.local_dissipator(jumps, 0, 0.4)
    ref = np.diag([np.exp(-0.4 * 0.7 / 2), np.exp(-0.4 * (0.3 + 0.7) / 2)])
    assert np.abs(D - ref).max() < 1e-15


# --------------------------------------------------------------------------
# O1 exact Lindblad: closed forms for one spin (Eq. Lindblad), and a second
# independent integrator
# --------------------------------------------------------------------------

def test_lindblad_amplitude_damping_closed_form():
    g, dt, n = 0.37, 0.25, 12
    H = np.zeros((2, 2), dtype=complex)
    out = lindblad.evolve_observables(H, [(0, model.SIGMA_MINUS, g)],
                                      np.array([0, 1], dtype=complex), dt, n, [(0, model.Z)])
    t = dt * np.arange(n + 1)
    assert np.abs(out[:, 0] - (1 - 2 * np.exp(-g * t))).max() < 1e-13


def test_lindblad_dephasing_closed_form():
    g, dt, n = 0.21, 0.3, 10
    H = np.zeros((2, 2), dtype=complex)
    plus = np.array([1, 1], dtype=complex) / np.sqrt(2)
    out = lindblad.evolve_observables(H, [(0, model.Z, g)], plus, dt, n, [(0, model.X)])
    t = dt * np.arange(n + 1)
    assert np.abs(out[:, 0] - np.exp(-2 * g * t)).max() < 1e-13


def test_lindblad_both_channels_closed_form():
    # population relaxes at gm; coherence decays at gm/2 + 2 gz; with a Z
    # field hz the coherence also precesses at 2 hz.
    gm, gz, hz, dt, n = 0.2, 0.05, 0.4, 0.2, 15
    H = -hz * model.Z
    psi = np.array([np.cos(0.3), np.sin(0.3) * np.exp(0.2j)])
    out = lindblad.evolve_observables(H, [(0, model.SIGMA_MINUS, gm), (0, model.Z, gz)], psi,
                                      dt, n, [(0, model.Z), (0, model.X), (0, model.Y)])
    t = dt * np.arange(n + 1)
    p1 = np.sin(0.3) ** 2 * np.exp(-gm * t)
    assert np.abs(out[:, 0] - (1 - 2 * p1)).max() < 1e-13
    c0 = np.cos(0.3) * np.sin(0.3) * np.exp(0.2j)          # rho_01 = a conj(b)... at t=0
    rho01_0 = np.cos(0.3) * np.conj(np.sin(0.3) * np.exp(0.2j))
    rho01 = rho01_0 * np.exp(-(gm / 2 + 2 * gz) * t) * np.exp(2j * hz * t)
    assert np.abs(out[:, 1] - 2 * rho01.real).max() < 1e-13
    assert np.abs(out[:, 2] - (-2 * rho01.imag)).max() < 1e-13
    del c0


def test_lindblad_relaxation_excitation_closed_form():
    # sigma_minus at gm and sigma_plus at gp: d<Z>/dt = (gm - gp) - (gm + gp) <Z>,
    # so <Z> relaxes to (gm - gp)/(gm + gp) at rate gm + gp; the coherence
    # decays at (gm + gp)/2
    gm, gp, dt, n = 0.3, 0.12, 0.25, 14
    H = np.zeros((2, 2), dtype=complex)
    psi = np.array([np.cos(0.4), np.sin(0.4)], dtype=complex)
    out = lindblad.evolve_observables(H, [(0, model.SIGMA_MINUS, gm), (0, model.SIGMA_PLUS, gp)], psi, dt, n,
                                      [(0, model.Z), (0, model.X)])
    t = dt * np.arange(n + 1)
    zinf = (gm - gp) / (gm + gp)
    z0 = np.cos(0.8)
    assert np.abs(out[:, 0] - (zinf + (z0 - zinf) * np.exp(-(gm + gp) * t))).max() < 1e-13
    assert np.abs(out[:, 1] - np.sin(0.8) * np.exp(-0.5 * (gm + gp) * t)).max() < 1e-13


def test_domain_wall_bits():
    # sites 1..L/2-1 in |0>, sites L/2..L in |1> (1-based), odd L included
    assert model.domain_wall_bits(30) == [0] * 14 + [1] * 16
    assert model.domain_wall_bits(7) == [0] * 3 + [1] * 4
    assert model.domain_wall_bits(2) == [1, 1]


def test_lindblad_vectorised_vs_rk4_three_sites():
    L = 3
    H = model.xxx_dense(L, 1.0, 0.5)
    jumps = model.relax_dephase_jumps(L, 0.1, 0.1)
    psi = model.product_dense(model.product_site_vectors(L, [0, 1, 0]))
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    a = lindblad.evolve_observables(H, jumps, psi, 0.1, 10, obs)
    b = lindblad.rk4_observables(H, jumps, psi, 0.1, 10, obs, substeps=100)
    assert np.abs(a - b).max() < 1e-10


def test_lindblad_sparse_path_matches_dense():
    # L = 7 takes the expm_multiply path; compare two sites' worth with the
    # dense path by embedding an idle site (H and jumps do not touch it).
    L = 3
    H3 = model.xxx_dense(L, 1.0, 0.5)
    jumps = model.relax_dephase_jumps(L, 0.1, 0.1)
    psi3 = model.product_dense(model.product_site_vectors(L, [0, 1, 0]))
    obs = [(0, model.Z), (1, model.X)]
    a = lindblad.evolve_observables(H3, jumps, psi3, 0.1, 5, obs)
    L7 = 7
    H7 = np.kron(H3, np.eye(2 ** 4))
    psi7 = np.kron(psi3, model.product_dense(model.product_site_vectors(4, [0, 0, 0, 0])))
    b = lindblad.evolve_observables(H7, jumps, psi7, 0.1, 5, obs)
    assert L7 == 7 and np.abs(a - b).max() < 1e-10


# --------------------------------------------------------------------------
# P2: exact discrete-time TJM expectations for one spin (schedule of
# Eq. TimeEvolutionFunctions with H0 = 0), per trajectory and in mean
# --------------------------------------------------------------------------

def _first_relaxation_event(seed, traj, g, dt, n):
    """Brute force from the draws: the first jump process where eps < dp."""
    dp_half = 1 - np.exp(-g * dt / 2)
    dp_full = 1 - np.exp(-g * dt)
    if philox.draws(seed, traj, 0, 0)[0] < dp_half:
        return (0, 0)
    for k in range(1, n + 1):
        if philox.draws(seed, traj, k, 1)[0] < dp_half:
            return (k, 1)
        if k < n and philox.draws(seed, traj, k, 0)[0] < dp_full:
            return (k, 0)
    return None


def test_single_spin_relaxation_jump_times_are_the_draws():
    g, dt, n, seed = 0.5, 0.1, 12, 99
    Ws = model.xxx_mpo(1, 0.0)
    jumps = [(0, model.SIGMA_MINUS, g)]
    psi0 = mps_tjm.product_mps(model.product_site_vectors(1, [1]))
    opt = mps_tjm.Options(chi_max=4)
    for traj in range(40):
        rec = {}
        out = mps_tjm.run_trajectory(Ws, jumps, psi0, dt, n, [(0, model.Z)], seed, traj, opt, rec)
        ev = _first_relaxation_event(seed, traj, g, dt, n)
        hits = [(k, b) for (k, b, m) in rec['jumps'] if m >= 0]
        if ev is None:
            assert hits == [] and np.all(np.abs(out[1:, 0] + 1) < 1e-14)
        else:
            assert hits[0] == ev
            if ev[1] == 0:      # main-branch jump: |0> from then on
                assert np.all(np.abs(out[ev[0] + 1:, 0] - 1) < 1e-14)
            else:               # sample-branch jump only affects that sample
                assert abs(out[ev[0], 0] - 1) < 1e-14


def test_single_spin_mean_relaxation_exact_in_dt():
    g, dt, n, N = 0.5, 0.2, 10, 1500
    Ws = model.xxx_mpo(1, 0.0)
    jumps = [(0, model.SIGMA_MINUS, g)]
    psi0 = mps_tjm.product_mps(model.product_site_vectors(1, [1]))
    opt = mps_tjm.Options(chi_max=2)
    zs = np.array([mps_tjm.run_trajectory(Ws, jumps, psi0, dt, n, [(0, model.Z)], 3, t, opt)[:, 0]
                   for t in range(N)])
    k = np.arange(n + 1)
    p = np.exp(-g * k * dt)                       # P(still |1>) at sample k
    exact = 1 - 2 * p
    se = 2 * np.sqrt(p * (1 - p) / N) + 1e-12
    assert np.all(np.abs(zs.mean(0) - exact) <= 4 * se)


def test_single_spin_mean_dephasing_exact_in_dt():
    g, dt, n, N = 0.4, 0.25, 8, 1500
    Ws = model.xxx_mpo(1, 0.0)
    jumps = [(0, model.Z, g)]
    psi0 = mps_tjm.product_mps([np.array([1, 1]) / np.sqrt(2)])
    opt = mps_tjm.Options(chi_max=2)
    xs = np.array([mps_tjm.run_trajectory(Ws, jumps, psi0, dt, n, [(0, model.X)], 8, t, opt)[:, 0]
                   for t in range(N)])
    k = np.arange(1, n + 1)
    exact = (2 * np.exp(-g * dt / 2) - 1) ** 2 * (2 * np.exp(-g * dt) - 1) ** (k - 1)
    # each sample is +-1: binomial standard error
    se = np.sqrt((1 - exact ** 2) / N)
    assert np.all(np.abs(xs.mean(0)[1:] - exact) <= 4 * se)
    assert abs(xs.mean(0)[0] - 1) < 1e-14


# --------------------------------------------------------------------------
# P3: gamma = 0, |0...0>, X field: independent spin rotation, <Z> = cos(2gt)
# (exact for any J: |0..0> stays in the maximal-spin multiplet)
# --------------------------------------------------------------------------

def test_free_rotation_closed_form_non_interacting():
    L, g, dt, n = 5, 0.5, 0.1, 20
    Ws = model.xxx_mpo(L, 0.0, g)
    psi0 = mps_tjm.product_mps(model.product_site_vectors(L, model.zero_bits(L)))
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    rec = {}
    out = mps_tjm.run_trajectory(Ws, [], psi0, dt, n, obs, 1, 0, mps_tjm.Options(chi_max=4), rec)
    t = dt * np.arange(n + 1)
    assert np.abs(out[:, :L] - np.cos(2 * g * t)[:, None]).max() < 1e-10
    assert np.abs(out[:, L:]).max() < 1e-10
    assert all(max(b) == 1 for b in rec['bonds'])


def test_free_rotation_interacting_second_order_in_dt():
    # With J != 0 the exact answer is still cos(2gt) (maximal-spin multiplet),
    # but the local two-site updates carry the O(dt^2) splitting error of a
    # second-order integrator (Sec. "Dynamic TDVP", Ref. Lubich 2008): the
    # error at fixed T must drop by 4 when dt halves.
    L, g, T = 5, 0.5, 2.0
    Ws = model.xxx_mpo(L, 1.0, g)
    obs = [(s, model.Z) for s in range(L)]
    errs = []
    for dt in (0.1, 0.05, 0.025):
        n = int(round(T / dt))
        psi0 = mps_tjm.product_mps(model.product_site_vectors(L, model.zero_bits(L)))
        out = mps_tjm.run_trajectory(Ws, [], psi0, dt, n, obs, 1, 0, mps_tjm.Options(chi_max=4))
        errs.append(np.abs(out[-1] - np.cos(2 * g * T)).max())
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5
    assert errs[-1] < 5e-4


# --------------------------------------------------------------------------
# P4: full-rank mode (no truncation, maximal bonds) makes projector-splitting
# TDVP exact, so the MPS oracle equals the dense-vector TJM per trajectory
# --------------------------------------------------------------------------

@pytest.mark.parametrize("L,chi_max", [(3, 8), (4, 2), (4, 16), (5, 4)])
def test_full_rank_mps_equals_dense_per_trajectory(L, chi_max):
    rng = np.random.default_rng(L * 100 + chi_max)
    psi = rng.normal(size=2 ** L) + 1j * rng.normal(size=2 ** L)
    psi /= np.linalg.norm(psi)
    m0 = mps_tjm.dense_to_mps(psi, L)
    assert np.abs(mps_tjm.mps_to_dense(m0) - psi).max() < 1e-14
    Ws = model.xxx_mpo(L, 1.0, 0.5)
    H = model.xxx_dense(L, 1.0, 0.5)
    jumps = model.relax_dephase_jumps(L, 0.2, 0.2)
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    opt = mps_tjm.Options(chi_max=chi_max, chi_cap=2 ** L, svd_discard=-1.0)
    n_jumps = 0
    for traj in range(5):
        r1, r2 = {}, {}
        a = mps_tjm.run_trajectory(Ws, jumps, m0, 0.1, 8, obs, 7, traj, opt, r1)
        b = dense_tjm.run_trajectory(H, jumps, psi, 0.1, 8, obs, 7, traj, r2)
        assert r1['jumps'] == r2['jumps']
        assert np.abs(a - b).max() < 1e-11
        n_jumps += sum(1 for x in r1['jumps'] if x[2] >= 0)
    assert n_jumps > 0


def test_two_site_chain_tdvp_is_exact_with_truncation_rule():
    # L = 2: the two-site effective Hamiltonian is H0 itself.
    L = 2
    Ws = model.xxx_mpo(L, 1.0, 0.5)
    H = model.xxx_dense(L, 1.0, 0.5)
    jumps = model.relax_dephase_jumps(L, 0.3, 0.1)
    sv = model.product_site_vectors(L, [0, 1])
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    for traj in range(8):
        r1, r2 = {}, {}
        a = mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, 10, obs, 5, traj,
                                   mps_tjm.Options(chi_max=4), r1)
        b = dense_tjm.run_trajectory(H, jumps, model.product_dense(sv), 0.1, 10, obs, 5, traj, r2)
        assert r1['jumps'] == r2['jumps']
        assert np.abs(a - b).max() < 1e-10


def test_zero_hamiltonian_entangled_state_dissipation_and_jumps_exact():
    # H0 = 0: U is the identity, D and J are exact (Sec. "Projection error"
    # statement that dissipation and jumps add no error); the only loss is
    # the <= 1e-12 discarded weight of the post-jump SVD sweeps.
    L = 5
    rng = np.random.default_rng(3)
    psi = rng.normal(size=2 ** L) + 1j * rng.normal(size=2 ** L)
    psi /= np.linalg.norm(psi)
    m0 = mps_tjm.dense_to_mps(psi, L)
    Ws = model.xxx_mpo(L, 0.0)
    H = np.zeros((2 ** L, 2 ** L), dtype=complex)
    jumps = model.relax_dephase_jumps(L, 0.3, 0.2)
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    for traj in range(5):
        r1, r2 = {}, {}
        a = mps_tjm.run_trajectory(Ws, jumps, m0, 0.1, 8, obs, 9, traj,
                                   mps_tjm.Options(chi_max=4), r1)
        b = dense_tjm.run_trajectory(H, jumps, psi, 0.1, 8, obs, 9, traj, r2)
        assert r1['jumps'] == r2['jumps']
        assert np.abs(a - b).max() < 1e-10


# --------------------------------------------------------------------------
# P5: invariants
# --------------------------------------------------------------------------

def _random_mps(L, chi, rng):
    psi = rng.normal(size=2 ** L) + 1j * rng.normal(size=2 ** L)
    m = mps_tjm.dense_to_mps(psi / np.linalg.norm(psi), L)
    return m


def test_tdvp_preserves_norm_canonical_form_and_energy():
    L = 6
    rng = np.random.default_rng(4)
    mps = _random_mps(L, 8, rng)
    mps_tjm.canonicalize(mps)
    Ws = model.xxx_mpo(L, 1.0, 0.5)
    H = model.xxx_dense(L, 1.0, 0.5)
    e0 = np.real(np.vdot(mps_tjm.mps_to_dense(mps), H @ mps_tjm.mps_to_dense(mps)))
    opt = mps_tjm.Options(chi_max=4)          # saturated bonds: 1TDVP in the bulk
    st = mps_tjm.Stats()
    for _ in range(5):
        mps_tjm.tdvp_step(mps, Ws, 0.1, opt, st)
        v = mps_tjm.mps_to_dense(mps)
        assert abs(np.linalg.norm(v) - 1) < 1e-11
        for s in range(1, L):                 # right-canonical away from the centre
            M = mps[s]
            G = np.einsum('sab,scb->ac', M, M.conj())
            assert np.abs(G - np.eye(G.shape[0])).max() < 1e-12
    assert st.one_site > 0
    e1 = np.real(np.vdot(v, H @ v))
    assert abs(e1 - e0) < 1e-9


def test_dissipation_keeps_bond_dimensions():
    L = 5
    rng = np.random.default_rng(5)
    mps = _random_mps(L, 4, rng)
    before = mps_tjm.bonds(mps)
    jumps = model.relax_dephase_jumps(L, 0.1, 0.1)
    mps_tjm.dissipate(mps, [model.local_dissipator(jumps, s, 0.1) for s in range(L)])
    assert mps_tjm.bonds(mps) == before


def test_gamma_zero_means_no_jumps_and_pure_tdvp():
    L = 4
    Ws = model.xxx_mpo(L, 1.0, 0.5)
    sv = model.product_site_vectors(L, model.neel_bits(L))
    obs = [(s, model.Z) for s in range(L)]
    opt = mps_tjm.Options(chi_max=4)
    rec = {}
    a = mps_tjm.run_trajectory(Ws, model.relax_dephase_jumps(L, 0.0, 0.0),
                               mps_tjm.product_mps(sv), 0.1, 6, obs, 1, 0, opt, rec)
    assert all(m < 0 for (_, _, m) in rec['jumps'])
    mps = mps_tjm.product_mps(sv)
    ref = [mps_tjm.expectation_values(mps, obs)]
    for _ in range(6):
        mps_tjm.tdvp_step(mps, Ws, 0.1, opt, mps_tjm.Stats())
        ref.append(mps_tjm.expectation_values(mps, obs))
    assert np.abs(a - np.array(ref)).max() < 1e-13


def test_relaxation_only_on_vacuum_is_static():
    L = 4
    Ws = model.xxx_mpo(L, 1.0, 0.0)
    jumps = [(s, model.SIGMA_MINUS, 0.3) for s in range(L)]
    psi0 = mps_tjm.product_mps(model.product_site_vectors(L, model.zero_bits(L)))
    rec = {}
    out = mps_tjm.run_trajectory(Ws, jumps, psi0, 0.1, 6, [(s, model.Z) for s in range(L)],
                                 2, 0, mps_tjm.Options(chi_max=4), rec)
    assert np.abs(out - 1).max() < 1e-12
    assert all(m < 0 for (_, _, m) in rec['jumps'])


def test_truncation_rule_cases():
    s = np.array([1.0, 0.5, 0.5, 1e-7, 1e-9])
    # tail after k=3 is 1e-14 + 1e-18 <= 1e-12 * total
    assert mps_tjm.truncation_rank(s, 1e-12, 10, 1e-12) == 3
    # cap 2 cuts the degenerate pair (0.5, 0.5): lowered to 1
    assert mps_tjm.truncation_rank(s, 1e-12, 2, 1e-12) == 1
    assert mps_tjm.truncation_rank(s, -1.0, 10, 1e-12) == 5
    assert mps_tjm.truncation_rank(np.array([1.0, 1.0]), 1e-12, 1, 1e-12) == 1


# --------------------------------------------------------------------------
# Krylov exponential against a dense matrix exponential
# --------------------------------------------------------------------------

def test_expm_krylov_matches_dense_expm():
    import scipy.linalg as sla
    rng = np.random.default_rng(6)
    n = 40
    A = rng.normal(size=(n, n)) + 1j * rng.normal(size=(n, n))
    Hm = (A + A.conj().T) / 2
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    for t in (0.05, -0.05, 0.3):
        ref = sla.expm(-1j * t * Hm) @ v
        got = mps_tjm.expm_krylov(lambda x: Hm @ x, v, t, 30, 1e-12)
        assert np.abs(got - ref).max() < 1e-10 * np.linalg.norm(v)
    small = mps_tjm.expm_krylov(lambda x: Hm[:2, :2] @ x, v[:2], 0.7, 30, 1e-12)
    assert np.abs(small - sla.expm(-0.7j * Hm[:2, :2]) @ v[:2]).max() < 1e-13


# --------------------------------------------------------------------------
# MPO observables (Eq. TJMExpVal with O an MPO; Methods, "Resources required
# for calculating expectation values"): the MPS-MPO-MPS contraction against
# dense linear algebra with operators built from Kronecker products
# --------------------------------------------------------------------------

def _random_mps_bonds(rng, bonds):
    L = len(bonds) - 1
    return [rng.normal(size=(2, bonds[s], bonds[s + 1])) + 1j * rng.normal(size=(2, bonds[s], bonds[s + 1]))
            for s in range(L)]


@pytest.mark.parametrize("bonds", [[1, 2, 4, 8, 4, 2, 1], [1, 2, 3, 3, 3, 2, 1], [1, 1, 1, 1, 1, 1, 1]])
def test_mpo_expectation_matches_dense(bonds):
    rng = np.random.default_rng(sum(bonds))
    L = len(bonds) - 1
    mps = _random_mps_bonds(rng, bonds)      # any gauge, any norm
    psi = mps_tjm.mps_to_dense(mps)
    nrm = np.real(np.vdot(psi, psi))

    def dense_ev(O):
        return np.real(np.vdot(psi, O @ psi)) / nrm

    H = model.xxx_dense(L, 1.0, 0.3, 0.7)
    assert abs(mps_tjm.mpo_expectation(mps, model.xxx_mpo(L, 1.0, 0.3, 0.7)) - dense_ev(H)) < 1e-12 * max(1, abs(dense_ev(H)))
    for i in range(L - 1):
        XX = model.site_op_dense(model.X, i, L) @ model.site_op_dense(model.X, i + 1, L)
        v = mps_tjm.mpo_expectation(mps, model.product_mpo(L, {i: model.X, i + 1: model.X}))
        assert abs(v - dense_ev(XX)) < 1e-12
    ZYZ = model.site_op_dense(model.Z, 0, L) @ model.site_op_dense(model.Y, 2, L) @ model.site_op_dense(model.Z, L - 1, L)
    v = mps_tjm.mpo_expectation(mps, model.product_mpo(L, {0: model.Z, 2: model.Y, L - 1: model.Z}))
    assert abs(v - dense_ev(ZYZ)) < 1e-12
    assert abs(mps_tjm.mpo_expectation(mps, model.product_mpo(L, {})) - 1.0) < 1e-12


def test_full_rank_mpo_observables_equal_dense_tjm_per_trajectory():
    # energy and nearest-neighbour XX correlators measured on the MPS
    # trajectories equal the dense-vector TJM's with Kronecker-product
    # operators, trajectory by trajectory
    L = 4
    rng = np.random.default_rng(44)
    psi = rng.normal(size=2 ** L) + 1j * rng.normal(size=2 ** L)
    psi /= np.linalg.norm(psi)
    m0 = mps_tjm.dense_to_mps(psi, L)
    Ws = model.xxx_mpo(L, 1.0, 0.5)
    H = model.xxx_dense(L, 1.0, 0.5)
    jumps = model.relax_dephase_jumps(L, 0.2, 0.2)
    obs = [(s, model.Z) for s in range(L)]
    mpo_obs = [Ws] + [model.product_mpo(L, {i: model.X, i + 1: model.X}) for i in range(L - 1)]
    dense_obs = [H] + [model.site_op_dense(model.X, i, L) @ model.site_op_dense(model.X, i + 1, L) for i in range(L - 1)]
    opt = mps_tjm.Options(chi_max=16, chi_cap=16, svd_discard=-1.0)
    for traj in range(4):
        r1, r2 = {}, {}
        a = mps_tjm.run_trajectory(Ws, jumps, m0, 0.1, 6, obs, 3, traj, opt, r1, mpo_observables=mpo_obs)
        b = dense_tjm.run_trajectory(H, jumps, psi, 0.1, 6, obs, 3, traj, r2, dense_observables=dense_obs)
        assert r1['jumps'] == r2['jumps']
        assert a.shape == b.shape == (7, L + L)
        assert np.abs(a - b).max() < 1e-11


# --------------------------------------------------------------------------
# The first-order splitting of Sec. "Higher-order Trotterization" against
# the second-order schedule: for one spin with a field and sigma_minus
# damping, every jump resets the spin to |0>, so the exact trajectory
# average of each schedule follows from the distribution of the last reset
# (computed here with 2x2 matrices from the definitions, independently of
# the oracle's TJM code) and is compared with the exact Lindblad solution
# from the 4x4 Liouvillian written out below.
# --------------------------------------------------------------------------

def _spin_setup(g, gam, dt):
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Zm = np.diag([1.0, -1.0]).astype(complex)
    sm = np.array([[0, 1], [0, 0]], dtype=complex)
    H = -g * X
    U = sla.expm(-1j * H * dt)
    Dof = lambda tau: sla.expm(-0.5 * tau * gam * sm.conj().T @ sm)
    return X, Zm, sm, H, U, Dof


def _exact_schedule_average(order, g, gam, dt, n, psi0):
    """E[<Z>(t_k)] over trajectories of the schedule (k = 0..n)."""
    X, Zm, sm, H, U, Dof = _spin_setup(g, gam, dt)
    Dh, Df = Dof(0.5 * dt), Dof(dt)
    zero = np.array([1.0, 0.0], dtype=complex)
    ez = lambda v: np.real(np.vdot(v, Zm @ v)) / np.real(np.vdot(v, v))

    def jump_step(D, v):
        """(no-jump state, no-jump probability) of J D applied to v (|v| = 1)."""
        w = D @ v
        p0 = np.real(np.vdot(w, w))
        return w / np.sqrt(p0), p0

    # a distribution over main-chain states: list of (probability, state)
    out = [ez(psi0)]
    if order == 1:
        dist = [(1.0, psi0)]
        for k in range(1, n + 1):
            nd, reset = [], 0.0
            for (p, v) in dist:
                w, p0 = jump_step(Df, U @ v)
                nd.append((p * p0, w))
                reset += p * (1 - p0)
            dist = nd + [(reset, zero)]
            out.append(sum(p * ez(v) for p, v in dist))
        return np.array(out)
    w, p0 = jump_step(Dh, psi0)                        # F_0 = J D[dt/2]
    dist = [(p0, w), (1 - p0, zero)]
    for k in range(1, n + 1):
        xs = [(p, U @ v) for (p, v) in dist]           # X = U Phi
        # measured sample J_s D[dt/2] X, averaged over its own draw
        e = 0.0
        for (p, x) in xs:
            ws, ps = jump_step(Dh, x)
            e += p * (ps * ez(ws) + (1 - ps) * ez(zero))
        out.append(e)
        nd, reset = [], 0.0
        for (p, x) in xs:                              # Phi = J D[dt] X
            w, p0 = jump_step(Df, x)
            nd.append((p * p0, w))
            reset += p * (1 - p0)
        dist = nd + [(reset, zero)]
    return np.array(out)


def _lindblad_spin_z(g, gam, T, psi0):
    X, Zm, sm, H, U, Dof = _spin_setup(g, gam, 1.0)
    I = np.eye(2)
    # vec(A rho B) = (B^T kron A) vec(rho), column stacking
    Lv = (-1j * (np.kron(I, H) - np.kron(H.T, I))
          + gam * (np.kron(sm.conj(), sm) - 0.5 * np.kron(I, sm.conj().T @ sm)
                   - 0.5 * np.kron((sm.conj().T @ sm).T, I)))
    rho = np.outer(psi0, psi0.conj()).reshape(-1, order='F')
    r = (sla.expm(Lv * T) @ rho).reshape(2, 2, order='F')
    return np.real(np.trace(Zm @ r))


def test_first_order_splitting_error_is_first_order_and_strang_second_order():
    g, gam, T = 1.0, 0.8, 2.0
    psi0 = np.array([np.cos(0.3), np.sin(0.3)], dtype=complex)
    exact = _lindblad_spin_z(g, gam, T, psi0)
    e1, e2 = [], []
    for dt in (0.1, 0.05, 0.025):
        n = int(round(T / dt))
        e1.append(abs(_exact_schedule_average(1, g, gam, dt, n, psi0)[-1] - exact))
        e2.append(abs(_exact_schedule_average(2, g, gam, dt, n, psi0)[-1] - exact))
    assert 1.7 < e1[0] / e1[1] < 2.3 and 1.7 < e1[1] / e1[2] < 2.3
    assert 3.4 < e2[0] / e2[1] < 4.6 and 3.4 < e2[1] / e2[2] < 4.6
    assert e2[-1] < e1[-1] / 10


def test_first_order_oracle_ensemble_matches_its_exact_average():
    # the oracle's first-order MPS TJM on one spin, averaged over trajectories,
    # against the exact average of the same schedule
    g, gam, dt, n, N = 1.0, 0.8, 0.1, 20, 3000
    psi0 = np.array([np.cos(0.3), np.sin(0.3)], dtype=complex)
    ref = _exact_schedule_average(1, g, gam, dt, n, psi0)
    Ws = model.xxx_mpo(1, 1.0, g)
    jumps = [(0, model.SIGMA_MINUS, gam)]
    per = np.array([mps_tjm.run_trajectory(Ws, jumps, [psi0.reshape(2, 1, 1)], dt, n, [(0, model.Z)], 11, t,
                                           mps_tjm.Options(chi_max=2), order=1)[:, 0] for t in range(N)])
    m, se = per.mean(0), per.std(0, ddof=1) / np.sqrt(N)
    assert np.all(np.abs(m - ref) <= 4 * se + 1e-12)


def test_first_order_full_rank_mps_equals_dense_per_trajectory():
    L = 4
    rng = np.random.default_rng(41)
    psi = rng.normal(size=2 ** L) + 1j * rng.normal(size=2 ** L)
    psi /= np.linalg.norm(psi)
    m0 = mps_tjm.dense_to_mps(psi, L)
    Ws = model.xxx_mpo(L, 1.0, 0.5)
    H = model.xxx_dense(L, 1.0, 0.5)
    jumps = model.relax_dephase_jumps(L, 0.3, 0.3)
    obs = [(s, model.Z) for s in range(L)] + [(s, model.X) for s in range(L)]
    opt = mps_tjm.Options(chi_max=16, chi_cap=16, svd_discard=-1.0)
    n_jumps = 0
    for traj in range(5):
        r1, r2 = {}, {}
        a = mps_tjm.run_trajectory(Ws, jumps, m0, 0.1, 8, obs, 13, traj, opt, r1, order=1)
        b = dense_tjm.run_trajectory(H, jumps, psi, 0.1, 8, obs, 13, traj, r2, order=1)
        assert r1['jumps'] == r2['jumps']
        assert np.abs(a - b).max() < 1e-11
        n_jumps += sum(1 for x in r1['jumps'] if x[2] >= 0)
    assert n_jumps > 0
