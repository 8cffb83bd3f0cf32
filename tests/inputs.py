"""Seeded synthetic workloads shared by the oracle side and the HIP side of the
tests.  Parameters only; no arithmetic of the method lives here.

The workloads are the XXX chain of Sec. "New frontiers" with a transverse
(X) field g, sigma_minus and Z jump operators on every site at one rate
(Sec. "Benchmarking"), open boundaries, product initial states.  No dataset
is involved: the paper's experiments run on synthetic chains of this kind.
"""

SEED = 0x250117913


def workload(name):
    """Named configurations: C1..C4 are the sizes the measurements use."""
    table = {
        # L=6, chi 8, 200 trajectories, T=2, |0...0>
        "C1": dict(L=6, J=1.0, g=0.5, gamma=0.1, chi_max=8, dt=0.1, T=2.0, n_traj=200, init="zero"),
        # L=40, chi 32, 1024 trajectories, T=5, Neel
        "C2": dict(L=40, J=1.0, g=0.5, gamma=0.1, chi_max=32, dt=0.1, T=5.0, n_traj=1024, init="neel"),
        # L=100, chi 64, 4096 trajectories, T=5, Neel
        "C3": dict(L=100, J=1.0, g=0.5, gamma=0.1, chi_max=64, dt=0.1, T=5.0, n_traj=4096, init="neel"),
        # L=1000, chi 16, 512 trajectories, T=2, |0...0>
        "C4": dict(L=1000, J=1.0, g=0.5, gamma=0.1, chi_max=16, dt=0.1, T=2.0, n_traj=512, init="zero"),
    }
    return dict(table[name], seed=SEED + int(name[1:]))


def init_bits(L, init):
    if init == "zero":
        return [0] * L
    if init == "neel":
        return [l % 2 for l in range(L)]
    raise ValueError(init)


def small_cases():
    """Ragged shapes that still exercise 1-site and 2-site updates, capped
    bonds, odd and tiny chains: (L, chi_max, init, n_steps, n_traj, g, gamma)."""
    return [
        (1, 4, "neel", 6, 6, 0.5, 0.1),
        (2, 4, "neel", 6, 6, 0.5, 0.2),
        (5, 4, "neel", 8, 8, 0.5, 0.1),
        (6, 8, "zero", 20, 16, 0.5, 0.1),
        (9, 6, "neel", 10, 8, 0.7, 0.15),
        (12, 6, "neel", 10, 8, 0.5, 0.1),
        (13, 5, "zero", 8, 8, 0.9, 0.3),
    ]


def serving_stream(K, seed=5):
    """The serving stream: K requests arriving as a Poisson process of mean
    inter-arrival 0.05 s, each an independent job on the XXX chain (J = 1)
    with L ~ U{20..200}, chi_max in {16, 32, 64}, one rate gamma ~ U[0.01,
    0.2] for both jump channels, field g ~ U[0, 1], N ~ U{64..512}
    trajectories, dt = 0.1, T ~ U[1, 5] rounded to a multiple of dt, Neel
    initial state.  Returns a list of dicts with arrival time t (s)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(K):
        t += rng.exponential(0.05)
        L = int(rng.integers(20, 201))
        chi = int(rng.choice([16, 32, 64]))
        gamma = float(rng.uniform(0.01, 0.2))
        g = float(rng.uniform(0.0, 1.0))
        N = int(rng.integers(64, 513))
        n = max(1, int(round(rng.uniform(1.0, 5.0) / 0.1)))
        out.append(dict(t=t, L=L, chi_max=chi, gamma=gamma, g=g, n_traj=N, dt=0.1, n_steps=n,
                        T=n * 0.1, seed=SEED + 1000 + i))
    return out
