"""Oracle trajectories computed in worker processes, for the GPU parity tests.

The workers are spawned (not forked from a process that may hold a GPU
context), import only the oracle and the input recipes, run single-threaded
BLAS, and never touch the GPU."""
import multiprocessing as mp
import os

_BLAS_VARS = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")


def _one(args):
    L, chi, cap, init, n, g, gamma, seed, t = args
    import numpy as np
    from oracle import model as om, mps_tjm
    from tests import inputs
    Ws = om.xxx_mpo(L, 1.0, g)
    jumps = om.relax_dephase_jumps(L, gamma, gamma)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, inputs.init_bits(L, init))
    rec = {}
    out = mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, n, obs, seed, t,
                                 mps_tjm.Options(chi_max=chi, chi_cap=cap), rec)
    return out, [m for (_, _, m) in rec["jumps"]], np.array(rec["bonds"])


def _one_domain_wall(args):
    L, chi, n, seed, t = args
    import numpy as np
    from oracle import model as om, mps_tjm
    Ws = om.xxx_mpo(L, 1.0, 0.0, 1.0)
    jumps = om.relax_excite_jumps(L, 0.1, 0.1)
    obs = [(q, om.Z) for q in range(L)] + [(q, om.X) for q in range(L)]
    sv = om.product_site_vectors(L, om.domain_wall_bits(L))
    rec = {}
    out = mps_tjm.run_trajectory(Ws, jumps, mps_tjm.product_mps(sv), 0.1, n, obs, seed, t,
                                 mps_tjm.Options(chi_max=chi), rec)
    return out, [m for (_, _, m) in rec["jumps"]], np.array(rec["bonds"])


def workers(n_tasks, cap=16):
    """Worker count: at most `cap` (the host cores one GPU is given) and the host's cores."""
    return max(1, min(n_tasks, cap, os.cpu_count() or 1))


def _pool_map(fn, tasks):
    saved = {v: os.environ.get(v) for v in _BLAS_VARS}
    for v in _BLAS_VARS:
        os.environ[v] = "1"
    try:
        with mp.get_context("spawn").Pool(workers(len(tasks))) as pool:
            return pool.map(fn, tasks, chunksize=1)
    finally:
        for v, x in saved.items():
            if x is None:
                os.environ.pop(v, None)
            else:
                os.environ[v] = x


def oracle_trajectories(L, chi, init, n, g, gamma, seed, ids, chi_cap=None):
    """{trajectory id: (observables [n+1][2L], jump log, bond log)} for the
    XXX chain with sigma- and Z jumps, observables Z then X on every site."""
    ids = list(ids)
    res = _pool_map(_one, [(L, chi, chi_cap, init, n, g, gamma, seed, t) for t in ids])
    return dict(zip(ids, res))


def domain_wall_trajectories(L, chi, n, seed, ids):
    """The same for the 30-site comparison chain: XXX with a Z field h = 1,
    sigma_minus and sigma_plus at 0.1 on every site, domain-wall start."""
    ids = list(ids)
    res = _pool_map(_one_domain_wall, [(L, chi, n, seed, t) for t in ids])
    return dict(zip(ids, res))
