"""Host logic of bench.py that needs no GPU: the comparison of mixed and
FP64 records that the bench line reports as error_vs_fp64."""
import numpy as np

import bench


def _records(rng, n=8, steps=5, obs=4):
    return {"per_traj": rng.normal(size=(n, steps + 1, obs)), "jumps": np.zeros((n, 2 * steps + 1), np.int32)}


def test_compare_counts_flips_tolerance_horizon_and_ensemble_error():
    rng = np.random.default_rng(0)
    b = _records(rng)
    a = {"per_traj": b["per_traj"].copy(), "jumps": b["jumps"].copy()}
    a["per_traj"][3, 4:, 1] += 1e-3          # trajectory 3 leaves the tolerance at step 4
    a["jumps"][5, 2] = 1                     # trajectory 5 took another jump
    a["per_traj"][5] += 0.5                  # (its records are excluded per trajectory)
    r = bench.compare(a, b)
    assert r["trajectories"] == 8 and r["flipped"] == 1 and r["steps"] == 5
    assert abs(r["max_abs"] - 1e-3) < 1e-12
    assert r["over_tol"] == 1 and r["within_tol_through_step"] == 3
    # the ensemble includes every id, trajectory 5 too
    dm = np.full(b["per_traj"].shape[1:], 0.5 / 8)
    dm[4:, 1] += 1e-3 / 8
    assert abs(r["ensemble_max_abs"] - dm.max()) < 1e-12
    sem = b["per_traj"].std(axis=0, ddof=1) / np.sqrt(8)
    assert abs(r["ensemble_max_over_sem"] - (dm / sem).max()) < 1e-9 * (dm / sem).max()


def test_compare_identical_records():
    rng = np.random.default_rng(1)
    b = _records(rng)
    r = bench.compare({"per_traj": b["per_traj"].copy(), "jumps": b["jumps"].copy()}, b)
    assert r["flipped"] == 0 and r["max_abs"] == 0.0 and r["over_tol"] == 0
    assert r["within_tol_through_step"] == 5 and r["ensemble_max_abs"] == 0.0 and r["ensemble_max_over_sem"] == 0.0
