"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol the headers declare, and rejects bad arguments with the status
codes include/tjm.h documents (validation precedes any device call)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2501_17913_amd", "libtjm.so")


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_2501_17913_amd import build
        build.build()


_ensure_built()
from paper_2501_17913_amd import models, tjm  # noqa: E402


def _declared():
    names = set()
    for h in ("tjm.h", "tjm_selftest.h"):
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names |= set(re.findall(r"\b(tjm_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    decl = _declared()
    assert "tjm_run" in decl and "tjm_selftest_cgemm" in decl
    for name in decl:
        assert hasattr(lib, name), name
    assert decl == set(tjm.EXPORTED)


def _create(L=3, d=2, bonds=None, mpo=None, sites=None, ops=None, rates=None):
    W = models.xxx_mpo(L, 1.0, 0.5) if mpo is None else mpo
    flat = np.concatenate([w.reshape(-1) for w in W]).astype(np.complex128)
    b = np.array([1] + [w.shape[3] for w in W], dtype=np.int32) if bonds is None else np.asarray(bonds, np.int32)
    s, o, r = models.relaxation_dephasing(L, 0.1, 0.1)
    s = s if sites is None else np.asarray(sites, np.int32)
    o = o if ops is None else ops
    r = r if rates is None else np.asarray(rates, np.float64)
    oo = np.ascontiguousarray(np.asarray(o, np.complex128).reshape(-1))
    h = C.c_void_p()
    st = tjm.lib.tjm_create(C.byref(h), L, d, b.ctypes.data_as(tjm._ip), flat.view(np.float64).ctypes.data_as(tjm._dp),
                            len(s), s.ctypes.data_as(tjm._ip), oo.view(np.float64).ctypes.data_as(tjm._dp),
                            r.ctypes.data_as(tjm._dp))
    return st, h


def test_create_accepts_valid_model_and_destroys():
    st, h = _create()
    assert st == tjm.OK and h.value
    tjm.lib.tjm_destroy(h)
    tjm.lib.tjm_destroy(None)


@pytest.mark.parametrize("case,expect", [
    ("L0", tjm.E_INVAL), ("d3", tjm.E_UNSUPPORTED), ("boundary", tjm.E_INVAL),
    ("rate", tjm.E_INVAL), ("nan_mpo", tjm.E_INVAL), ("site", tjm.E_INVAL), ("nan_rate", tjm.E_INVAL)])
def test_create_rejects_bad_models(case, expect):
    L = 3
    kw = {}
    if case == "L0":
        st, h = _create(L=3)
        tjm.lib.tjm_destroy(h)
        hh = C.c_void_p()
        b = np.array([1], np.int32)
        z = np.zeros(8)
        st = tjm.lib.tjm_create(C.byref(hh), 0, 2, b.ctypes.data_as(tjm._ip), z.ctypes.data_as(tjm._dp), 0, None, None, None)
        assert st == expect and not hh.value
        assert tjm.lib.tjm_last_error(None)
        return
    if case == "d3":
        st, h = _create(d=3)
    elif case == "boundary":
        W = models.xxx_mpo(L)
        st, h = _create(bonds=[5] + [w.shape[3] for w in W])
    elif case == "rate":
        st, h = _create(rates=[0.1, -0.1] * L)
    elif case == "nan_rate":
        st, h = _create(rates=[0.1, np.nan] * L)
    elif case == "nan_mpo":
        W = models.xxx_mpo(L)
        W[1] = W[1].copy()
        W[1][0, 0, 0, 0] = np.nan
        st, h = _create(mpo=W)
    else:
        s, _, _ = models.relaxation_dephasing(L, 0.1, 0.1)
        s = s.copy()
        s[3] = L
        st, h = _create(sites=s)
    assert st == expect
    assert not h.value
    assert len(tjm.lib.tjm_last_error(None)) > 0


def _model(L=4):
    mpo, s, o, r = models.xxx_model(L, 1.0, 0.5, 0.1)
    return tjm.Model(L, mpo, s, o, r)


def test_initial_product_validation():
    m = _model()
    with pytest.raises(tjm.TjmError) as e:
        m.set_initial_product(np.zeros((4, 2)))
    assert e.value.status == tjm.E_INVAL
    v = models.neel(4).copy()
    v[1, 0] = np.nan
    with pytest.raises(tjm.TjmError):
        m.set_initial_product(v)
    m.set_initial_product(models.neel(4))


def test_initial_mps_validation():
    m = _model()
    rng = np.random.default_rng(7)
    good = [rng.normal(size=(2, a, b)) + 0j for a, b in [(1, 2), (2, 4), (4, 2), (2, 1)]]
    m.set_initial_mps(good)
    with pytest.raises(tjm.TjmError) as e:                 # right boundary bond must be 1
        m.set_initial_mps(good[:3] + [rng.normal(size=(2, 2, 2)) + 0j])
    assert e.value.status == tjm.E_INVAL
    bad = [t.copy() for t in good]
    bad[2][0, 0, 0] = np.inf
    with pytest.raises(tjm.TjmError) as e:
        m.set_initial_mps(bad)
    assert e.value.status == tjm.E_INVAL
    with pytest.raises(ValueError):
        m.set_initial_mps(good[:3])
    m.set_initial_product(models.neel(4))                 # back to a product state


@pytest.mark.parametrize("kw,expect", [
    (dict(n_traj=0), tjm.E_INVAL), (dict(dt=0.0), tjm.E_INVAL), (dict(T=0.25), tjm.E_INVAL),
    (dict(chi_max=0), tjm.E_INVAL), (dict(obs_site=9), tjm.E_INVAL),
    (dict(opt=dict(chi_cap=128)), tjm.E_UNSUPPORTED), (dict(opt=dict(krylov_max=40)), tjm.E_INVAL),
    (dict(opt=dict(precision=7)), tjm.E_INVAL), (dict(opt=dict(sweep_jumps=0)), tjm.E_UNSUPPORTED),
    (dict(opt=dict(trotter_order=3)), tjm.E_INVAL), (dict(opt=dict(trotter_order=0)), tjm.E_INVAL),
    (dict(opt=dict(tile_mode=8)), tjm.E_INVAL), (dict(opt=dict(tile_mode=-1)), tjm.E_INVAL)])
def test_run_rejects_bad_arguments_before_touching_the_device(kw, expect):
    m = _model()
    args = dict(n_traj=4, dt=0.1, T=0.3, chi_max=4, obs_site=0)
    args.update({k: v for k, v in kw.items() if k != "opt"})
    opt = tjm.default_options(**kw.get("opt", {}))
    obs = [(args["obs_site"], models.PAULI_Z)]
    with pytest.raises(tjm.TjmError) as e:
        m.run(args["n_traj"], args["dt"], args["T"], args["chi_max"], obs, 1, opt)
    assert e.value.status == expect


@pytest.mark.parametrize("kw", [dict(warm_steps=2, timed_steps=2), dict(warm_steps=-1), dict(timed_steps=0),
                                dict(n_traj=0), dict(chi_max=0), dict(opt=dict(tile_mode=9))])
def test_autotune_rejects_bad_arguments_before_touching_the_device(kw):
    # a 3-step run (T = 0.3): warm_steps + timed_steps must stay within it
    m = _model()
    args = dict(n_traj=4, chi_max=4, warm_steps=1, timed_steps=1)
    args.update({k: v for k, v in kw.items() if k != "opt"})
    opt = tjm.default_options(**kw.get("opt", {}))
    with pytest.raises(tjm.TjmError) as e:
        m.autotune(args["n_traj"], 0.1, 0.3, args["chi_max"], [(0, models.PAULI_Z)], 1, opt,
                   warm_steps=args["warm_steps"], timed_steps=args["timed_steps"])
    assert e.value.status == tjm.E_INVAL


def test_session_calls_out_of_order_are_busy():
    m = _model()
    with pytest.raises(tjm.TjmError) as e:
        m.advance(1)
    assert e.value.status == tjm.E_BUSY
    st = tjm.lib.tjm_run_end(m.h, None, None, None, None, None)
    assert st == tjm.E_BUSY


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_valid_run_without_gpu_reports_device_error():
    m = _model()
    with pytest.raises(tjm.TjmError) as e:
        m.run(2, 0.1, 0.2, 4, [(0, models.PAULI_Z)], 1)
    assert e.value.status == tjm.E_DEVICE


def test_package_mpo_matches_oracle_hamiltonian():
    from oracle import model as om
    for L in (1, 2, 4):
        for (J, hx, hz) in [(1.0, 0.5, 0.0), (0.3, 0.0, 0.8)]:
            H = om.mpo_to_dense(models.xxx_mpo(L, J, hx, hz))
            assert np.abs(H - om.xxx_dense(L, J, hx, hz)).max() < 1e-13
    H = om.mpo_to_dense(models.tfim_mpo(3, 1.0, 0.7))
    assert np.abs(H - om.tfim_dense(3, 1.0, 0.7)).max() < 1e-13


def test_server_calls_reject_null_arguments():
    """The serving entry points validate their pointers before any device
    work."""
    job = C.c_uint64()
    assert tjm.lib.tjm_server_create(None, 0, 0) == tjm.E_INVAL
    assert tjm.lib.tjm_submit(None, None, None, C.byref(job)) == tjm.E_INVAL
    assert tjm.lib.tjm_server_last_error().decode() == "NULL argument"
    done = C.c_int()
    assert tjm.lib.tjm_poll(None, 1, C.byref(done)) == tjm.E_INVAL
    assert tjm.lib.tjm_wait(None, 1, None, None, None) == tjm.E_INVAL
    assert tjm.lib.tjm_server_reserve(None, None, None) == tjm.E_INVAL
    traj, steps = C.c_int(), C.c_ulonglong()
    assert tjm.lib.tjm_job_progress(None, 1, C.byref(traj), C.byref(steps)) == tjm.E_INVAL
    tjm.lib.tjm_server_destroy(None)
    h = C.c_void_p()
    assert tjm.lib.tjm_server_create(C.byref(h), -1, 0) in (tjm.E_INVAL, tjm.E_DEVICE)
    assert not h.value


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path")
def test_server_without_gpu_reports_device_error():
    with pytest.raises(tjm.TjmError) as e:
        tjm.Server(0)
    assert e.value.status == tjm.E_DEVICE


def test_serving_stream_recipe():
    """The serving stream's requests follow the stated recipe and are
    reproducible: every parameter in range, T an exact multiple of dt."""
    from tests import inputs
    a = inputs.serving_stream(200)
    assert a == inputs.serving_stream(200)
    t = np.array([q["t"] for q in a])
    assert np.all(np.diff(t) > 0) and 0.03 < t[-1] / len(a) < 0.07
    for q in a:
        assert 20 <= q["L"] <= 200 and q["chi_max"] in (16, 32, 64) and 64 <= q["n_traj"] <= 512
        assert 0.01 <= q["gamma"] <= 0.2 and 0.0 <= q["g"] <= 1.0
        assert 10 <= q["n_steps"] <= 50 and abs(q["T"] / q["dt"] - q["n_steps"]) < 1e-9
    assert len({q["seed"] for q in a}) == len(a)


def test_svd_noalloc_validates_before_touching_the_device():
    import ctypes as C
    bogus = C.c_void_p(1)          # never dereferenced: the sizes are rejected first
    for (m, n, absorb) in [(300, 8, 0), (8, 200, 0), (200, 8, 1), (0, 4, 0)]:
        st = tjm.lib.tjm_svd_noalloc(m, n, bogus, 1e-12, 4, 1e-12, absorb, bogus, bogus, bogus, bogus, None)
        assert st == tjm.E_INVAL, (m, n, absorb)
    assert tjm.lib.tjm_svd_noalloc(8, 8, None, 1e-12, 4, 1e-12, 0, None, None, None, None, None) == tjm.E_INVAL


def test_mpo_observable_registration_validation():
    m = _model()
    L = m.L
    good = models.xxx_mpo(L, 1.0, 0.5)
    assert m.add_mpo_observable(good) == 0
    xx = [np.eye(2, dtype=np.complex128).reshape(2, 2, 1, 1) for _ in range(L)]
    assert m.add_mpo_observable(xx) == 1 and m.n_mpo_obs == 2
    # boundary bond, bond range and non-finite entries are rejected
    bad = [W.copy() for W in good]
    bad[-1] = np.zeros((2, 2, 5, 2), dtype=np.complex128)      # right boundary bond 2
    with pytest.raises(tjm.TjmError) as e:
        m.add_mpo_observable(bad)
    assert e.value.status == tjm.E_INVAL
    with pytest.raises(ValueError):                             # inconsistent neighbouring bonds
        m.add_mpo_observable([good[0][:, :, :, :2]] + good[1:])
    nan = [W.copy() for W in good]
    nan[1][0, 0, 0, 0] = np.nan
    with pytest.raises(tjm.TjmError) as e:
        m.add_mpo_observable(nan)
    assert e.value.status == tjm.E_INVAL
    assert m.n_mpo_obs == 2
    m.clear_mpo_observables()
    assert m.n_mpo_obs == 0
    assert tjm.lib.tjm_add_mpo_observable(None, None, None, None) == tjm.E_INVAL
    assert tjm.lib.tjm_clear_mpo_observables(None) == tjm.E_INVAL
