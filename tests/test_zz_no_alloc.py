"""The no-allocation SVD entry point (tjm_svd_noalloc) against the entry
point it varies (tjm_selftest_svd): same kernel, caller-owned device
buffers, work arrays in the library's fixed device array.  Two calls in a
row, the second smaller, each bit-identical to the allocating call."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_2501_17913_amd import tjm  # noqa: E402


def _matrix(m, n, seed):
    rng = np.random.default_rng(seed)
    k0 = min(m, n)
    U0, _ = np.linalg.qr(rng.normal(size=(m, k0)) + 1j * rng.normal(size=(m, k0)))
    V0, _ = np.linalg.qr(rng.normal(size=(n, k0)) + 1j * rng.normal(size=(n, k0)))
    s = np.exp(-np.arange(k0) / 5.0)
    return (U0 * s) @ V0.conj().T


def _noalloc(G, discard, cap, deg_tol, absorb):
    m, n = G.shape
    kmax = min(m, n)
    dev = torch.device("cuda", 0)
    dG = torch.from_numpy(np.ascontiguousarray(G).view(np.float64).reshape(-1).copy()).to(dev)
    dleft = torch.full((2 * m * kmax,), np.nan, dtype=torch.float64, device=dev)
    dright = torch.full((2 * kmax * n,), np.nan, dtype=torch.float64, device=dev)
    dS = torch.full((kmax,), np.nan, dtype=torch.float64, device=dev)
    dk = torch.zeros(1, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()
    st = tjm.lib.tjm_svd_noalloc(m, n, C.c_void_p(dG.data_ptr()), discard, cap, deg_tol, int(absorb),
                                 C.c_void_p(dleft.data_ptr()), C.c_void_p(dright.data_ptr()),
                                 C.c_void_p(dS.data_ptr()), C.c_void_p(dk.data_ptr()), None)
    assert st == tjm.OK, tjm.lib.tjm_last_error(None)
    torch.cuda.synchronize()
    k = int(dk.cpu().item())
    left = dleft.cpu().numpy()[:2 * m * k].view(np.complex128).reshape(m, k)
    right = dright.cpu().numpy()[:2 * k * n].view(np.complex128).reshape(k, n)
    return left, dS.cpu().numpy()[:k], right


def test_svd_noalloc_equals_allocating_entry_point():
    # the first call is the largest the fixed work arrays admit on the
    # rotated side (128 columns), the second is smaller
    for (m, n, absorb, seed) in [(256, 128, False, 11), (40, 24, True, 12)]:
        G = _matrix(m, n, seed)
        l_ref, s_ref, r_ref = tjm.selftest_svd(G, discard=1e-12, cap=1 << 20, deg_tol=1e-12, absorb_left=absorb)
        left, S, right = _noalloc(G, 1e-12, 1 << 20, 1e-12, absorb)
        print("m=%d n=%d absorb=%d: kept %d" % (m, n, absorb, len(S)), flush=True)
        assert len(S) == len(s_ref)
        assert np.array_equal(S, s_ref)
        assert np.array_equal(left, l_ref)
        assert np.array_equal(right, r_ref)


def test_svd_noalloc_rejects_sizes_beyond_its_work_arrays():
    st = tjm.lib.tjm_svd_noalloc(300, 8, C.c_void_p(1), 1e-12, 4, 1e-12, 0, C.c_void_p(1), C.c_void_p(1),
                                 C.c_void_p(1), C.c_void_p(1), None)
    assert st == tjm.E_INVAL
    assert b"256" in tjm.lib.tjm_last_error(None)
