"""The no-allocation SVD entry point (tjm_svd_noalloc) against the entry
point it varies (tjm_selftest_svd): same kernel, caller-owned device
buffers, work arrays in the library's fixed device array.  Two calls in a
row, the second smaller, each bit-identical to the allocating call."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

from paper_2501_17913_amd import tjm  # noqa: E402

# Device buffers come from the HIP runtime the library itself links (loaded
# by soname, so this is the same copy): a second runtime in the process
# (for example the one a framework bundles) would not share its devices.
_hip = C.CDLL("libamdhip64.so.7")
_hip.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
_hip.hipFree.argtypes = [C.c_void_p]
_hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
_hip.hipDeviceSynchronize.argtypes = []
_H2D, _D2H = 1, 2


class _Dev:
    """A device buffer holding a copy of a host array (or n bytes of NaN)."""

    def __init__(self, host):
        self.host = np.ascontiguousarray(host)
        self.p = C.c_void_p()
        assert _hip.hipMalloc(C.byref(self.p), max(self.host.nbytes, 16)) == 0
        assert _hip.hipMemcpy(self.p, self.host.ctypes.data, self.host.nbytes, _H2D) == 0

    def get(self):
        out = np.empty_like(self.host)
        assert _hip.hipMemcpy(out.ctypes.data, self.p, out.nbytes, _D2H) == 0
        return out

    def free(self):
        _hip.hipFree(self.p)


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
    bufs = [_Dev(np.ascontiguousarray(G, np.complex128).view(np.float64)),
            _Dev(np.full(2 * m * kmax, np.nan)), _Dev(np.full(2 * kmax * n, np.nan)),
            _Dev(np.full(kmax, np.nan)), _Dev(np.zeros(1, np.int32))]
    dG, dleft, dright, dS, dk = bufs
    assert _hip.hipDeviceSynchronize() == 0
    st = tjm.lib.tjm_svd_noalloc(m, n, dG.p, discard, cap, deg_tol, int(absorb), dleft.p, dright.p, dS.p, dk.p,
                                 None)
    assert st == tjm.OK, tjm.lib.tjm_last_error(None)
    assert _hip.hipDeviceSynchronize() == 0
    k = int(dk.get()[0])
    left = dleft.get()[:2 * m * k].view(np.complex128).reshape(m, k)
    right = dright.get()[:2 * k * n].view(np.complex128).reshape(k, n)
    S = dS.get()[:k]
    for b in bufs:
        b.free()
    return left, S, right


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
