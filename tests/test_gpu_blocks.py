"""Device building blocks (one workgroup each, the routines the TJM kernel
runs) against independent host references: numpy complex128 products,
numpy/LAPACK QR and SVD, scipy's matrix exponential, the published Philox
known-answer vectors, and the oracle's truncation rule."""
import os

import numpy as np
import pytest
import scipy.linalg as sla

pytestmark = pytest.mark.gpu

from paper_2501_17913_amd import tjm  # noqa: E402
from oracle import mps_tjm  # noqa: E402

RNG = np.random.default_rng(20250117)


def cr(*shape):
    return RNG.normal(size=shape) + 1j * RNG.normal(size=shape)


def _op(X, trans, conj):
    Y = X.T if trans else X
    return Y.conj() if conj else Y


@pytest.mark.parametrize("prec", [tjm.PREC_FP64, tjm.PREC_MIXED])
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (16, 8, 2), (33, 17, 9), (64, 64, 64),
                                   (100, 37, 64), (128, 64, 128),
                                   (64, 128, 64), (128, 64, 64), (100, 200, 37), (200, 100, 70), (64, 256, 64), (256, 64, 64)])
def test_cgemm_plain(prec, M, N, K):
    A, B = cr(M, K), cr(K, N)
    C = tjm.selftest_cgemm(prec, M, N, K, A, B).reshape(M, N)
    ref = A @ B
    tol = 1e-13 if prec == tjm.PREC_FP64 else 2e-6
    assert np.abs(C - ref).max() <= tol * max(1.0, np.abs(A).max() * np.abs(B).max() * K)


@pytest.mark.parametrize("prec", [tjm.PREC_FP64, tjm.PREC_MIXED])
@pytest.mark.parametrize("tA,cA,tB,cB", [(0, 0, 0, 0), (1, 1, 0, 0), (0, 0, 1, 1), (1, 0, 0, 1), (1, 1, 1, 1)])
def test_cgemm_transpose_conjugate(prec, tA, cA, tB, cB):
    M, N, K = 23, 41, 30
    A = cr(K, M) if tA else cr(M, K)
    B = cr(N, K) if tB else cr(K, N)
    C = tjm.selftest_cgemm(prec, M, N, K, A, B, transA=bool(tA), conjA=bool(cA), transB=bool(tB),
                           conjB=bool(cB)).reshape(M, N)
    ref = _op(A, tA, cA) @ _op(B, tB, cB)
    tol = 1e-13 if prec == tjm.PREC_FP64 else 2e-6
    assert np.abs(C - ref).max() <= tol * K * 4


@pytest.mark.parametrize("prec", [tjm.PREC_FP64, tjm.PREC_MIXED])
@pytest.mark.parametrize("sum_batches", [True, False])
@pytest.mark.parametrize("M,N,K", [(19, 24, 13), (64, 128, 40), (128, 64, 40)])
def test_cgemm_batched_and_accumulate(prec, sum_batches, M, N, K):
    nb = 5
    A, B = cr(nb, M, K), cr(nb, K, N)
    C0 = cr(M, N) if sum_batches else cr(nb, M, N)
    C = tjm.selftest_cgemm(prec, M, N, K, A, B, C0=C0, nb=nb, sum_batches=sum_batches, bsA=M * K, bsB=K * N,
                           csC=0 if sum_batches else M * N, accumulate=True)
    if sum_batches:
        ref = C0 + np.einsum('bik,bkj->ij', A, B)
    else:
        ref = C0 + np.einsum('bik,bkj->bij', A, B)
    tol = 1e-13 if prec == tjm.PREC_FP64 else 5e-6
    assert np.abs(C.reshape(ref.shape) - ref).max() <= tol * K * nb * 4


@pytest.mark.parametrize("m,n,r", [(2, 1, 1), (8, 6, 6), (12, 6, 3), (6, 8, 6), (128, 64, 64),
                                   (64, 128, 64), (128, 64, 20), (1, 1, 1), (128, 64, 0), (100, 50, 50),
                                   (3, 64, 3), (128, 1, 1), (127, 63, 63), (128, 128, 100)])
def test_qr(m, n, r):
    X = cr(m, r) @ cr(r, n)
    Q, R = tjm.selftest_qr(X)
    k = min(m, n)
    assert np.abs(Q @ R - X).max() < 1e-13 * max(1, np.abs(X).max()) * m
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() < 1e-13
    assert np.abs(np.tril(R, -1)).max() == 0.0
    d = np.diag(R)
    assert np.all(d.real >= 0) and np.abs(d.imag).max() < 1e-15 * max(1, np.abs(d).max())


def _svd_cases():
    cases = []
    for (m, n, r) in [(8, 6, 6), (6, 8, 6), (12, 8, 4), (128, 128, 128), (128, 64, 64), (64, 128, 40), (1, 5, 1)]:
        cases.append(("random", m, n, r))
    cases += [("zero_rows", 8, 6, 0), ("zero_cols", 6, 8, 0), ("graded", 20, 20, 0), ("degenerate", 16, 16, 0)]
    # working matrices above 64x64 swept in column blocks: ragged last blocks
    # (72 = 4 x 16 + 8 columns), a dummy block (100 columns in blocks of 20),
    # and the exponentially decaying spectra of MPS bonds
    cases += [("random", 128, 72, 72), ("random", 100, 128, 100), ("expdecay", 128, 128, 0),
              ("expdecay", 100, 128, 0)]
    return cases


@pytest.mark.parametrize("kind,m,n,r", _svd_cases())
@pytest.mark.parametrize("absorb", [False, True])
def test_svd(kind, m, n, r, absorb):
    if kind == "random":
        G = cr(m, r) @ cr(r, n)
    elif kind == "zero_rows":
        G = cr(m, n)
        G[m // 2:] = 0
    elif kind == "zero_cols":
        G = cr(m, n)
        G[:, n // 2:] = 0
    elif kind == "graded":
        U0, _ = np.linalg.qr(cr(m, m))
        V0, _ = np.linalg.qr(cr(n, n))
        G = (U0 * np.logspace(0, -10, m)) @ V0.conj().T
    elif kind == "expdecay":
        k0 = min(m, n)
        U0, _ = np.linalg.qr(cr(m, k0))
        V0, _ = np.linalg.qr(cr(n, k0))
        G = (U0 * np.exp(-np.arange(k0) / 6.0)) @ V0.conj().T
    else:
        U0, _ = np.linalg.qr(cr(m, m))
        V0, _ = np.linalg.qr(cr(n, n))
        G = (U0 * np.repeat([1.0, 0.5, 0.25, 0.125], m // 4)) @ V0.conj().T
    left, S, right = tjm.selftest_svd(G, discard=1e-12, cap=1 << 20, absorb_left=absorb)
    s_ref = np.linalg.svd(G, compute_uv=False)
    k = len(S)
    assert k == mps_tjm.truncation_rank(s_ref, 1e-12, 1 << 20, 1e-12)
    assert np.abs(S - s_ref[:k]).max() < 1e-13 * s_ref[0]
    U = left / S[None, :] if absorb else left
    Vh = right if absorb else right / S[:, None]
    # the factor taken from the Jacobi columns is orthonormal to rounding; the
    # other one is recovered by a product with G, accurate to eps * s0 / s_j
    cond_tol = 1e-15 * max(m, n) * s_ref[0] / S[-1]
    eu = np.abs(U.conj().T @ U - np.eye(k)).max()
    ev = np.abs(Vh @ Vh.conj().T - np.eye(k)).max()
    assert (ev if absorb else eu) < 1e-12              # the canonical factor
    assert max(eu, ev) < max(1e-12, cond_tol)
    discarded = np.sqrt(np.sum(s_ref[k:] ** 2))
    assert np.linalg.norm(left @ right - G) <= discarded + 1e-12 * s_ref[0] * max(m, n)


def test_svd_cap_respects_multiplets():
    m = n = 12
    U0, _ = np.linalg.qr(cr(m, m))
    V0, _ = np.linalg.qr(cr(n, n))
    s = np.array([1.0, 0.8, 0.5, 0.5, 0.5, 0.3, 0.2, 0.1, 0.05, 0.02, 0.01, 0.005])
    G = (U0 * s) @ V0.conj().T
    for cap in (1, 3, 4, 5, 6):
        _, S, _ = tjm.selftest_svd(G, cap=cap)
        assert len(S) == mps_tjm.truncation_rank(s, 1e-12, cap, 1e-12)


@pytest.mark.parametrize("n,t", [(1, 0.3), (2, 0.7), (40, 0.05), (40, -0.05), (128, 0.3), (300, 0.1)])
def test_lanczos_expm(n, t):
    A = cr(n, n)
    H = (A + A.conj().T) / 2
    v = cr(n)
    out, it = tjm.selftest_expm(H, v, t, 30, 1e-12)
    ref = sla.expm(-1j * t * H) @ v
    assert np.abs(out - ref).max() < 1e-10 * np.linalg.norm(v)
    assert 1 <= it <= min(30, n)


def test_philox_known_answers_on_device():
    rows = []
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    for r in rows:
        out = tjm.selftest_philox(np.array([r[0:4]], dtype=np.uint32), r[4], r[5])
        assert list(out[0]) == r[6:10]
