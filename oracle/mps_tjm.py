"""CPU MPS tensor jump method, FP64 (oracle O3).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's Sec. "Tensor jump method" step by step:
  * schedule of the sampling MPS: Eq. (TimeEvolutionFunctions), Eq.
    (SimulationStep) and Sec. "Algorithm";
  * dynamic TDVP U[dt]: Sec. "Dynamic TDVP", Eqs. (1TDVP_ForwardEvolving),
    (1TDVP_BackwardEvolving), (2TDVP_ForwardEvolving), Sec. "Hybrid strategy";
  * dissipative contraction D[dt]: Sec. "Dissipative contraction", Eq.
    (DissipativeMPO);
  * jump process J: Sec. "Stochastic jump process".
Layouts are the paper's: M[s, a_left, a_right] (Methods, MPS), W[s_out, s_in,
w_left, w_right] (Methods, MPO).  Environments are Lenv[a_bra, w, a_ket] and
Renv[b_bra, w, b_ket].

Readings of points where the paper is silent or inconsistent (each also
listed in the design notes of the repository):
  R1  each half-sweep evolves by tau = dt/2 (second-order symmetric sweep);
  R2  the 1TDVP/2TDVP switch is local: bond l uses 2TDVP iff chi_l < chi_max
      at the moment the sweep reaches it;
  R3  SVD truncation keeps the smallest k with discarded weight
      sum_{i>=k} s_i^2 <= svd_discard * sum s_i^2 (k >= 1), capped at chi_cap;
      when the cap cuts a multiplet (s_{k-1} - s_k <= deg_tol * s_0) k is
      lowered until it does not;
  R4  Lanczos: full re-orthogonalisation (one classical Gram-Schmidt pass),
      stop when beta_j |[exp(-i t T)]_{j,0}| <= tol or at krylov_max;
  R5  the turning unit of a sweep is evolved again (no merging);
  R6  the jump distribution is normalised by its own sum (the printed Pi_m
      does not sum to one with an exact delta p); candidates in site-major
      order, operators in input order; the first index whose running sum
      exceeds r * W is taken;
  R7  "normalised through successive SVDs": an SVD-truncation sweep from the
      jump site to the right end, then from the right end to site 1;
  R8  at most one jump per jump process;
  R9  the sampling layer uses its own draws;
  R10 t = 0 observables are measured on Psi(0).
  R19 the first-order variant of Sec. "Higher-order Trotterization" (the
      baseline splitting e^{-i H_D dt} e^{-i H_0 dt}): no F_0, every step
      F_k = J D[dt] U[dt] with the main draws of step k, measured on its
      result (no separate sampling layer).
"""
import numpy as np

from . import model, philox


class Options:
    def __init__(self, chi_max, chi_cap=None, svd_discard=1e-12, krylov_max=30,
                 krylov_tol=1e-12, deg_tol=1e-12):
        self.chi_max = int(chi_max)
        self.chi_cap = int(chi_max if chi_cap is None else chi_cap)
        self.svd_discard = float(svd_discard)
        self.krylov_max = int(krylov_max)
        self.krylov_tol = float(krylov_tol)
        self.deg_tol = float(deg_tol)


class Stats:
    def __init__(self):
        self.krylov_calls = 0
        self.krylov_iters = 0
        self.two_site = 0
        self.one_site = 0


# --------------------------------------------------------------------------
# Lanczos matrix exponential (Sec. "Hybrid strategy")
# --------------------------------------------------------------------------

def expm_krylov(apply_h, v, t, m_max, tol, stats=None):
    """exp(-i t H) v for Hermitian H given as a matrix-free product (R4)."""
    shape = v.shape
    v = v.reshape(-1)
    beta0 = np.linalg.norm(v)
    if beta0 == 0.0:
        return v.reshape(shape).copy()
    m_max = min(m_max, v.size)
    Q = [v / beta0]
    alpha, beta = [], []
    for j in range(m_max):
        w = apply_h(Q[j].reshape(shape)).reshape(-1)
        a = np.real(np.vdot(Q[j], w))
        alpha.append(a)
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[j - 1] * Q[j - 1]
        Qm = np.array(Q)                      # (j+1, n)
        w = w - Qm.T @ (Qm.conj() @ w)        # full re-orthogonalisation
        b = np.linalg.norm(w)
        T = np.diag(alpha) + np.diag(beta, 1) + np.diag(beta, -1)
        lam, Zv = np.linalg.eigh(T)
        c = Zv @ (np.exp(-1j * t * lam) * Zv[0, :])
        if b * abs(c[j]) <= tol or j == m_max - 1:
            if stats is not None:
                stats.krylov_calls += 1
                stats.krylov_iters += j + 1
            return (beta0 * (Qm.T @ c)).reshape(shape)
        beta.append(b)
        Q.append(w / b)


# --------------------------------------------------------------------------
# Effective Hamiltonians and environments (Fig. TDVP, Sec. "Hybrid strategy")
# --------------------------------------------------------------------------

def left_update(Lenv, A, W):
    """L_l[b', w', b] = sum L_{l-1}[a', w, a] conj(A[s', a', b']) W[s', s, w, w'] A[s, a, b]."""
    T = np.tensordot(Lenv, A, axes=([2], [1]))               # [a', w, s, b]
    T = np.tensordot(T, W, axes=([1, 2], [2, 1]))            # [a', b, s', w']
    T = np.tensordot(A.conj(), T, axes=([0, 1], [2, 0]))     # [b', b, w']
    return T.transpose(0, 2, 1)


def right_update(Renv, B, W):
    """R_{l-1}[a', w, a] = sum conj(B[s', a', b']) W[s', s, w, w'] B[s, a, b] R_l[b', w', b]."""
    T = np.tensordot(B, Renv, axes=([2], [2]))               # [s, a, b', w']
    T = np.tensordot(T, W, axes=([0, 3], [1, 3]))            # [a, b', s', w]
    T = np.tensordot(B.conj(), T, axes=([0, 2], [2, 1]))     # [a', a, w]
    return T.transpose(0, 2, 1)


def h1_apply(Lenv, W, Renv, M):
    """One-site H^eff_l applied to M (degree-6 network of Fig. TDVP):
    y[s', a', b'] = sum L[a', w, a] W[s', s, w, w'] M[s, a, b] R[b', w', b]."""
    T = np.tensordot(Lenv, M, axes=([2], [1]))               # [a', w, s, b]
    T = np.tensordot(T, W, axes=([1, 2], [2, 1]))            # [a', b, s', w']
    T = np.tensordot(T, Renv, axes=([1, 3], [2, 1]))         # [a', s', b']
    return T.transpose(1, 0, 2)


def h0_apply(Lenv, Renv, C):
    """Bond H~^eff_l applied to the bond tensor C (degree-4 network):
    y[b', c'] = sum L[b', w, b] C[b, c] R[c', w, c]."""
    T = np.tensordot(Lenv, C, axes=([2], [0]))               # [b', w, c]
    return np.tensordot(T, Renv, axes=([1, 2], [1, 2]))      # [b', c']


def h2_apply(Lenv, W1, W2, Renv, theta):
    """Two-site H^eff_{l,l+1} applied to theta[s1, s2, a, c] (degree-8 network):
    y[p, q, a', c'] = sum L[a', w, a] W1[p, s1, w, u] W2[q, s2, u, v] theta[s1, s2, a, c] R[c', v, c]."""
    T = np.tensordot(Lenv, theta, axes=([2], [2]))           # [a', w, s1, s2, c]
    T = np.tensordot(T, W1, axes=([1, 2], [2, 1]))           # [a', s2, c, p, u]
    T = np.tensordot(T, W2, axes=([1, 4], [1, 2]))           # [a', c, p, q, v]
    T = np.tensordot(T, Renv, axes=([1, 4], [2, 1]))         # [a', p, q, c']
    return T.transpose(1, 2, 0, 3)


# --------------------------------------------------------------------------
# Factorisations
# --------------------------------------------------------------------------

def qr_left(M):
    """M[s,a,b] as the (s a) x b matrix = A C with A left-canonical."""
    d, a, b = M.shape
    Q, R = np.linalg.qr(M.reshape(d * a, b))
    return Q.reshape(d, a, Q.shape[1]), R


def lq_right(M):
    """M[s,a,b] as the a x (s b) matrix = C B with B right-canonical."""
    d, a, b = M.shape
    mat = M.transpose(1, 0, 2).reshape(a, d * b)
    Q, R = np.linalg.qr(mat.conj().T)
    k = Q.shape[1]
    B = Q.conj().T.reshape(k, d, b).transpose(1, 0, 2)
    return R.conj().T, B


def truncation_rank(s, discard, cap, deg_tol):
    """Kept rank under reading R3 (s sorted non-increasing)."""
    n = len(s)
    s2 = s * s
    total = np.sum(s2)
    tail = np.zeros(n + 1)
    for i in range(n - 1, -1, -1):            # tail[k] = sum_{i >= k} s_i^2
        tail[i] = tail[i + 1] + s2[i]
    k = n
    for kk in range(1, n + 1):
        if tail[kk] <= discard * total:
            k = kk
            break
    if k > cap:
        k = cap
        while k > 1 and s[k - 1] - s[k] <= deg_tol * s[0]:
            k -= 1
    return max(k, 1)


def svd_split(mat, opt):
    U, S, Vh = np.linalg.svd(mat, full_matrices=False)
    k = truncation_rank(S, opt.svd_discard, opt.chi_cap, opt.deg_tol)
    return U[:, :k], S[:k], Vh[:k, :]


def theta_split_left(theta, opt):
    """theta[s1,s2,a,c] -> A[s1,a,k] (left-canonical), M[s2,k,c] = S V^dag."""
    d1, d2, a, c = theta.shape
    U, S, Vh = svd_split(theta.transpose(0, 2, 1, 3).reshape(d1 * a, d2 * c), opt)
    k = len(S)
    A = U.reshape(d1, a, k)
    M = (S[:, None] * Vh).reshape(k, d2, c).transpose(1, 0, 2)
    return A, M


def theta_split_right(theta, opt):
    """theta -> M[s1,a,k] = U S, B[s2,k,c] (right-canonical)."""
    d1, d2, a, c = theta.shape
    U, S, Vh = svd_split(theta.transpose(0, 2, 1, 3).reshape(d1 * a, d2 * c), opt)
    k = len(S)
    M = (U * S[None, :]).reshape(d1, a, k)
    B = Vh.reshape(k, d2, c).transpose(1, 0, 2)
    return M, B


def absorb_right(C, M):
    return np.einsum('ac,scb->sab', C, M)


def absorb_left(M, C):
    return np.einsum('sac,cb->sab', M, C)


# --------------------------------------------------------------------------
# Dynamic TDVP U[dt] (Sec. "Dynamic TDVP")
# --------------------------------------------------------------------------

def tdvp_step(mps, Ws, dt, opt, stats):
    """One U[dt]: an L->R and an R->L half-sweep of tau = dt/2 each (R1).

    Precondition: centre at site 0, all other sites right-canonical."""
    L = len(mps)
    tau = 0.5 * dt
    one = np.ones((1, 1, 1), dtype=np.complex128)
    Lenv = [None] * (L + 1)
    Renv = [None] * (L + 1)
    Lenv[0] = one
    Renv[L] = one
    for s in range(L - 1, 0, -1):
        Renv[s] = right_update(Renv[s + 1], mps[s], Ws[s])
    km, kt = opt.krylov_max, opt.krylov_tol

    def ex(fn, v, t):
        return expm_krylov(fn, v, t, km, kt, stats)

    # left-to-right half-sweep
    last_two = False
    for s in range(L - 1):
        if mps[s].shape[2] < opt.chi_max:                  # R2: 2TDVP on (s, s+1)
            stats.two_site += 1
            theta = np.einsum('sab,tbc->stac', mps[s], mps[s + 1])
            Le, W1, W2, Re = Lenv[s], Ws[s], Ws[s + 1], Renv[s + 2]
            theta = ex(lambda v: h2_apply(Le, W1, W2, Re, v), theta, tau)
            A, M = theta_split_left(theta, opt)
            mps[s], mps[s + 1] = A, M
            Lenv[s + 1] = left_update(Lenv[s], A, Ws[s])
            if s + 1 < L - 1:
                Le2, W, Re2 = Lenv[s + 1], Ws[s + 1], Renv[s + 2]
                mps[s + 1] = ex(lambda v: h1_apply(Le2, W, Re2, v), mps[s + 1], -tau)
            last_two = True
        else:                                              # 1TDVP at s, bond s+1
            stats.one_site += 1
            Le, W, Re = Lenv[s], Ws[s], Renv[s + 1]
            mps[s] = ex(lambda v: h1_apply(Le, W, Re, v), mps[s], tau)
            A, C = qr_left(mps[s])
            mps[s] = A
            Lenv[s + 1] = left_update(Lenv[s], A, Ws[s])
            Lb, Rb = Lenv[s + 1], Renv[s + 1]
            C = ex(lambda v: h0_apply(Lb, Rb, v), C, -tau)
            mps[s + 1] = absorb_right(C, mps[s + 1])
            last_two = False
    if L == 1 or not last_two:
        Le, W, Re = Lenv[L - 1], Ws[L - 1], Renv[L]
        mps[L - 1] = ex(lambda v: h1_apply(Le, W, Re, v), mps[L - 1], tau)

    # right-to-left half-sweep (R5: the turning unit is evolved again)
    last_two = False
    for s in range(L - 1, 0, -1):
        if mps[s].shape[1] < opt.chi_max:                  # 2TDVP on (s-1, s)
            stats.two_site += 1
            theta = np.einsum('sab,tbc->stac', mps[s - 1], mps[s])
            Le, W1, W2, Re = Lenv[s - 1], Ws[s - 1], Ws[s], Renv[s + 1]
            theta = ex(lambda v: h2_apply(Le, W1, W2, Re, v), theta, tau)
            M, B = theta_split_right(theta, opt)
            mps[s - 1], mps[s] = M, B
            Renv[s] = right_update(Renv[s + 1], B, Ws[s])
            if s - 1 > 0:
                Le2, W, Re2 = Lenv[s - 1], Ws[s - 1], Renv[s]
                mps[s - 1] = ex(lambda v: h1_apply(Le2, W, Re2, v), mps[s - 1], -tau)
            last_two = True
        else:                                              # 1TDVP at s, bond s
            stats.one_site += 1
            Le, W, Re = Lenv[s], Ws[s], Renv[s + 1]
            mps[s] = ex(lambda v: h1_apply(Le, W, Re, v), mps[s], tau)
            C, B = lq_right(mps[s])
            mps[s] = B
            Renv[s] = right_update(Renv[s + 1], B, Ws[s])
            Lb, Rb = Lenv[s], Renv[s]
            C = ex(lambda v: h0_apply(Lb, Rb, v), C, -tau)
            mps[s - 1] = absorb_left(mps[s - 1], C)
            last_two = False
    if L == 1 or not last_two:
        Le, W, Re = Lenv[0], Ws[0], Renv[1]
        mps[0] = ex(lambda v: h1_apply(Le, W, Re, v), mps[0], tau)


# --------------------------------------------------------------------------
# Dissipation and jump process (Secs. "Dissipative contraction",
# "Stochastic jump process")
# --------------------------------------------------------------------------

def dissipate(mps, Dloc):
    for s in range(len(mps)):
        mps[s] = np.einsum('st,tab->sab', Dloc[s], mps[s])


def sweep_qr_right(mps, start, stop):
    """Move the centre from `start` to `stop` (> start) with QR."""
    for s in range(start, stop):
        A, C = qr_left(mps[s])
        mps[s] = A
        mps[s + 1] = absorb_right(C, mps[s + 1])


def sweep_lq_left(mps, start, stop):
    """Move the centre from `start` to `stop` (< start) with LQ."""
    for s in range(start, stop, -1):
        C, B = lq_right(mps[s])
        mps[s] = B
        mps[s - 1] = absorb_left(mps[s - 1], C)


def jump_process(mps, jumps, eps, r, opt):
    """J_eps acting on an (unnormalised) MPS with centre at site 0.

    Returns (index of the applied jump or -1, delta p).  On return the MPS is
    normalised with its centre at site 0."""
    L = len(mps)
    sweep_qr_right(mps, 0, L - 1)
    norm2 = np.real(np.vdot(mps[L - 1], mps[L - 1]))
    dp = max(0.0, 1.0 - norm2)
    if eps >= dp:                                     # no jump: normalise
        mps[L - 1] = mps[L - 1] / np.sqrt(norm2)
        sweep_lq_left(mps, L - 1, 0)
        return -1, dp
    # jump probabilities: centre swept R->L, ||L_j M_l||^2 at each centre
    w = np.zeros(len(jumps))
    for s in range(L - 1, -1, -1):
        for j, (site, op, g) in enumerate(jumps):
            if site == s:
                N = np.einsum('st,tab->sab', op, mps[s])
                w[j] = g * np.real(np.vdot(N, N))
        if s > 0:
            C, B = lq_right(mps[s])
            mps[s] = B
            mps[s - 1] = absorb_left(mps[s - 1], C)
    cum = np.cumsum(w)
    W = cum[-1] if len(cum) else 0.0
    if not W > 1e-300:
        mps[0] = mps[0] / np.linalg.norm(mps[0])
        return -1, dp
    m = int(np.argmax(cum > r * W)) if np.any(cum > r * W) else int(np.nonzero(w)[0][-1])
    site, op, _ = jumps[m]
    sweep_qr_right(mps, 0, site)
    mps[site] = np.einsum('st,tab->sab', op, mps[site])
    mps[site] = mps[site] / np.linalg.norm(mps[site])
    # R7: successive SVDs, jump site -> right end, then right end -> site 0
    for s in range(site, L - 1):
        d, a, b = mps[s].shape
        U, S, Vh = svd_split(mps[s].reshape(d * a, b), opt)
        k = len(S)
        mps[s] = U.reshape(d, a, k)
        mps[s + 1] = absorb_right(S[:, None] * Vh, mps[s + 1])
    for s in range(L - 1, 0, -1):
        d, a, b = mps[s].shape
        U, S, Vh = svd_split(mps[s].transpose(1, 0, 2).reshape(a, d * b), opt)
        k = len(S)
        mps[s] = Vh.reshape(k, d, b).transpose(1, 0, 2)
        mps[s - 1] = absorb_left(mps[s - 1], U * S[None, :])
    mps[0] = mps[0] / np.linalg.norm(mps[0])
    return m, dp


# --------------------------------------------------------------------------
# Observables (Eq. TJMExpVal, per trajectory)
# --------------------------------------------------------------------------

def expectation_values(mps, observables):
    """<Psi|O_s|Psi>/<Psi|Psi> for single-site O, by full contraction."""
    L = len(mps)
    El = [None] * (L + 1)
    Er = [None] * (L + 1)
    El[0] = np.ones((1, 1), dtype=np.complex128)
    Er[L] = np.ones((1, 1), dtype=np.complex128)
    for s in range(L):
        El[s + 1] = np.einsum('xa,sxy,sab->yb', El[s], mps[s].conj(), mps[s])
    for s in range(L - 1, -1, -1):
        Er[s] = np.einsum('sxy,sab,yb->xa', mps[s].conj(), mps[s], Er[s + 1])
    nrm = np.real(El[L][0, 0])
    out = np.zeros(len(observables))
    for i, (s, O) in enumerate(observables):
        v = np.einsum('xa,txy,ts,sab,yb->', El[s], mps[s].conj(), O, mps[s], Er[s + 1])
        out[i] = np.real(v) / nrm
    return out


def mpo_expectation(mps, Wo):
    """<Psi|O|Psi>/<Psi|Psi> for an MPO O (Eq. TJMExpVal with O stored as an
    MPO; Methods, "Resources required for calculating expectation values"):
    the MPS-MPO-MPS network contracted site by site from the left, with the
    same environment update as TDVP; the real part (O Hermitian)."""
    E = np.ones((1, 1, 1), dtype=np.complex128)
    N = np.ones((1, 1), dtype=np.complex128)
    for M, W in zip(mps, Wo):
        E = left_update(E, M, W)
        N = np.einsum('xa,sxy,sab->yb', N, M.conj(), M)
    return float(np.real(E[0, 0, 0]) / np.real(N[0, 0]))


# --------------------------------------------------------------------------
# States and the trajectory schedule
# --------------------------------------------------------------------------

def product_mps(site_vecs):
    return [np.asarray(v, dtype=np.complex128).reshape(-1, 1, 1) for v in site_vecs]


def dense_to_mps(psi, L, d=2):
    """Exact (non-truncating) MPS of a dense state by successive QR, left to
    right; bonds are min(d^l, d^(L-l))."""
    mps = []
    rest = psi.reshape(1, -1)
    for s in range(L - 1):
        a = rest.shape[0]
        mat = rest.reshape(a, d, -1).transpose(1, 0, 2).reshape(d * a, -1)
        Q, R = np.linalg.qr(mat)
        mps.append(Q.reshape(d, a, Q.shape[1]))
        rest = R
    a = rest.shape[0]
    mps.append(rest.reshape(a, d, 1).transpose(1, 0, 2))
    return mps


def mps_to_dense(mps):
    psi = mps[0][:, 0, :]                      # (s, b)
    for M in mps[1:]:
        psi = np.einsum('pb,sbc->psc', psi, M).reshape(-1, M.shape[2])
    return psi[:, 0]


def canonicalize(mps):
    """Centre at site 0, normalised."""
    sweep_lq_left(mps, len(mps) - 1, 0)
    mps[0] = mps[0] / np.linalg.norm(mps[0])


def bonds(mps):
    return [1] + [M.shape[2] for M in mps]


def run_trajectory(Ws, jumps, psi0, dt, n_steps, observables, seed, traj, opt,
                   record=None, mpo_observables=(), order=2):
    """One trajectory; returns [n_steps+1, n_obs + n_mpo] expectation values:
    the single-site observables, then the MPO observables (each a list of
    site tensors W[s', s, w, w']), all measured on the same states.

    record (optional dict) receives 'jumps' [(step, branch, index)], 'bonds'
    (bond dimensions of the sampling MPS after each U), 'stats'."""
    L = len(Ws)
    Dh = [model.local_dissipator(jumps, s, 0.5 * dt) for s in range(L)]   # D_s[dt/2]
    Df = [model.local_dissipator(jumps, s, dt) for s in range(L)]         # D_s[dt]
    stats = Stats()
    phi = [M.copy() for M in psi0]
    canonicalize(phi)
    n_site = len(observables)

    def measure(psi):
        return np.concatenate([expectation_values(psi, observables),
                               [mpo_expectation(psi, Wo) for Wo in mpo_observables]])

    out = np.zeros((n_steps + 1, n_site + len(mpo_observables)))
    out[0] = measure(phi)
    jlog = []
    blog = []
    if order == 1:
        # first-order splitting (R19): F_k = J D[dt] U[dt] for k = 1..n
        for k in range(1, n_steps + 1):
            tdvp_step(phi, Ws, dt, opt, stats)
            blog.append(bonds(phi))
            dissipate(phi, Df)
            eps, r = philox.draws(seed, traj, k, philox.BRANCH_MAIN)
            m, _ = jump_process(phi, jumps, eps, r, opt)
            jlog.append((k, philox.BRANCH_MAIN, m))
            out[k] = measure(phi)
        if record is not None:
            record['jumps'] = jlog
            record['bonds'] = blog
            record['stats'] = stats
        return out
    # F_0 = J D[dt/2]
    dissipate(phi, Dh)
    eps, r = philox.draws(seed, traj, 0, philox.BRANCH_MAIN)
    m, _ = jump_process(phi, jumps, eps, r, opt)
    jlog.append((0, philox.BRANCH_MAIN, m))
    for k in range(1, n_steps + 1):
        tdvp_step(phi, Ws, dt, opt, stats)                # X = U[dt] Phi
        blog.append(bonds(phi))
        y = [M.copy() for M in phi]                       # sampling layer F_n
        dissipate(y, Dh)
        eps, r = philox.draws(seed, traj, k, philox.BRANCH_SAMPLE)
        m, _ = jump_process(y, jumps, eps, r, opt)
        jlog.append((k, philox.BRANCH_SAMPLE, m))
        out[k] = measure(y)
        if k < n_steps:                                   # F_k = J D[dt] U[dt]
            dissipate(phi, Df)
            eps, r = philox.draws(seed, traj, k, philox.BRANCH_MAIN)
            m, _ = jump_process(phi, jumps, eps, r, opt)
            jlog.append((k, philox.BRANCH_MAIN, m))
    if record is not None:
        record['jumps'] = jlog
        record['bonds'] = blog
        record['stats'] = stats
    return out
