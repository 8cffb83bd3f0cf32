"""Model builders for the oracle: operators, Hamiltonians, jump sets, dissipators.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Conventions (Sec. "Benchmarking" and Sec. "New frontiers"):
  * computational basis (|0>, |1>), Z = diag(1, -1), so <Z> = +1 on |0>;
  * sigma_minus = [[0, 1], [0, 0]] = |0><1| (relaxation towards |0>);
  * an MPO site tensor is W[s_out, s_in, w_left, w_right] as in the Methods
    section on matrix product operators (O = sum W^{s,s'} |s><s'|);
  * an MPS site tensor is M[s, a_left, a_right] as in the Methods section on
    matrix product states.

Field-direction reading: the XXX Hamiltonian of Sec. "New frontiers" carries a
Z field h.  The workloads here name a *transverse* field g, which is taken as
an X field (h_x = g, h_z = 0), matching the TFIM of Sec. "Benchmarking" where
g multiplies X.  Both fields are parameters, so either reading can be run.
"""
import numpy as np
import scipy.linalg as sla

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
SIGMA_MINUS = np.array([[0, 1], [0, 0]], dtype=np.complex128)
SIGMA_PLUS = np.array([[0, 0], [1, 0]], dtype=np.complex128)     # |1><0|, the adjoint of SIGMA_MINUS
SIGMA_PLUS = SIGMA_MINUS.conj().T


# --------------------------------------------------------------------------
# Hamiltonians
# --------------------------------------------------------------------------

def xxx_dense(L, J, hx=0.0, hz=0.0):
    """H0 = -J sum_i (X_i X_{i+1} + Y_i Y_{i+1} + Z_i Z_{i+1}) - hx sum X - hz sum Z,
    as an explicit sum of Kronecker products (Sec. "New frontiers")."""
    dim = 2 ** L

    def site_op(op, i):
        mats = [I2] * L
        mats[i] = op
        out = np.array([[1.0 + 0j]])
        for m in mats:
            out = np.kron(out, m)
        return out

    H = np.zeros((dim, dim), dtype=np.complex128)
    for i in range(L - 1):
        for P in (X, Y, Z):
            H -= J * site_op(P, i) @ site_op(P, i + 1)
    for i in range(L):
        H -= hx * site_op(X, i) + hz * site_op(Z, i)
    return H


def tfim_dense(L, J, g):
    """H0 = -J sum Z_i Z_{i+1} - g sum X_i (Sec. "Benchmarking")."""
    dim = 2 ** L

    def site_op(op, i):
        out = np.array([[1.0 + 0j]])
        for j in range(L):
            out = np.kron(out, op if j == i else I2)
        return out

    H = np.zeros((dim, dim), dtype=np.complex128)
    for i in range(L - 1):
        H -= J * site_op(Z, i) @ site_op(Z, i + 1)
    for i in range(L):
        H -= g * site_op(X, i)
    return H


def _lower_triangular_mpo(L, bulk):
    """Cut the first/last row/column of a D x D bulk operator matrix.

    bulk[w][w'] is a 2x2 operator.  The left boundary keeps the last row, the
    right boundary the first column (standard lower-triangular finite-state
    MPO).  Returns W[s_out, s_in, wl, wr] tensors.
    """
    D = len(bulk)
    Wb = np.zeros((2, 2, D, D), dtype=np.complex128)
    for a in range(D):
        for b in range(D):
            Wb[:, :, a, b] = bulk[a][b]
    if L == 1:
        return [Wb[:, :, D - 1:D, 0:1].copy()]
    Ws = [Wb[:, :, D - 1:D, :].copy()]
    for _ in range(1, L - 1):
        Ws.append(Wb.copy())
    Ws.append(Wb[:, :, :, 0:1].copy())
    return Ws


def xxx_mpo(L, J, hx=0.0, hz=0.0):
    """XXX chain as a bond-dimension-5 MPO; row-major operator-valued matrix

        [ I            0    0    0    0 ]
        [ X            0    0    0    0 ]
        [ Y            0    0    0    0 ]
        [ Z            0    0    0    0 ]
        [ -hx X - hz Z -J X -J Y -J Z I ]
    """
    O = np.zeros((2, 2), dtype=np.complex128)
    f = -hx * X - hz * Z
    bulk = [[I2, O, O, O, O],
            [X, O, O, O, O],
            [Y, O, O, O, O],
            [Z, O, O, O, O],
            [f, -J * X, -J * Y, -J * Z, I2]]
    return _lower_triangular_mpo(L, bulk)


def tfim_mpo(L, J, g):
    """TFIM as a bond-dimension-3 MPO: [[I,0,0],[Z,0,0],[-gX,-JZ,I]]."""
    O = np.zeros((2, 2), dtype=np.complex128)
    bulk = [[I2, O, O],
            [Z, O, O],
            [-g * X, -J * Z, I2]]
    return _lower_triangular_mpo(L, bulk)


def product_mpo(L, ops):
    """MPO of bond dimension 1 of the product operator prod_l O_l, with
    O_l = ops[l] where given and the identity elsewhere (for instance
    X_i X_{i+1} of Sec. "Effect of bond dimension and elapsed time")."""
    Ws = []
    for l in range(L):
        O = ops.get(l, I2)
        Ws.append(np.asarray(O, dtype=np.complex128).reshape(2, 2, 1, 1).copy())
    return Ws


def mpo_to_dense(Ws):
    """Contract an MPO into the dense operator (Methods, MPO section):
    O[(s1..sL), (s1'..sL')] = prod_l W_l^{s_l, s_l'}."""
    # T[s_out_block, s_in_block, w]
    T = Ws[0][:, :, 0, :]           # (2, 2, D1)
    for W in Ws[1:]:
        # T[A, B, w] W[s, t, w, v] -> T'[(A s), (B t), v]
        T = np.einsum('abw,stwv->asbtv', T, W)
        a, s, b, t, v = T.shape
        T = T.reshape(a * s, b * t, v)
    return T[:, :, 0]


# --------------------------------------------------------------------------
# Jump operators and dissipators
# --------------------------------------------------------------------------

def relax_dephase_jumps(L, gamma_minus, gamma_z):
    """Jump set of Sec. "Benchmarking": sigma_minus and Z on every site.

    Returned as a list of (site, 2x2 operator, rate) in site-major order with
    sigma_minus before Z at each site (the order the jump distribution is
    accumulated in)."""
    out = []
    for l in range(L):
        out.append((l, SIGMA_MINUS.copy(), float(gamma_minus)))
        out.append((l, Z.copy(), float(gamma_z)))
    return out


def relax_excite_jumps(L, gamma_minus, gamma_plus):
    """Relaxation and excitation on every site (Sec. "New frontiers", the
    30-site comparison): sigma_minus then sigma_plus at each site, site-major."""
    out = []
    for l in range(L):
        out.append((l, SIGMA_MINUS.copy(), float(gamma_minus)))
        out.append((l, SIGMA_PLUS.copy(), float(gamma_plus)))
    return out


def local_dissipator(jumps, site, tau, d=2):
    """D_l[tau] = exp(-1/2 tau sum_{j in S(l)} gamma_j L_j^dag L_j)
    (Eq. DissipativeMPO)."""
    G = np.zeros((d, d), dtype=np.complex128)
    for (s, op, g) in jumps:
        if s == site:
            G += g * op.conj().T @ op
    return sla.expm(-0.5 * tau * G)


# --------------------------------------------------------------------------
# States
# --------------------------------------------------------------------------

def product_site_vectors(L, bits):
    """Site vectors of the computational product state |bits>."""
    v = np.zeros((L, 2), dtype=np.complex128)
    for l in range(L):
        v[l, bits[l]] = 1.0
    return v


def neel_bits(L):
    """Neel state |0101...> (site 1 in |0>): a reading, the orientation is not given."""
    return [l % 2 for l in range(L)]


def zero_bits(L):
    return [0] * L


def domain_wall_bits(L):
    """Domain wall of Sec. "New frontiers": site l (1-based) in |0> for
    l < L/2 and in |1> for l >= L/2."""
    return [0 if (s + 1) < L / 2 else 1 for s in range(L)]


def product_dense(site_vecs):
    psi = np.array([1.0 + 0j])
    for v in site_vecs:
        psi = np.kron(psi, v)
    return psi


def site_op_dense(op, site, L):
    out = np.array([[1.0 + 0j]])
    for j in range(L):
        out = np.kron(out, op if j == site else I2)
    return out
