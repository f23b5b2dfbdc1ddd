"""Operators of the CN-FV scheme: dense assembly for tiny grids and plain
structured (axis-by-axis) application for any grid.

Test infrastructure only (see the package docstring).

Array convention: a grid function on n_1 x ... x n_d interior nodes is a NumPy
array of shape (n_d, ..., n_1) in C order, so the x index runs fastest exactly
as in the vector ordering of Section 2 (the definition of u^m and F^{m-1/2}).
Axis i (1-based: x=1, y=2, z=3) is NumPy axis d - i.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Sequence

import numpy as np
import scipy.fft as sfft

from . import coeffs


@dataclasses.dataclass
class Problem:
    """Parameters of one CN-FV problem (Section 1 model, Section 2 grid).

    dim: 2 or 3; n: interior nodes per axis; delta: (alpha, beta, gamma);
    kplus/kminus: the diffusivities k_{i,+}, k_{i,-}; domain (a_i, b_i);
    M steps to final time T.
    """
    dim: int
    n: Sequence[int]
    delta: Sequence[float]
    kplus: Sequence[float]
    kminus: Sequence[float]
    T: float = 1.0
    M: int = 1
    a: Sequence[float] = (0.0, 0.0, 0.0)
    b: Sequence[float] = (1.0, 1.0, 1.0)

    def __post_init__(self):
        d = self.dim
        self.n = [int(v) for v in self.n][:d]
        self.delta = [float(v) for v in self.delta][:d]
        self.kplus = [float(v) for v in self.kplus][:d]
        self.kminus = [float(v) for v in self.kminus][:d]
        self.a = [float(v) for v in self.a][:d]
        self.b = [float(v) for v in self.b][:d]
        self.dt = self.T / self.M
        # h_i = (b_i - a_i)/(n_i + 1)  (Section 2 grid)
        self.h = [(self.b[i] - self.a[i]) / (self.n[i] + 1) for i in range(d)]
        self.eta = [coeffs.eta(self.delta[i], self.h[i], self.dt) for i in range(d)]
        qs = [coeffs.q_coeffs_split(self.delta[i], self.n[i]) for i in range(d)]
        self.q = [hi for hi, _ in qs]       # float64 q_k (the matrices)
        self.q_lo = [lo for _, lo in qs]    # remainders (the tau eigenvalues)

    @property
    def shape(self):
        return tuple(reversed(self.n))

    @property
    def N(self):
        return int(np.prod(self.n))

    @property
    def symmetric(self) -> bool:
        """k_{i,+} == k_{i,-} on every axis (Remark after ``linear_sys``)."""
        return all(self.kplus[i] == self.kminus[i] for i in range(self.dim))


# --------------------------------------------------------------------------
# One-dimensional factors
# --------------------------------------------------------------------------

def A_mat(n: int) -> np.ndarray:
    """A_n = tridiag(1, 6, 1)/8 (Section 2, ``tridiag_matrix``)."""
    A = np.zeros((n, n))
    for i in range(n):
        A[i, i] = 6.0 / 8.0
        if i > 0:
            A[i, i - 1] = 1.0 / 8.0
        if i + 1 < n:
            A[i, i + 1] = 1.0 / 8.0
    return A


def T_mat(q: np.ndarray, n: int) -> np.ndarray:
    """T_n[i, p] = q_{i-p+1} for i-p+1 >= 0, else 0 (Section 2, ``T_ni``):
    q_1 on the diagonal, q_0 above it, q_2..q_n below."""
    T = np.zeros((n, n))
    for i in range(n):
        for p in range(n):
            k = i - p + 1
            if k >= 0:
                T[i, p] = q[k]
    return T


def B_mat(q: np.ndarray, n: int, kp: float, km: float) -> np.ndarray:
    """B_n = k_+ T_n + k_- T_n^T (Section 2, ``stiff_matrix``)."""
    T = T_mat(q, n)
    return kp * T + km * T.T


def B_from_hat_functions(delta: float, n: int, kp: float, km: float) -> np.ndarray:
    """B_n assembled entry by entry from the finite-volume definition, without
    using s_k or q_k.

    The left and right Riemann-Liouville derivatives of order 1-delta of a ramp
    (x-c)_+ (resp. (c-x)_+) are (x-c)_+^delta / Gamma(delta+1) (resp.
    (c-x)_+^delta / Gamma(delta+1)); a hat function is a second difference of
    ramps.  The flux D phi_p = k_+ d^{1-d}_x phi_p - k_- d^{1-d}_{-x} phi_p is
    evaluated at the faces x_{i+-1/2}; the scheme (Section 2, ``fvm_sol``)
    carries -[D phi_p]_{x_{i-1/2}}^{x_{i+1/2}}, which after division by
    h^{delta-1}/Gamma(delta+1) is the (i, p) entry of B_n.
    Exact arithmetic is done in mpmath and rounded once.
    """
    import mpmath as mp
    with mp.workdps(40):
        d = mp.mpf(delta)

        def pos(v):
            return v ** d if v > 0 else mp.mpf(0)

        def left(i_face2, p):
            # face at (i_face2/2) h, node p at p h; unit h (scaled out).
            x = mp.mpf(i_face2) / 2
            return pos(x - (p - 1)) - 2 * pos(x - p) + pos(x - (p + 1))

        def right(i_face2, p):
            x = mp.mpf(i_face2) / 2
            return pos((p + 1) - x) - 2 * pos(p - x) + pos((p - 1) - x)

        B = np.zeros((n, n))
        for i in range(1, n + 1):
            for p in range(1, n + 1):
                up, lo = 2 * i + 1, 2 * i - 1
                flux_up = kp * left(up, p) - km * right(up, p)
                flux_lo = kp * left(lo, p) - km * right(lo, p)
                B[i - 1, p - 1] = float(-(flux_up - flux_lo))
    return B


def tau_of_symmetric_toeplitz(t: np.ndarray) -> np.ndarray:
    """tau(T) = T - H for the symmetric Toeplitz matrix T with first column t
    (Bini and Capovani's tau matrix, cited in Section 3 for
    ``pre_definition``): H is the Hankel matrix with first row
    (t_2, ..., t_{n-1}, 0, 0) and last row (0, 0, t_{n-1}, ..., t_2)."""
    n = len(t)
    T = np.array([[t[abs(i - j)] for j in range(n)] for i in range(n)])
    H = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            s = i + j
            if s + 2 <= n - 1:
                H[i, j] = t[s + 2]
            elif s >= n + 1:
                H[i, j] = t[2 * n - s]
    return T - H


def dst1_mat(n: int) -> np.ndarray:
    """S_n[j, k] = sqrt(2/(n+1)) sin(j k pi/(n+1)), 1 <= j, k <= n (Section 3,
    below ``pre_definition``)."""
    j = np.arange(1, n + 1)
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.outer(j, j) * np.pi / (n + 1))


# --------------------------------------------------------------------------
# Dense assembly (tiny grids)
# --------------------------------------------------------------------------

def _kron_list(mats):
    """Kronecker product M_d (x) ... (x) M_1 of mats = [M_1, ..., M_d]
    (x fastest, Section 2 ordering)."""
    out = mats[-1]
    for Mi in reversed(mats[:-1]):
        out = np.kron(out, Mi)
    return out


def dense_system(prob: Problem, B_source: str = "q"):
    """Dense (A, R) with A u^m = R u^{m-1} + dt F (Section 2,
    ``original_matrix_form`` / ``linear_sys``), the 2D case obtained by
    dropping the z factor.

    B_source = "q" builds B from q_k (``stiff_matrix``); "hat" builds it from
    the hat-function derivatives (:func:`B_from_hat_functions`).
    """
    d = prob.dim
    As = [A_mat(prob.n[i]) for i in range(d)]
    if B_source == "q":
        Bs = [B_mat(prob.q[i], prob.n[i], prob.kplus[i], prob.kminus[i]) for i in range(d)]
    else:
        Bs = [B_from_hat_functions(prob.delta[i], prob.n[i], prob.kplus[i], prob.kminus[i])
              for i in range(d)]
    AN = _kron_list(As)
    K = np.zeros_like(AN)
    for i in range(d):
        mats = list(As)
        mats[i] = Bs[i]
        K += prob.eta[i] * _kron_list(mats)
    return AN + K, AN - K


def dense_preconditioner(prob: Problem) -> np.ndarray:
    """P = A_N + sum_i eta_i (k_{i,+}+k_{i,-}) (A (x) .. (x) tau(H(T_i)) (x) .. (x) A)
    built explicitly from tau matrices (Section 3, ``pre_definition``)."""
    d = prob.dim
    As = [A_mat(prob.n[i]) for i in range(d)]
    P = _kron_list(As)
    for i in range(d):
        t = coeffs.sym_first_column(prob.q[i], prob.n[i])
        mats = list(As)
        mats[i] = tau_of_symmetric_toeplitz(t)
        P = P + prob.eta[i] * (prob.kplus[i] + prob.kminus[i]) * _kron_list(mats)
    return P


# --------------------------------------------------------------------------
# Structured application (any grid)
# --------------------------------------------------------------------------

def _along(M: np.ndarray, X: np.ndarray, axis: int, dim: int) -> np.ndarray:
    """Apply the n_i x n_i matrix M along axis i (1-based) of X."""
    ax = dim - axis
    Y = np.tensordot(M, X, axes=([1], [ax]))  # new axis 0
    return np.moveaxis(Y, 0, ax)


def _terms(prob: Problem, X: np.ndarray):
    """Return (A_N X, [A..B_i..A X for each i])."""
    d = prob.dim
    As = [A_mat(prob.n[i]) for i in range(d)]
    Bs = [B_mat(prob.q[i], prob.n[i], prob.kplus[i], prob.kminus[i]) for i in range(d)]
    AN = X
    for i in range(d):
        AN = _along(As[i], AN, i + 1, d)
    Ks = []
    for j in range(d):
        Y = X
        for i in range(d):
            Y = _along(Bs[i] if i == j else As[i], Y, i + 1, d)
        Ks.append(Y)
    return AN, Ks


def apply_A(prob: Problem, X: np.ndarray) -> np.ndarray:
    """A X with A = A_N + sum_i eta_i (.. (x) B_i (x) ..) (``linear_sys``),
    each Kronecker term applied axis by axis with dense factors."""
    AN, Ks = _terms(prob, X)
    return AN + sum(prob.eta[i] * Ks[i] for i in range(prob.dim))


def apply_rhs(prob: Problem, U: np.ndarray, F: np.ndarray | None) -> np.ndarray:
    """b^m = (A_N - sum_i eta_i (..B_i..)) u^{m-1} + dt F^{m-1/2}
    (``linear_sys``; the source factor printed as tau is the time step)."""
    AN, Ks = _terms(prob, U)
    out = AN - sum(prob.eta[i] * Ks[i] for i in range(prob.dim))
    if F is not None:
        out = out + prob.dt * F
    return out


def toeplitz_generator(prob: Problem, sign: float = 1.0) -> dict:
    """Diagonal generators of the multilevel Toeplitz matrix A_N + sign*K:
    a dict mapping offset tuples (d_d, ..., d_1) (row minus column index per
    axis) to coefficients.  Used by the circulant-embedding route."""
    d = prob.dim
    a1 = {-1: 1.0 / 8.0, 0: 6.0 / 8.0, 1: 1.0 / 8.0}
    gens = []
    for i in range(d):
        n = prob.n[i]
        q = prob.q[i]
        kp, km = prob.kplus[i], prob.kminus[i]
        b = {}
        # B[i,p] = kp q_{i-p+1} + km q_{p-i+1}; offset o = i - p
        for o in range(-(n - 1), n):
            v = 0.0
            if o + 1 >= 0:
                v += kp * q[o + 1]
            if -o + 1 >= 0:
                v += km * q[-o + 1]
            b[o] = v
        gens.append(b)
    import itertools
    G = {}
    for o in itertools.product(*[range(-(prob.n[i] - 1), prob.n[i]) for i in reversed(range(d))]):
        offs = list(reversed(o))  # offs[i] for axis i+1
        base = 1.0
        for i in range(d):
            base *= a1.get(offs[i], 0.0)
        v = base
        for j in range(d):
            t = sign * prob.eta[j]
            for i in range(d):
                t *= gens[i][offs[i]] if i == j else a1.get(offs[i], 0.0)
            v += t
        if v != 0.0:
            G[o] = v
    return G


def apply_A_circulant(prob: Problem, X: np.ndarray, sign: float = 1.0) -> np.ndarray:
    """(A_N + sign*K) X by embedding the d-level Toeplitz matrix in a d-level
    circulant of size 2 n_i per axis and multiplying with a d-dimensional real
    FFT (the fast matvec the paper refers to in Section 1).  An independent
    route to :func:`apply_A` used as a cross-check; only practical for small
    grids because the generator is built entry by entry."""
    d = prob.dim
    L = [2 * prob.n[i] for i in reversed(range(d))]
    C = np.zeros(L)
    for o, v in toeplitz_generator(prob, sign).items():
        idx = tuple(o[k] % L[k] for k in range(d))
        C[idx] += v
    Xp = np.zeros(L)
    Xp[tuple(slice(0, s) for s in X.shape)] = X
    Y = sfft.irfftn(sfft.rfftn(C) * sfft.rfftn(Xp), s=L)
    return Y[tuple(slice(0, s) for s in X.shape)]


def precond_eigs(prob: Problem) -> np.ndarray:
    """Lambda of P = S_N Lambda S_N as a grid array (Section 3,
    ``diag_tau_pre``):
    Lambda = prod_i a_i + sum_i c_i lambda_i prod_{j != i} a_j,
    c_i = eta_i (k_{i,+} + k_{i,-})."""
    d = prob.dim
    a = [coeffs.a_eigs(prob.n[i]) for i in range(d)]
    lam = [coeffs.tau_eigs(prob.q[i], prob.n[i], prob.q_lo[i]) for i in range(d)]

    def grid(vecs):
        out = vecs[-1]
        for v in reversed(vecs[:-1]):
            out = np.multiply.outer(out, v)
        return out  # shape (n_d, ..., n_1)

    L = grid(a)
    for i in range(d):
        vecs = list(a)
        vecs[i] = lam[i]
        L = L + prob.eta[i] * (prob.kplus[i] + prob.kminus[i]) * grid(vecs)
    return L


def dst_all(X: np.ndarray) -> np.ndarray:
    """S_N X: orthonormal DST-I along every axis."""
    return sfft.dstn(X, type=1, norm="ortho")


def apply_Pinv(prob: Problem, R: np.ndarray, Lam: np.ndarray | None = None) -> np.ndarray:
    """P^{-1} R = S_N Lambda^{-1} S_N R (Section 3, ``diag_tau_pre``; S_N is
    symmetric and orthogonal)."""
    if Lam is None:
        Lam = precond_eigs(prob)
    return dst_all(dst_all(R) / Lam)


def apply_Pinv_half(prob: Problem, R: np.ndarray, Lam: np.ndarray | None = None) -> np.ndarray:
    """P^{-1/2} R = S_N Lambda^{-1/2} S_N R, the half preconditioner of the
    two-sided system (Section 3.2, ``two_side_system``)."""
    if Lam is None:
        Lam = precond_eigs(prob)
    return dst_all(dst_all(R) / np.sqrt(Lam))


def apply_P_half(prob: Problem, X: np.ndarray, Lam: np.ndarray | None = None) -> np.ndarray:
    """P^{1/2} X = S_N Lambda^{1/2} S_N X."""
    if Lam is None:
        Lam = precond_eigs(prob)
    return dst_all(dst_all(X) * np.sqrt(Lam))


def apply_P(prob: Problem, X: np.ndarray, Lam: np.ndarray | None = None) -> np.ndarray:
    """P X = S_N Lambda S_N X."""
    if Lam is None:
        Lam = precond_eigs(prob)
    return dst_all(dst_all(X) * Lam)


def apply_A_at(prob: Problem, X: np.ndarray, idx, sign: float = 1.0) -> float:
    """Entry ``idx`` (a NumPy index tuple (k, j, i) / (j, i)) of
    (A_N + sign*K) X, from the definition of the Kronecker terms: each term
    is a product of one row per axis, contracted with X.  Cheap for any grid
    size (dense B rows of length n_i, tridiagonal A rows)."""
    d = prob.dim
    rows_A, rows_B = [], []
    for i in range(d):
        n = prob.n[i]
        r = idx[d - 1 - i]
        a = np.zeros(n)
        a[r] = 0.75
        if r > 0:
            a[r - 1] = 0.125
        if r + 1 < n:
            a[r + 1] = 0.125
        q = prob.q[i]
        b = np.zeros(n)
        for p in range(n):
            v = 0.0
            if r - p + 1 >= 0:
                v += prob.kplus[i] * q[r - p + 1]
            if p - r + 1 >= 0:
                v += prob.kminus[i] * q[p - r + 1]
            b[p] = v
        rows_A.append(a)
        rows_B.append(b)

    def contract(rows):
        Y = X
        for i in reversed(range(d)):          # outermost axis first
            Y = np.tensordot(rows[i], Y, axes=([0], [0]))
        return float(Y)

    out = contract(rows_A)
    for j in range(d):
        rows = [rows_B[i] if i == j else rows_A[i] for i in range(d)]
        out += sign * prob.eta[j] * contract(rows)
    return out
