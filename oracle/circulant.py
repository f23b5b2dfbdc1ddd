"""Comparator preconditioners of the experiments (Section 4, the columns
next to PCG(tau)/PGMRES(tau) in Tables 1-4): no preconditioner, T. Chan's
optimal circulant and Strang's circulant.  For the circulant ones every
Toeplitz factor of the coefficient matrix (``original_matrix_form``: the
tridiagonal A_i and the fractional B_i) is replaced by its circulant
approximation of the same size.

Test infrastructure only (see the package docstring).

The paper cites both circulants without restating them; the definitions
used are the textbook ones (R. Chan and X. Jin, An Introduction to Iterative
Toeplitz Solvers, SIAM 2007, Chapter 2).  For an n x n Toeplitz matrix T with
entries T[j, k] = t_{j-k}:

* Strang's circulant keeps the central diagonals: first column
  s_j = t_j for 0 <= j <= floor(n/2) and s_j = t_{j-n} for floor(n/2) < j < n.
* T. Chan's optimal circulant is the circulant nearest to T in the Frobenius
  norm: first column c_j = ((n - j) t_j + j t_{j-n}) / n.

A circulant with first column c acts as x -> ifft(fft(c) * fft(x)), so its
eigenvalues are fft(c) in the DFT basis.  The multilevel preconditioner
P = C(A_3) (x) C(A_2) (x) C(A_1) + sum_i eta_i (.. C(B_i) ..) is therefore
diagonalised by the d-dimensional DFT with eigenvalues
Lambda = prod_i a_i + sum_i eta_i b_i prod_{j != i} a_j (a_i, b_i the
eigenvalues of C(A_i), C(B_i)), and P^{-1} R = ifftn(fftn(R) / Lambda).
In the non-symmetric case (k_{i,+} != k_{i,-}) the b_i are complex; P is
still real.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import operators

KINDS = ("none", "tchan", "strang")


def first_column(T: np.ndarray, kind: str) -> np.ndarray:
    """First column of the circulant approximation of the dense Toeplitz
    matrix T ("strang" or "tchan")."""
    n = T.shape[0]
    t_pos = T[:, 0]                                    # t_j, j = 0..n-1
    t_neg = np.concatenate([[0.0], T[0, 1:][::-1]])    # t_{j-n}, j = 0..n-1 (j = 0 unused)
    j = np.arange(n)
    if kind == "strang":
        return np.where(j <= n // 2, t_pos, t_neg)
    if kind == "tchan":
        return ((n - j) * t_pos + j * t_neg) / n
    raise ValueError(f"unknown circulant kind {kind!r}")


def factor_matrices(prob: operators.Problem, i: int):
    """The dense Toeplitz factors (A_i, B_i) of axis i (0-based)."""
    n = prob.n[i]
    return operators.A_mat(n), operators.B_mat(prob.q[i], n, prob.kplus[i], prob.kminus[i])


def factor_eigs(prob: operators.Problem, kind: str):
    """Eigenvalues (a_i, b_i) of the circulants of A_i and B_i, per axis, in
    the order of numpy's fft."""
    a, b = [], []
    for i in range(prob.dim):
        A, B = factor_matrices(prob, i)
        a.append(np.fft.fft(first_column(A, kind)))
        b.append(np.fft.fft(first_column(B, kind)))
    return a, b


def precond_eigs(prob: operators.Problem, kind: str) -> np.ndarray:
    """Lambda as a complex grid of shape prob.shape (axis 1 = x last)."""
    a, b = factor_eigs(prob, kind)
    d = prob.dim

    def grid(vecs):
        out = vecs[-1]
        for v in reversed(vecs[:-1]):
            out = np.multiply.outer(out, v)
        return out

    L = grid(a)
    for i in range(d):
        vecs = list(a)
        vecs[i] = b[i]
        L = L + prob.eta[i] * grid(vecs)
    return L


def apply_Pinv(prob: operators.Problem, R: np.ndarray, Lam: np.ndarray) -> np.ndarray:
    """P^{-1} R = ifftn(fftn(R) / Lambda); the result is real up to
    rounding and its real part is returned."""
    return np.real(np.fft.ifftn(np.fft.fftn(R) / Lam))


def dense_precond(prob: operators.Problem, kind: str) -> np.ndarray:
    """P as a dense matrix, assembled from dense circulants (an independent
    route to :func:`apply_Pinv` for tiny grids)."""
    d = prob.dim
    CA, CB = [], []
    for i in range(d):
        A, B = factor_matrices(prob, i)
        CA.append(sla.circulant(first_column(A, kind)))
        CB.append(sla.circulant(first_column(B, kind)))

    def kron_list(mats):
        # mats[i] acts on axis i+1; x is the fastest index
        out = mats[-1]
        for m in reversed(mats[:-1]):
            out = np.kron(out, m)
        return out

    P = kron_list(CA)
    for i in range(d):
        mats = list(CA)
        mats[i] = CB[i]
        P = P + prob.eta[i] * kron_list(mats)
    return P


def minv(prob: operators.Problem, kind: str):
    """The map r -> P^{-1} r of a comparator ("none": the identity)."""
    if kind == "none":
        return lambda v: v.copy()
    Lam = precond_eigs(prob, kind)
    return lambda v: apply_Pinv(prob, v, Lam)
