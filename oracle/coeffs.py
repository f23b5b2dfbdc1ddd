"""Scalar and per-axis coefficients of the CN-FV scheme.

Test infrastructure only (see the package docstring).

References are to arXiv 2511.21198:
  * s_k, q_k: Section 2, the definitions accompanying the Toeplitz matrix T
    (label ``coef_expression``) and the hat-function derivative values at the
    control-volume faces.
  * eta_delta: Section 2, below the matrix form (label
    ``original_matrix_form``): eta = dt / (2 Gamma(delta+1) h^(2-delta)).
  * A_n eigenvalues: Lemma 3.1 (``tridiag_eig``); A_n = tridiag(1,6,1)/8 is a
    tau matrix, so its eigenvalues are (6 + 2 cos(k pi/(n+1)))/8.
  * tau eigenvalues: Lemma 3.2 (``1D_tau_SPD``), read with the summation index
    as j (the printed subscript k+1 inside the sum is a typo for j+1).
"""
from __future__ import annotations

import math

import mpmath as mp
import numpy as np

_DPS = 50  # working precision (decimal digits) for s_k / q_k


def s_coeffs_mp(delta: float, n: int):
    """s_k^{(delta)}, k = 0..n, in mpmath at 50 digits (Section 2).

    s_0 = (1/2)^d, s_1 = (3/2)^d - 2 (1/2)^d,
    s_k = (k+1/2)^d - 2 (k-1/2)^d + (k-3/2)^d  for k >= 2.
    The range is extended to k <= n on every axis (the paper writes the range
    for the first axis only).
    """
    with mp.workdps(_DPS):
        d = mp.mpf(delta)
        half = mp.mpf(1) / 2
        out = []
        for k in range(n + 1):
            if k == 0:
                v = half ** d
            elif k == 1:
                v = (3 * half) ** d - 2 * half ** d
            else:
                kk = mp.mpf(k)
                v = (kk + half) ** d - 2 * (kk - half) ** d + (kk - 3 * half) ** d
            out.append(v)
        return out


def q_coeffs_mp(delta: float, n: int):
    """q_k^{(delta)}, k = 0..n (Section 2, ``coef_expression``):
    q_0 = -s_0 and q_k = s_{k-1} - s_k for 1 <= k <= n.  mpmath values."""
    s = s_coeffs_mp(delta, n)
    with mp.workdps(_DPS):
        return [-s[0]] + [s[k - 1] - s[k] for k in range(1, n + 1)]


def s_coeffs(delta: float, n: int) -> np.ndarray:
    """float64 rounding of :func:`s_coeffs_mp`."""
    return np.array([float(v) for v in s_coeffs_mp(delta, n)], dtype=np.float64)


def q_coeffs(delta: float, n: int) -> np.ndarray:
    """float64 rounding of :func:`q_coeffs_mp` (each q_k rounded once, so the
    catastrophic cancellation of the third difference at large k is avoided)."""
    return np.array([float(v) for v in q_coeffs_mp(delta, n)], dtype=np.float64)


def q_coeffs_split(delta: float, n: int):
    """(hi, lo) float64 arrays with hi + lo = q_k to about 106 bits: hi is
    :func:`q_coeffs`, lo the float64 rounding of the remainder.  Used where a
    float64 rounding of the q_k themselves would show (the cancelling sum of
    :func:`tau_eigs`)."""
    qm = q_coeffs_mp(delta, n)
    hi = np.array([float(v) for v in qm], dtype=np.float64)
    with mp.workdps(_DPS):
        lo = np.array([float(v - mp.mpf(float(v))) for v in qm], dtype=np.float64)
    return hi, lo


def eta(delta: float, h: float, dt: float) -> float:
    """eta_delta = dt / (2 Gamma(delta+1) h^(2-delta)) (Section 2)."""
    return dt / (2.0 * math.gamma(delta + 1.0) * h ** (2.0 - delta))


def a_eigs(n: int) -> np.ndarray:
    """Eigenvalues of A_n = tridiag(1,6,1)/8 in the DST-I basis ordering,
    (3 + cos(k pi/(n+1)))/4, k = 1..n (Lemma 3.1; A_n is a tau matrix)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return (3.0 + np.cos(k * np.pi / (n + 1))) / 4.0


def tau_eigs(q: np.ndarray, n: int, q_lo: np.ndarray | None = None) -> np.ndarray:
    """Eigenvalues of tau(H(T_n)), k = 1..n (Lemma 3.2, index read as j):

        lambda_k = q_1 + (q_0 + q_2) cos(theta_k) + sum_{j=2}^{n-1} q_{j+1} cos(j theta_k),
        theta_k = k pi / (n+1).

    ``q`` holds q_0..q_n (``q_lo`` optionally the float64 remainders of
    q_coeffs_split).  For n = 1 the sum and the cosine term vanish
    (H(T_1) = [q_1]).

    The q_j sum to zero (Lemma 2.1), so for small theta_k the sum cancels:
    the smallest eigenvalue is of order theta_1^(1+delta) (5e-6 at n = 4095,
    delta = 0.35) while its terms are of order one.  A float64 evaluation
    loses about five digits of it there, and so does rounding the q_j to
    float64 first.  The sum is therefore taken in the extended precision of
    numpy.longdouble (cosines included), from q_j to extended precision
    when q_lo is given, and rounded once."""
    ld = np.longdouble
    k = np.arange(1, n + 1, dtype=ld)
    th = k * (ld(np.pi) + ld(1.2246467991473532e-16)) / ld(n + 1)   # pi to extended precision
    ql = np.asarray(q, dtype=np.float64).astype(ld)
    if q_lo is not None:
        ql = ql + np.asarray(q_lo, dtype=np.float64).astype(ld)
    lam = np.full(n, ql[1], dtype=ld)
    if n >= 2:
        lam = lam + (ql[0] + ql[2]) * np.cos(th)
    for j in range(2, n):
        lam = lam + ql[j + 1] * np.cos(ld(j) * th)
    return lam.astype(np.float64)


def sym_first_column(q: np.ndarray, n: int) -> np.ndarray:
    """First column of H(T_n) = (T + T^T)/2 (proof of Theorem 3.1):
    [q_1, (q_0+q_2)/2, q_3/2, ..., q_n/2]."""
    t = np.zeros(n, dtype=np.float64)
    t[0] = q[1]
    if n >= 2:
        t[1] = 0.5 * (q[0] + q[2])
    for j in range(2, n):
        t[j] = 0.5 * q[j + 1]
    return t
