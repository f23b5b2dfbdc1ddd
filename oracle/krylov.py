"""Textbook preconditioned Krylov solvers.

Test infrastructure only (see the package docstring).

* :func:`pcg` - preconditioned conjugate gradients with the preconditioner P
  (Section 3.1; used when k_{i,+} = k_{i,-}).  Stops when the recursively
  updated residual satisfies ||r_k||_2 <= tol ||b||_2.
* :func:`gmres_left` - restarted GMRES on the left-preconditioned system
  P^{-1} A u = P^{-1} b (Section 3.2, ``one_side_system``), modified
  Gram-Schmidt Arnoldi and Givens rotations.  Stops when the preconditioned
  residual satisfies ||P^{-1}(b - A x_k)||_2 <= tol ||P^{-1} b||_2.
* :func:`gmres_two_sided` - restarted GMRES on the two-sided system
  P^{-1/2} A P^{-1/2} v = P^{-1/2} b, u = P^{-1/2} v (Section 3.2,
  ``two_side_system``, the system Theorem 3.2 bounds).  Stops when
  ||P^{-1/2}(b - A x_k)||_2 <= tol ||P^{-1/2} b||_2.

The experiments (Section 4) run MATLAB's pcg/gmres with restart 20,
tol 1e-9 and maxit n^3; the initial guess and the stopping norms are not
stated.  The readings used here (zero initial guess for replication,
recursive residual for PCG, preconditioned residual for left GMRES) reproduce
the printed iteration counts.
"""
from __future__ import annotations

import dataclasses
from typing import Callable

import numpy as np


@dataclasses.dataclass
class SolveInfo:
    iters: int
    converged: bool
    relres: float          # the solver's own stopping quantity at exit
    history: list


def _dot(a, b):
    return float(np.sum(a * b))


def _nrm(a):
    return float(np.sqrt(np.sum(a * a)))


def pcg(A: Callable, Minv: Callable, b: np.ndarray, x0: np.ndarray | None,
        tol: float, maxit: int) -> tuple[np.ndarray, SolveInfo]:
    """PCG: alpha = (r,z)/(p,Ap), x += alpha p, r -= alpha Ap, z = P^{-1} r,
    beta = (r_new, z_new)/(r, z), p = z + beta p."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    nb = _nrm(b)
    if nb == 0.0:
        return np.zeros_like(b), SolveInfo(0, True, 0.0, [0.0])
    r = b - A(x)
    hist = [_nrm(r) / nb]
    if hist[-1] <= tol:
        return x, SolveInfo(0, True, hist[-1], hist)
    z = Minv(r)
    p = z.copy()
    rz = _dot(r, z)
    for it in range(1, maxit + 1):
        q = A(p)
        alpha = rz / _dot(p, q)
        x += alpha * p
        r -= alpha * q
        hist.append(_nrm(r) / nb)
        if hist[-1] <= tol:
            return x, SolveInfo(it, True, hist[-1], hist)
        z = Minv(r)
        rz_new = _dot(r, z)
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, SolveInfo(maxit, False, hist[-1], hist)


def gmres_left(A: Callable, Minv: Callable, b: np.ndarray, x0: np.ndarray | None,
               tol: float, restart: int, maxit: int) -> tuple[np.ndarray, SolveInfo]:
    """Left-preconditioned restarted GMRES(restart).  ``iters`` counts inner
    iterations over all cycles."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    pb = Minv(b)
    npb = _nrm(pb)
    if npb == 0.0:
        return np.zeros_like(b), SolveInfo(0, True, 0.0, [0.0])
    total = 0
    r = Minv(b - A(x))
    beta = _nrm(r)
    hist = [beta / npb]
    if hist[-1] <= tol:
        return x, SolveInfo(0, True, hist[-1], hist)
    while total < maxit:
        m = restart
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_done = 0
        converged = False
        for j in range(m):
            w = Minv(A(V[j]))
            for i in range(j + 1):           # modified Gram-Schmidt
                H[i, j] = _dot(w, V[i])
                w = w - H[i, j] * V[i]
            hnext = _nrm(w)
            H[j + 1, j] = hnext
            for i in range(j):               # apply the previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k_done = j + 1
            hist.append(abs(g[j + 1]) / npb)
            if hist[-1] <= tol or total >= maxit or hnext == 0.0:
                converged = hist[-1] <= tol or hnext == 0.0
                break
            V.append(w / hnext)
        # least squares: upper-triangular solve H[:k,:k] y = g[:k]
        k = k_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            x = x + y[i] * V[i]
        if converged:
            return x, SolveInfo(total, True, hist[-1], hist)
        r = Minv(b - A(x))
        beta = _nrm(r)
        if beta / npb <= tol:
            return x, SolveInfo(total, True, beta / npb, hist)
    return x, SolveInfo(total, False, hist[-1], hist)


def gmres_two_sided(A: Callable, Mh: Callable, b: np.ndarray, v0: np.ndarray | None,
                    tol: float, restart: int, maxit: int) -> tuple[np.ndarray, SolveInfo]:
    """Restarted GMRES(restart) on Z v = w with Z = P^{-1/2} A P^{-1/2} and
    w = P^{-1/2} b (Mh applies P^{-1/2}); v0 is the initial guess of v (the
    initial u is P^{-1/2} v0).  Returns u = P^{-1/2} v and the history of
    ||w - Z v_k|| / ||w|| (the residual of Theorem 3.2, relative)."""
    Z = lambda v: Mh(A(Mh(v)))
    w0 = Mh(b)
    nw = _nrm(w0)
    if nw == 0.0:
        return np.zeros_like(b), SolveInfo(0, True, 0.0, [0.0])
    v = np.zeros_like(b) if v0 is None else v0.copy()
    total = 0
    r = w0 - Z(v)
    beta = _nrm(r)
    hist = [beta / nw]
    if hist[-1] <= tol:
        return Mh(v), SolveInfo(0, True, hist[-1], hist)
    while total < maxit:
        m = restart
        V = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_done = 0
        converged = False
        for j in range(m):
            q = Z(V[j])
            for i in range(j + 1):           # modified Gram-Schmidt
                H[i, j] = _dot(q, V[i])
                q = q - H[i, j] * V[i]
            hnext = _nrm(q)
            H[j + 1, j] = hnext
            for i in range(j):               # apply the previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k_done = j + 1
            hist.append(abs(g[j + 1]) / nw)
            if hist[-1] <= tol or total >= maxit or hnext == 0.0:
                converged = hist[-1] <= tol or hnext == 0.0
                break
            V.append(q / hnext)
        k = k_done
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        for i in range(k):
            v = v + y[i] * V[i]
        if converged:
            return Mh(v), SolveInfo(total, True, hist[-1], hist)
        r = w0 - Z(v)
        beta = _nrm(r)
        if beta / nw <= tol:
            return Mh(v), SolveInfo(total, True, beta / nw, hist)
    return Mh(v), SolveInfo(total, False, hist[-1], hist)
