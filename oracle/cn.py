"""Crank-Nicolson time loop (Section 2, ``CN`` and ``linear_sys``).

Test infrastructure only (see the package docstring).

For m = 1..M: b^m = (A_N - K) u^{m-1} + dt F^{m-1/2}; u^m = A^{-1} b^m,
solved by PCG when k_{i,+} = k_{i,-} on every axis, else by left-preconditioned
GMRES (Remark after ``linear_sys``; Section 3), on request by GMRES on the
two-sided system (``two_side_system``, solver "gmres2"), or directly by LU
for tiny grids.
"""
from __future__ import annotations

from typing import Callable

import numpy as np

from . import circulant, krylov, operators


def solve_step(prob: operators.Problem, b: np.ndarray, x0: np.ndarray | None,
               tol: float, solver: str = "auto", restart: int = 20,
               maxit: int | None = None, Lam: np.ndarray | None = None,
               precond: str = "tau"):
    """One linear solve A u = b with the tau preconditioner, or with one of
    the comparators of Section 4 (precond "none", "tchan", "strang"; see
    :mod:`oracle.circulant`)."""
    if maxit is None:
        maxit = int(np.prod(prob.n))
    A = lambda v: operators.apply_A(prob, v)
    if precond == "tau":
        if Lam is None:
            Lam = operators.precond_eigs(prob)
        Minv = lambda v: operators.apply_Pinv(prob, v, Lam)
    else:
        Minv = circulant.minv(prob, precond)
    if solver == "auto":
        solver = "pcg" if prob.symmetric else "gmres"
    if solver == "pcg":
        return krylov.pcg(A, Minv, b, x0, tol, maxit)
    if solver == "gmres2":
        if precond != "tau":
            raise ValueError("the two-sided system is built for the tau preconditioner")
        # two-sided system; the initial u = x0 is P^{-1/2} v0 with v0 = P^{1/2} x0
        Mh = lambda v: operators.apply_Pinv_half(prob, v, Lam)
        v0 = None if x0 is None else operators.apply_P_half(prob, x0, Lam)
        return krylov.gmres_two_sided(A, Mh, b, v0, tol, restart, maxit)
    return krylov.gmres_left(A, Minv, b, x0, tol, restart, maxit)


def run(prob: operators.Problem, u0: np.ndarray, F_of_m: Callable[[int], np.ndarray | None],
        tol: float, x0_mode: str = "prev", solver: str = "auto", restart: int = 20,
        maxit: int | None = None, steps: int | None = None, precond: str = "tau"):
    """Advance ``steps`` (default M) CN steps from u0.  F_of_m(m) returns
    F^{m-1/2} (or None for f = 0).  x0_mode: "zero" (replication of the
    experiments) or "prev" (u^{m-1}).  precond: "tau" (the method) or a
    comparator ("none", "tchan", "strang").  Returns (u, per-step iteration
    counts)."""
    Lam = operators.precond_eigs(prob) if precond == "tau" else None
    u = u0.copy()
    iters = []
    for m in range(1, (steps or prob.M) + 1):
        b = operators.apply_rhs(prob, u, F_of_m(m))
        x0 = None if x0_mode == "zero" else u
        u, info = solve_step(prob, b, x0, tol, solver, restart, maxit, Lam, precond)
        iters.append(info.iters)
    return u, iters


def run_direct(prob: operators.Problem, u0: np.ndarray,
               F_of_m: Callable[[int], np.ndarray | None], steps: int | None = None):
    """Same loop with a dense LU solve per step (tiny grids only)."""
    A, R = operators.dense_system(prob)
    u = u0.reshape(-1).copy()
    for m in range(1, (steps or prob.M) + 1):
        F = F_of_m(m)
        b = R @ u + (prob.dt * F.reshape(-1) if F is not None else 0.0)
        u = np.linalg.solve(A, b)
    return u.reshape(u0.shape)
