"""Seeded synthetic inputs for the solver workloads.

This module holds input generation only (parameters, initial data and
sources); it contains none of the solver's arithmetic, so both the oracle
tests and the HIP path may draw from it.

Conventions: domain (0,1)^d, h = 1/(n+1), nodes x_i = i h; arrays have shape
(n_d, ..., n_1) with x fastest; a "Gaussian bump of width w centred at c" is
exp(-|x - c|^2 / (2 w^2)) with amplitude 1; sources are point values at the
nodes in float64.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Workload:
    name: str
    dim: int
    n: list
    delta: list
    kplus: list
    kminus: list
    M: int
    T: float
    tol: float
    solver: str                  # "pcg" | "gmres"
    u0: np.ndarray
    F: Optional[np.ndarray]      # time-independent source (None: f = 0)
    bumps: Optional[dict] = None  # moving-bump description for time-dependent sources


def _axes(n):
    return [np.arange(1, k + 1, dtype=np.float64) / (k + 1) for k in n]


def bumps_source(n, centres, width=0.1):
    """Sum of Gaussian bumps at the nodes of an n_1 x n_2 (x n_3) grid."""
    d = len(n)
    ax = _axes(n)
    out = np.zeros(tuple(reversed(n)))
    for c in centres:
        g = None
        for i in reversed(range(d)):
            e = np.exp(-((ax[i] - c[i]) ** 2) / (2.0 * width * width))
            g = e if g is None else np.multiply.outer(g, e)
        out += g
    return out


def sine_profile(n):
    """prod_i sin(pi x_i) at the nodes."""
    ax = _axes(n)
    g = None
    for i in reversed(range(len(n))):
        e = np.sin(np.pi * ax[i])
        g = e if g is None else np.multiply.outer(g, e)
    return g


def config_2d_symmetric(seed: int = 0, n: int = 63) -> Workload:
    """2D symmetric plain method: alpha = beta = 0.5, k+- = 1, 63 x 63,
    M = 64 steps to T = 1, u0 = amp sin(pi x) sin(pi y) with amp ~ U(0.5, 1.5),
    f = 0, PCG, tol 1e-10."""
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.5, 1.5)
    return Workload("2d_sym_63", 2, [n, n], [0.5, 0.5], [1.0, 1.0], [1.0, 1.0],
                    64, 1.0, 1e-10, "pcg", amp * sine_profile([n, n]), None)


def config_3d_symmetric(seed: int = 0, n: int = 127, M: int = 32) -> Workload:
    """3D symmetric: (alpha, beta, gamma) = (0.3, 0.5, 0.7), k+- = 1, 127^3,
    32 steps to T = 1, f = 8 Gaussian bumps (centres U(0.2,0.8)^3, width 0.1),
    u0 = 0, PCG, tol 1e-10."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, (8, 3))
    F = bumps_source([n, n, n], centres)
    return Workload(f"3d_sym_{n}", 3, [n, n, n], [0.3, 0.5, 0.7], [1.0] * 3, [1.0] * 3,
                    M, 1.0, 1e-10, "pcg", np.zeros_like(F), F)


def config_3d_nonsymmetric(seed: int = 0, n: int = 255, M: int = 16) -> Workload:
    """3D non-symmetric: (0.4, 0.6, 0.8), k+ = (1.0, 0.8, 1.2),
    k- = (0.5, 1.0, 0.3), 255^3, 16 steps to T = 1, 8 bumps, u0 = 0,
    PGMRES(20), tol 1e-8."""
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.2, 0.8, (8, 3))
    F = bumps_source([n, n, n], centres)
    return Workload(f"3d_nonsym_{n}", 3, [n, n, n], [0.4, 0.6, 0.8], [1.0, 0.8, 1.2],
                    [0.5, 1.0, 0.3], M, 1.0, 1e-8, "gmres", np.zeros_like(F), F)


# Solver settings of the benchmark's headline workload (3D non-symmetric
# 255^3, left GMRES(20) from u^{m-1}): the relative tolerance of both the
# float64 and the mixed-precision solvers is the paper's 1e-9 (Section 4),
# which keeps u^M within 1e-8 of the tightly solved trajectory in the
# 2-norm and in the max-norm (at 1e-8 the per-step solve errors add up over
# the 16 steps to 2e-8 in the 2-norm and 7e-8 to 1.2e-7 in the max-norm);
# inner tolerance and outer-step limit of the float32 solves.
HEADLINE_SOLVER = dict(tol=1e-9, inner_tol=1e-3, max_outer=8, restart=20, x0="prev")


def config_batched(count: int = 64, base_seed: int = 1000,
                   sizes_2d=(127, 255, 511, 1023), sizes_3d=(63, 95, 127)):
    """Batched instances: instance i uses seed base_seed + i; 2D for the first
    half, 3D for the rest; each axis size drawn from the size list; orders
    U(0.1, 0.9); k+ ~ U(0.5, 2); k- = k+ for even i (PCG), else U(0.5, 2)
    (PGMRES); M = 8, T = 1, u0 = 0, 8 bumps of width 0.1; tol 1e-8."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(base_seed + i)
        dim = 2 if i < count // 2 else 3
        sizes = sizes_2d if dim == 2 else sizes_3d
        n = [int(rng.choice(sizes)) for _ in range(dim)]
        delta = list(rng.uniform(0.1, 0.9, dim))
        kp = list(rng.uniform(0.5, 2.0, dim))
        km = list(kp) if i % 2 == 0 else list(rng.uniform(0.5, 2.0, dim))
        centres = rng.uniform(0.2, 0.8, (8, dim))
        F = bumps_source(n, centres)
        out.append(Workload(f"batch_{i}", dim, n, delta, kp, km, 8, 1.0, 1e-8,
                            "pcg" if i % 2 == 0 else "gmres", np.zeros_like(F), F))
    return out


def moving_bumps(seed: int, count: int = 8):
    """Centres c_b(t) = c_b0 + v_b t with c_b0 ~ U(0.3, 0.7)^3 and
    v_b ~ U(-0.2, 0.2)^3."""
    rng = np.random.default_rng(seed)
    c0 = rng.uniform(0.3, 0.7, (count, 3))
    v = rng.uniform(-0.2, 0.2, (count, 3))
    return {"c0": c0, "v": v, "width": 0.1}


def moving_bumps_source(n, bumps, t):
    return bumps_source(n, bumps["c0"] + bumps["v"] * t, bumps["width"])


def config_learned(seed: int, n: int = 255, M: int = 200) -> Workload:
    """Learned warm start workload: 3D symmetric, orders U(0.2, 0.8) per run,
    k+- = 1, M = 200 steps to T = 1, u0 = 0, source = 8 moving bumps
    evaluated at t_{m-1/2}, tol 1e-8."""
    rng = np.random.default_rng(seed)
    delta = list(rng.uniform(0.2, 0.8, 3))
    bumps = moving_bumps(seed + 7919)
    return Workload(f"learned_{seed}_{n}", 3, [n, n, n], delta, [1.0] * 3, [1.0] * 3,
                    M, 1.0, 1e-8, "pcg", np.zeros((n, n, n)), None, bumps)


def random_grid(shape, seed: int):
    """Standard-normal test vector of the given grid shape."""
    return np.random.default_rng(seed).standard_normal(shape)


def nn_initial_params(seed: int, layers) -> np.ndarray:
    """He-uniform initial weights for a stack of 3x3x3 convolutions, biases
    zero; the last layer starts at zero (the initial prediction is the
    network's residual base).  layers: sequence of (c_in, c_out).  Flat
    float32 vector, per layer W[o, i, 3, 3, 3] (C order) then b[o]."""
    rng = np.random.default_rng(seed)
    parts = []
    for k, (ci, co) in enumerate(layers):
        lim = np.sqrt(6.0 / (ci * 27))
        wk = rng.uniform(-lim, lim, co * ci * 27)
        if k == len(layers) - 1:
            wk[:] = 0.0
        parts.append(wk)
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def bumps_source_torch(n, centres, width, device):
    """bumps_source evaluated with torch on `device` (float64): the same
    separable outer products, for sources generated per time step on the
    GPU."""
    import torch
    d = len(n)
    ax = [torch.arange(1, k + 1, dtype=torch.float64, device=device) / (k + 1) for k in n]
    out = torch.zeros(tuple(reversed(n)), dtype=torch.float64, device=device)
    for c in centres:
        g = None
        for i in reversed(range(d)):
            e = torch.exp(-((ax[i] - float(c[i])) ** 2) / (2.0 * width * width))
            g = e if g is None else torch.einsum("...,k->...k", g, e)
        out += g
    return out
