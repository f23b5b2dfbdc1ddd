"""Manufactured solutions of Examples 4.1 (2D) and 4.2 (3D), Section 4.

Test infrastructure only (see the package docstring).

The sources are derived here from the Riemann-Liouville definitions
(Section 1) rather than transcribed: for a polynomial profile
p(x) = sum_m c_m x^m = sum_m d_m (1-x)^m on (0,1), extended by zero,

    d/dx [k_+ d^{1-delta}_x p - k_- d^{1-delta}_{-x} p]
      = k_+ sum_m c_m Gamma(m+1)/Gamma(m+delta-1) x^(m+delta-2)
      + k_- sum_m d_m Gamma(m+1)/Gamma(m+delta-1) (1-x)^(m+delta-2),

valid for profiles with p(0) = p(1) = 0 and no constant or linear term at
the ends (both examples use x^2 (1-x)^2).  The printed source formulas are
checked against this in the tests.
"""
from __future__ import annotations

import math

import numpy as np

# x^2 (1-x)^2 = x^2 - 2 x^3 + x^4, symmetric under x -> 1-x
_PROFILE = {2: 1.0, 3: -2.0, 4: 1.0}


def profile(x):
    return x ** 2 * (1.0 - x) ** 2


def flux_derivative(x, delta: float, kp: float, km: float, coeffs=_PROFILE):
    """d/dx D^delta p for p = sum c_m x^m (and, by the symmetry of the
    profile, the same coefficients in powers of (1-x))."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for m, c in coeffs.items():
        g = math.gamma(m + 1) / math.gamma(m + delta - 1)
        out = out + kp * c * g * x ** (m + delta - 2) + km * c * g * (1.0 - x) ** (m + delta - 2)
    return out


def ex41_exact(x, y, t):
    """u = 4 e^t x^2(1-x)^2 y^2(1-y)^2 (Example 4.1)."""
    return 4.0 * math.exp(t) * profile(x) * profile(y)


def ex41_source(x, y, t, delta, kp, km):
    """f = u_t - d_x D_x u - d_y D_y u for Example 4.1."""
    X, Y = profile(x), profile(y)
    return 4.0 * math.exp(t) * (X * Y
                                - Y * flux_derivative(x, delta[0], kp[0], km[0])
                                - X * flux_derivative(y, delta[1], kp[1], km[1]))


def ex42_exact(x, y, z, t):
    """u = sin(t+1) x^2(1-x)^2 y^2(1-y)^2 z^2(1-z)^2 (Example 4.2)."""
    return math.sin(t + 1.0) * profile(x) * profile(y) * profile(z)


def ex42_source(x, y, z, t, delta, kp, km):
    """f = u_t - sum_i d_i D_i u for Example 4.2."""
    X, Y, Z = profile(x), profile(y), profile(z)
    return (math.cos(t + 1.0) * X * Y * Z
            - math.sin(t + 1.0) * (Y * Z * flux_derivative(x, delta[0], kp[0], km[0])
                                   + X * Z * flux_derivative(y, delta[1], kp[1], km[1])
                                   + X * Y * flux_derivative(z, delta[2], kp[2], km[2])))


def ex42_source_parts(x, y, z, delta, kp, km):
    """(P, D) with f = cos(t+1) P - sin(t+1) D for Example 4.2: the source
    separates into two functions of space, so its cell averages at every
    step are two fixed grids combined with cos(t+1) and sin(t+1) (the cell
    average is linear).  Example 4.1's source is e^t times its value at
    t = 0 in the same way."""
    X, Y, Z = profile(x), profile(y), profile(z)
    P = X * Y * Z
    D = (Y * Z * flux_derivative(x, delta[0], kp[0], km[0])
         + X * Z * flux_derivative(y, delta[1], kp[1], km[1])
         + X * Y * flux_derivative(z, delta[2], kp[2], km[2]))
    return P, D


def ex41_source_printed(x, y, t, delta, kp, km):
    """The source of Example 4.1 in the paper's own form (binomial sum over
    k = 0..2 of Gamma(5-k)/Gamma(3-k+alpha) times the two one-sided powers);
    used only to check :func:`ex41_source`."""
    X, Y = profile(x), profile(y)

    def term(s, d, kpl, kmi):
        acc = 0.0
        for k in range(3):
            c = (-1.0) ** (2 - k) * math.comb(2, k) * math.gamma(5 - k) / math.gamma(3 - k + d)
            acc = acc + c * (kpl * s ** (2 - k + d) + kmi * (1.0 - s) ** (2 - k + d))
        return acc

    return 4.0 * math.exp(t) * (X * Y - Y * term(x, delta[0], kp[0], km[0])
                                - X * term(y, delta[1], kp[1], km[1]))


_GL4_X, _GL4_W = np.polynomial.legendre.leggauss(4)


def cell_average(f, n, h, a=None):
    """F_{i..} = (1/prod h) * integral of f over the control volume
    [x_{i-1/2}, x_{i+1/2}] x ... (Section 2, definition of F^{m-1/2}), by
    4-point Gauss-Legendre per axis.  f takes d coordinate arrays (x first);
    returns an array of shape (n_d, ..., n_1)."""
    d = len(n)
    a = a or [0.0] * d
    grids = []
    wts = []
    for i in range(d):
        centres = a[i] + h[i] * np.arange(1, n[i] + 1)
        pts = centres[:, None] + 0.5 * h[i] * _GL4_X[None, :]   # (n_i, 4)
        grids.append(pts)
        wts.append(0.5 * _GL4_W)
    if d == 2:
        X = grids[0][None, :, None, :]
        Y = grids[1][:, None, :, None]
        vals = f(X, Y)                                  # (n2, n1, 4, 4)
        W = wts[1][:, None] * wts[0][None, :]
        return np.einsum("abij,ij->ab", vals, W)
    X = grids[0][None, None, :, None, None, :]
    Y = grids[1][None, :, None, None, :, None]
    Z = grids[2][:, None, None, :, None, None]
    vals = f(X, Y, Z)                                   # (n3, n2, n1, 4, 4, 4)
    W = wts[2][:, None, None] * wts[1][None, :, None] * wts[0][None, None, :]
    return np.einsum("abcijk,ijk->abc", vals, W)


def cell_average_1d(f, n: int, h: float, a: float = 0.0):
    """(1/h) * integral of f over [x_{i-1/2}, x_{i+1/2}], i = 1..n, by the
    same 4-point Gauss-Legendre rule: the one-dimensional factor of
    :func:`cell_average`, whose tensor-product rule averages a product of
    functions of one coordinate each as the product of these averages."""
    centres = a + h * np.arange(1, n + 1)
    pts = centres[:, None] + 0.5 * h * _GL4_X[None, :]
    return f(pts) @ (0.5 * _GL4_W)


def ex41_source_cells(n, h, delta, kp, km):
    """Cell averages of Example 4.1's source at t = 0 (e^t times this at time
    t), assembled from one-dimensional averages: the source is
    4 (X Y - Y g_x - X g_y) with X, Y the profile and g the flux derivative
    of one coordinate each (:func:`ex41_source`), so its tensor-product
    Gauss average is 4 (avg X avg Y - avg Y avg g_x - avg X avg g_y).
    Shape (n_2, n_1)."""
    X = cell_average_1d(profile, n[0], h[0])
    Y = cell_average_1d(profile, n[1], h[1])
    gx = cell_average_1d(lambda x: flux_derivative(x, delta[0], kp[0], km[0]), n[0], h[0])
    gy = cell_average_1d(lambda y: flux_derivative(y, delta[1], kp[1], km[1]), n[1], h[1])
    return 4.0 * (np.outer(Y, X) - np.outer(Y, gx) - np.outer(gy, X))


def ex42_source_parts_cells(n, h, delta, kp, km):
    """Cell averages (P, D) of :func:`ex42_source_parts` from one-dimensional
    averages (every term is a product of functions of one coordinate).
    Shapes (n_3, n_2, n_1)."""
    avg = [cell_average_1d(profile, n[i], h[i]) for i in range(3)]
    g = [cell_average_1d(lambda s, i=i: flux_derivative(s, delta[i], kp[i], km[i]), n[i], h[i])
         for i in range(3)]

    def outer3(fx, fy, fz):
        return fz[:, None, None] * fy[None, :, None] * fx[None, None, :]

    P = outer3(avg[0], avg[1], avg[2])
    D = outer3(g[0], avg[1], avg[2]) + outer3(avg[0], g[1], avg[2]) + outer3(avg[0], avg[1], g[2])
    return P, D


def nodal(f, n, h, a=None):
    """f at the interior nodes, shape (n_d, ..., n_1)."""
    d = len(n)
    a = a or [0.0] * d
    axes = [a[i] + h[i] * np.arange(1, n[i] + 1) for i in range(d)]
    mesh = np.meshgrid(*reversed(axes), indexing="ij")   # z, y, x order
    return f(*reversed(mesh))
