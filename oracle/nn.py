"""Reference 3D convolution network of the learned warm start (float64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The warm start is not part of the paper: it is an extension that predicts
the next Crank-Nicolson iterate u^{m} so that the Krylov solve of Section 3
starts closer to its solution.  It corrects the linear extrapolation
2 u^{m-1} - u^{m-2}.  The Crank-Nicolson matrices do not change with m, so
the extrapolation error u^m - 2 u^{m-1} + u^{m-2} is A^{-1} applied to
dt (F^{m-1/2} - F^{m-3/2}) - 2 K (u^{m-1} - u^{m-2}): a linear map of the
last increment and the last change of the source, which is what the
network sees.  This module is the plain definition of that network,
written out in NumPy:

* features: x = [du / s, dt dF / s, log(eta_1)/4, log(eta_2)/4,
  log(eta_3)/4] with du = u^{m-1} - u^{m-2}, dF = F^{m-1/2} - F^{m-3/2}
  and s = rms(du) + rms(dt dF) (+1e-30), on the n_3 x n_2 x n_1 grid; the
  first step has no history (du = 0, dF = F);
* a four-level U-shaped network (levels 0..3, each level half the size of
  the previous one, rounded up):

      e0 = relu(conv(x, 5 -> 16))                  level 0
      e1 = relu(conv(pool(e0), 16 -> 32))          level 1
      e2 = relu(conv(pool(e1), 32 -> 64))          level 2
      e3 = relu(conv(pool(e2), 64 -> 64))          level 3
      d2 = relu(conv(up(e3) + e2, 64 -> 32))       level 2
      d1 = relu(conv(up(d2) + e1, 32 -> 16))       level 1
      y  = conv(up(d1) + e0, 16 -> 1)              level 0

  conv: 3x3x3 cross-correlation with zero padding and a bias,
      out[o, z, y, x] = b[o] + sum_{i, a, c, d} W[o, i, a, c, d] in[i, z+a-1, y+c-1, x+d-1];
  pool: 2x2x2 average with stride 2, out size ceil(n/2), absent inputs zero;
  up:   nearest-neighbour, out[j] = in[j // 2], cropped to the finer size;
* prediction: guess = u + (u - u_prev) + s * y, the linear extrapolation in
  time corrected by the network.

Training minimises the mean squared error between y and the scaled
extrapolation error t = (u^{m} - 2 u^{m-1} + u^{m-2}) / s over an interior
region, with Adam (Kingma and Ba, 2015).

Pins (tests/test_oracle_nn.py): conv against a brute-force loop; pool and
up against their adjoint identities and brute force; the backward pass
against central finite differences of the loss; Adam's first step against
its closed form lr * sign(g).
"""
from __future__ import annotations

import numpy as np

# name, input channels, output channels, level, relu
LAYERS = (
    ("e0", 5, 16, 0, True),
    ("e1", 16, 32, 1, True),
    ("e2", 32, 64, 2, True),
    ("e3", 64, 64, 3, True),
    ("d2", 64, 32, 2, True),
    ("d1", 32, 16, 1, True),
    ("d0", 16, 1, 0, False),
)
N_IN = 5


def param_count():
    return sum(co * ci * 27 + co for _, ci, co, _, _ in LAYERS)


def unflatten(flat):
    """Flat parameter vector (per layer: W[o, i, 3, 3, 3] in C order, then
    b[o]) -> dict name -> (W, b)."""
    flat = np.asarray(flat, dtype=np.float64)
    out, k = {}, 0
    for name, ci, co, _, _ in LAYERS:
        nw = co * ci * 27
        W = flat[k:k + nw].reshape(co, ci, 3, 3, 3)
        k += nw
        b = flat[k:k + co]
        k += co
        out[name] = (W, b)
    assert k == flat.size
    return out


def flatten(d):
    return np.concatenate([np.concatenate([d[name][0].ravel(), d[name][1].ravel()])
                           for name, *_ in LAYERS])


# ------------------------------------------------------------------ layers

def conv(x, W, b):
    """3x3x3 zero-padded cross-correlation.  x: (ci, D, H, W)."""
    ci, D, H, Wd = x.shape
    co = W.shape[0]
    xp = np.zeros((ci, D + 2, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    out = np.empty((co, D, H, Wd))
    out[:] = b[:, None, None, None]
    for a in range(3):
        for c in range(3):
            for d in range(3):
                win = xp[:, a:a + D, c:c + H, d:d + Wd].reshape(ci, -1)
                out += (W[:, :, a, c, d] @ win).reshape(co, D, H, Wd)
    return out


def conv_backward(x, W, gout):
    """Gradients of sum(gout * conv(x, W, b)) w.r.t. x, W and b."""
    ci, D, H, Wd = x.shape
    co = W.shape[0]
    xp = np.zeros((ci, D + 2, H + 2, Wd + 2))
    xp[:, 1:-1, 1:-1, 1:-1] = x
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    g2 = gout.reshape(co, -1)
    for a in range(3):
        for c in range(3):
            for d in range(3):
                win = xp[:, a:a + D, c:c + H, d:d + Wd].reshape(ci, -1)
                gW[:, :, a, c, d] = g2 @ win.T
                gxp[:, a:a + D, c:c + H, d:d + Wd] += (W[:, :, a, c, d].T @ g2).reshape(ci, D, H, Wd)
    gb = g2.sum(axis=1)
    return gxp[:, 1:-1, 1:-1, 1:-1], gW, gb


def coarse(shape):
    return tuple((s + 1) // 2 for s in shape)


def pool(x):
    """2x2x2 average, stride 2, output size ceil(n/2), absent inputs zero."""
    c = x.shape[0]
    D, H, Wd = x.shape[1:]
    Dc, Hc, Wc = coarse((D, H, Wd))
    xp = np.zeros((c, 2 * Dc, 2 * Hc, 2 * Wc))
    xp[:, :D, :H, :Wd] = x
    return xp.reshape(c, Dc, 2, Hc, 2, Wc, 2).mean(axis=(2, 4, 6))


def pool_backward(gout, fine_shape):
    c, Dc, Hc, Wc = gout.shape
    g = np.repeat(np.repeat(np.repeat(gout, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0
    D, H, Wd = fine_shape
    return g[:, :D, :H, :Wd]


def up(x, fine_shape):
    """Nearest-neighbour upsampling, out[j] = in[j // 2]."""
    g = np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)
    D, H, Wd = fine_shape
    return g[:, :D, :H, :Wd]


def up_backward(gout, coarse_shape):
    c, D, H, Wd = gout.shape
    Dc, Hc, Wc = coarse_shape
    gp = np.zeros((c, 2 * Dc, 2 * Hc, 2 * Wc))
    gp[:, :D, :H, :Wd] = gout
    return gp.reshape(c, Dc, 2, Hc, 2, Wc, 2).sum(axis=(2, 4, 6))


def relu(x):
    return np.maximum(x, 0.0)


# ------------------------------------------------------------------ network

def features(u, F, dt, eta, u_prev=None, F_prev=None):
    """Network input and scale s at step m: u = u^{m-1}, u_prev = u^{m-2},
    F = F^{m-1/2}, F_prev = F^{m-3/2} (None: no history / zero source)."""
    u = np.asarray(u, dtype=np.float64)
    z = np.zeros_like(u)
    du = z if u_prev is None else u - np.asarray(u_prev, dtype=np.float64)
    f = z if F is None else np.asarray(F, dtype=np.float64)
    fp = z if F_prev is None else np.asarray(F_prev, dtype=np.float64)
    df = dt * (f - fp)
    s = np.sqrt(np.mean(du * du)) + np.sqrt(np.mean(df * df)) + 1e-30
    x = np.empty((N_IN,) + u.shape)
    x[0] = du / s
    x[1] = df / s
    for i in range(3):
        x[2 + i] = np.log(eta[i]) / 4.0
    return x, s


def forward(params, x):
    """params: dict from unflatten; x: (5, D, H, W).  Returns (y, acts) with
    y of shape (D, H, W) and the intermediate activations for backward."""
    p = params
    a = {"x": x}
    a["e0"] = relu(conv(x, *p["e0"]))
    a["p1"] = pool(a["e0"])
    a["e1"] = relu(conv(a["p1"], *p["e1"]))
    a["p2"] = pool(a["e1"])
    a["e2"] = relu(conv(a["p2"], *p["e2"]))
    a["p3"] = pool(a["e2"])
    a["e3"] = relu(conv(a["p3"], *p["e3"]))
    a["s2"] = up(a["e3"], a["e2"].shape[1:]) + a["e2"]
    a["d2"] = relu(conv(a["s2"], *p["d2"]))
    a["s1"] = up(a["d2"], a["e1"].shape[1:]) + a["e1"]
    a["d1"] = relu(conv(a["s1"], *p["d1"]))
    a["s0"] = up(a["d1"], a["e0"].shape[1:]) + a["e0"]
    y = conv(a["s0"], *p["d0"])[0]
    return y, a


def backward(params, acts, gy):
    """Gradient of sum(gy * y) with respect to every parameter."""
    p = params
    a = acts
    g = {}
    gs0, gW, gb = conv_backward(a["s0"], p["d0"][0], gy[None])
    g["d0"] = (gW, gb)
    ge0 = gs0.copy()
    gd1 = up_backward(gs0, a["d1"].shape[1:]) * (a["d1"] > 0)
    gs1, gW, gb = conv_backward(a["s1"], p["d1"][0], gd1)
    g["d1"] = (gW, gb)
    ge1 = gs1.copy()
    gd2 = up_backward(gs1, a["d2"].shape[1:]) * (a["d2"] > 0)
    gs2, gW, gb = conv_backward(a["s2"], p["d2"][0], gd2)
    g["d2"] = (gW, gb)
    ge2 = gs2.copy()
    ge3 = up_backward(gs2, a["e3"].shape[1:]) * (a["e3"] > 0)
    gp3, gW, gb = conv_backward(a["p3"], p["e3"][0], ge3)
    g["e3"] = (gW, gb)
    ge2 = (ge2 + pool_backward(gp3, a["e2"].shape[1:])) * (a["e2"] > 0)
    gp2, gW, gb = conv_backward(a["p2"], p["e2"][0], ge2)
    g["e2"] = (gW, gb)
    ge1 = (ge1 + pool_backward(gp2, a["e1"].shape[1:])) * (a["e1"] > 0)
    gp1, gW, gb = conv_backward(a["p1"], p["e1"][0], ge1)
    g["e1"] = (gW, gb)
    ge0 = (ge0 + pool_backward(gp1, a["e0"].shape[1:])) * (a["e0"] > 0)
    _, gW, gb = conv_backward(a["x"], p["e0"][0], ge0)
    g["e0"] = (gW, gb)
    return g


def interior(shape, margin):
    m = np.zeros(shape, dtype=bool)
    sl = tuple(slice(margin, s - margin) for s in shape)
    m[sl] = True
    return m


def loss_and_grad(params, x, t, margin=0):
    """Mean squared error over the interior (margin cells dropped on every
    side) and its gradient with respect to the flat parameter vector."""
    y, acts = forward(params, x)
    m = interior(y.shape, margin)
    cnt = m.sum()
    r = (y - t) * m
    L = float((r * r).sum() / cnt)
    g = backward(params, acts, 2.0 * r / cnt)
    return L, flatten(g)


def target(u, u_prev, u_next, s):
    """Scaled extrapolation error (u_next - 2 u + u_prev) / s."""
    up = u if u_prev is None else u_prev
    return (u_next - 2.0 * u + up) / s


def predict(params, u, F, dt, eta, u_prev=None, F_prev=None):
    """guess = u + (u - u_prev) + s * y."""
    x, s = features(u, F, dt, eta, u_prev, F_prev)
    y, _ = forward(params, x)
    du = 0.0 if u_prev is None else u - u_prev
    return u + du + s * y


def adam(p, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
