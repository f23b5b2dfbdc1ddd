"""Pins of the reference warm-start network (oracle/nn.py)."""
import numpy as np
import pytest

import workloads
from oracle import nn


def _brute_conv(x, W, b):
    ci, D, H, Wd = x.shape
    co = W.shape[0]
    out = np.zeros((co, D, H, Wd))
    for o in range(co):
        for z in range(D):
            for y in range(H):
                for xx in range(Wd):
                    s = b[o]
                    for i in range(ci):
                        for a in range(3):
                            for c in range(3):
                                for d in range(3):
                                    zz, yy, x3 = z + a - 1, y + c - 1, xx + d - 1
                                    if 0 <= zz < D and 0 <= yy < H and 0 <= x3 < Wd:
                                        s += W[o, i, a, c, d] * x[i, zz, yy, x3]
                    out[o, z, y, xx] = s
    return out


def test_conv_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 3, 5))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    assert np.allclose(nn.conv(x, W, b), _brute_conv(x, W, b), rtol=1e-13, atol=1e-13)


def test_conv_identity_kernel():
    # a centred delta kernel reproduces the input (plus bias)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 5, 4, 6))
    W = np.zeros((3, 3, 3, 3, 3))
    for i in range(3):
        W[i, i, 1, 1, 1] = 1.0
    assert np.array_equal(nn.conv(x, W, np.zeros(3)), x)


def test_conv_backward_finite_difference():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 4, 3))
    W = rng.standard_normal((3, 2, 3, 3, 3))
    b = rng.standard_normal(3)
    g = rng.standard_normal((3, 3, 4, 3))
    gx, gW, gb = nn.conv_backward(x, W, g)
    f = lambda x_, W_, b_: float(np.sum(g * nn.conv(x_, W_, b_)))
    h = 1e-6
    dx = rng.standard_normal(x.shape)
    dW = rng.standard_normal(W.shape)
    db = rng.standard_normal(b.shape)
    # the map is linear in each argument: central differences are exact up to rounding
    assert np.isclose((f(x + h * dx, W, b) - f(x - h * dx, W, b)) / (2 * h), np.sum(gx * dx), rtol=1e-7)
    assert np.isclose((f(x, W + h * dW, b) - f(x, W - h * dW, b)) / (2 * h), np.sum(gW * dW), rtol=1e-7)
    assert np.isclose((f(x, W, b + h * db) - f(x, W, b - h * db)) / (2 * h), np.sum(gb * db), rtol=1e-7)


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 7), (1, 2, 1)])
def test_pool_up_brute_force_and_adjoint(shape):
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2,) + shape)
    p = nn.pool(x)
    cs = nn.coarse(shape)
    assert p.shape == (2,) + cs
    for c in range(2):
        for k in np.ndindex(*cs):
            acc = 0.0
            for o in np.ndindex(2, 2, 2):
                j = tuple(2 * k[i] + o[i] for i in range(3))
                if all(j[i] < shape[i] for i in range(3)):
                    acc += x[(c,) + j]
            assert np.isclose(p[(c,) + k], acc / 8.0, rtol=1e-14)
    u = nn.up(p, shape)
    for c in range(2):
        for j in np.ndindex(*shape):
            assert u[(c,) + j] == p[(c,) + tuple(v // 2 for v in j)]
    y = rng.standard_normal((2,) + shape)
    yc = rng.standard_normal((2,) + cs)
    assert np.isclose(np.sum(nn.up(yc, shape) * y), np.sum(yc * nn.up_backward(y, cs)), rtol=1e-13)
    assert np.isclose(np.sum(nn.pool(y) * yc), np.sum(y * nn.pool_backward(yc, shape)), rtol=1e-13)


def _params(seed=0):
    return workloads.nn_initial_params(seed, [(ci, co) for _, ci, co, _, _ in nn.LAYERS])


def test_param_count_and_layout():
    flat = _params()
    assert flat.size == nn.param_count() == 251649
    d = nn.unflatten(flat)
    assert d["e0"][0].shape == (16, 5, 3, 3, 3) and d["d0"][1].shape == (1,)
    assert not d["d0"][0].any() and not d["d0"][1].any()
    assert np.array_equal(nn.flatten(d), flat.astype(np.float64))


def test_network_gradient_finite_difference():
    rng = np.random.default_rng(4)
    flat = _params(1).astype(np.float64)
    flat += 0.05 * rng.standard_normal(flat.size)   # biases non-zero as well
    shape = (7, 6, 9)
    x = rng.standard_normal((nn.N_IN,) + shape)
    t = rng.standard_normal(shape)
    L, g = nn.loss_and_grad(nn.unflatten(flat), x, t, margin=1)
    for trial in range(3):
        d = rng.standard_normal(flat.size)
        h = 1e-6
        Lp, _ = nn.loss_and_grad(nn.unflatten(flat + h * d), x, t, margin=1)
        Lm, _ = nn.loss_and_grad(nn.unflatten(flat - h * d), x, t, margin=1)
        fd = (Lp - Lm) / (2 * h)
        assert np.isclose(fd, float(g @ d), rtol=1e-5), (trial, fd, float(g @ d))
    # per-layer directions: every layer's gradient block is exercised
    k = 0
    for name, ci, co, _, _ in nn.LAYERS:
        n = co * ci * 27 + co
        d = np.zeros(flat.size)
        d[k:k + n] = rng.standard_normal(n)
        h = 1e-6
        Lp, _ = nn.loss_and_grad(nn.unflatten(flat + h * d), x, t, margin=1)
        Lm, _ = nn.loss_and_grad(nn.unflatten(flat - h * d), x, t, margin=1)
        assert np.isclose((Lp - Lm) / (2 * h), float(g @ d), rtol=1e-5), name
        k += n


def test_features_scale_and_shift_invariance():
    rng = np.random.default_rng(5)
    u, up, F, Fp = (rng.standard_normal((4, 5, 6)) for _ in range(4))
    x1, s1 = nn.features(u, F, 0.01, [2.0, 3.0, 4.0], up, Fp)
    x2, s2 = nn.features(7.0 * u, 7.0 * F, 0.01, [2.0, 3.0, 4.0], 7.0 * up, 7.0 * Fp)
    assert np.allclose(x1, x2, rtol=1e-13, atol=1e-14)
    assert np.isclose(s2, 7.0 * s1, rtol=1e-14)
    # adding the same field to both time levels changes nothing
    c = rng.standard_normal((4, 5, 6))
    x3, s3 = nn.features(u + c, F + c, 0.01, [2.0, 3.0, 4.0], up + c, Fp + c)
    assert np.allclose(x1, x3, rtol=1e-12, atol=1e-12) and np.isclose(s1, s3, rtol=1e-12)
    assert np.allclose(x1[3], np.log(3.0) / 4.0)
    assert np.allclose(x1[0] * s1, u - up)
    assert np.allclose(x1[1] * s1, 0.01 * (F - Fp))


def test_zero_network_is_linear_extrapolation():
    # with the initial (zero) last layer the prediction is 2 u - u_prev
    rng = np.random.default_rng(9)
    u, up, F = (rng.standard_normal((5, 4, 6)) for _ in range(3))
    p = nn.unflatten(_params(3))
    g = nn.predict(p, u, F, 0.02, [1.5, 2.5, 3.5], up, 0.5 * F)
    assert np.allclose(g, 2 * u - up, rtol=0, atol=1e-14)
    t = nn.target(u, up, 2 * u - up, 1.0)
    assert np.allclose(t, 0.0, atol=1e-14)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(6)
    p = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = nn.adam(p, g, np.zeros(10), np.zeros(10), 1, lr=1e-3, eps=0.0)
    assert np.allclose(p1, p - 1e-3 * np.sign(g), rtol=1e-15, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bumps_source_torch_matches_numpy():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    c = rng.uniform(0.2, 0.8, (3, 3))
    a = workloads.bumps_source([9, 7, 5], c, 0.1)
    b = workloads.bumps_source_torch([9, 7, 5], c, 0.1, "cpu").numpy()
    assert np.allclose(a, b, rtol=1e-14, atol=1e-300)
