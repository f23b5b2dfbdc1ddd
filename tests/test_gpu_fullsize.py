"""Parity at the benchmark's full size, 255^3 (the 3D non-symmetric
workload: the shapes and launch configuration `bench.py` times).

The float64 operator is checked on sampled outputs the oracle computes one
by one (`apply_A_at`: one row per axis contracted with the whole grid), the
preconditioners against the oracle's full sine transforms (scipy DST-I over
the 255^3 grid), and one mixed-precision CN step by a property: its
residual, sampled with the oracle's rows, is at the solver tolerance.

The float32 operators of the mixed-precision inner solve (matvec and
preconditioner) are compared with the oracle's full 255^3 results, and two
CN steps of the headline configuration (mixed precision at the benchmark's
settings) with the oracle's tightly solved steps.

Tolerances: float64 1e-12 relative (round-off of FFTs of length 512);
float32 operators 1e-5 (float32 round-off over the transforms); the
sampled residual of the step <= 1e-7 of max |b| (the solves stop at 1e-8
relative in the preconditioned norm, and P^{-1} is well conditioned,
Theorem 3.1); the headline steps 1e-8.  Every full-grid comparison holds in
the relative 2-norm and in the relative max-norm (max |a - b| / max |b|).
"""
import os
import time

import numpy as np
import pytest
import scipy.fft as sfft

import workloads
from oracle import cn, operators as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 255


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_21198_amd.solver import Problem
    w = workloads.config_3d_nonsymmetric(seed=0, n=N, M=16)
    orc = op.Problem(3, w.n, w.delta, w.kplus, w.kminus, T=w.T, M=w.M)
    return Problem, w, orc


def _samples(shape, count, seed):
    """Corner, edge and face points plus seeded random interior points."""
    rng = np.random.default_rng(seed)
    n = shape[0] - 1
    idx = [(0, 0, 0), (n, n, n), (0, n, 0), (n, 0, n), (0, 0, n), (n // 2, 0, n // 2),
           (n // 2, n // 2, n), (1, n - 1, 1)]
    idx += [tuple(int(v) for v in rng.integers(0, shape[0], 3)) for _ in range(count)]
    return idx


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _relerr(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _close(a, b, bound):
    e2 = _relerr(a, b)
    em = float(np.abs(a - b).max() / np.abs(b).max())
    assert e2 <= bound and em <= bound, (e2, em, bound)


def test_operator_sampled(setup):
    Problem, w, orc = setup
    prob = Problem(3, w.n, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="gmres")
    X = workloads.random_grid(orc.shape, 31)
    Y = _host(prob.apply_A(_dev(X)))
    scale = np.abs(Y).max()
    for idx in _samples(orc.shape, 24, 5):
        assert abs(Y[idx] - op.apply_A_at(orc, X, idx)) <= 1e-12 * scale, idx


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_preconditioner_full(setup, precision):
    Problem, w, orc = setup
    prob = Problem(3, w.n, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="gmres",
                   precision=precision)
    X = workloads.random_grid(orc.shape, 32)
    ref = op.apply_Pinv(orc, X)
    if precision == "fp64":
        z = _host(prob.apply_Pinv(_dev(X)))
        _close(z, ref, 1e-12)
    else:
        z = _host(prob.apply_Pinv32(_dev(X)))
        _close(z, ref, 1e-5)


def test_float32_matvec_full(setup):
    """The float32 matvec of the inner solve on the full grid: the wave
    engine's x pass and the column engine's y and z passes (length 512)
    against the oracle's A X (the bound is derived in
    test_gpu_parity.test_float32_matvec)."""
    Problem, w, orc = setup
    prob = Problem(3, w.n, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="gmres",
                   precision="mixed")
    X = workloads.random_grid(orc.shape, 34)
    _close(_host(prob.apply_A32(_dev(X))), op.apply_A(orc, X), 1e-5)


@pytest.mark.timeout(900)
def test_headline_steps_vs_oracle(setup):
    """Two CN steps of the benchmark's headline configuration (3D
    non-symmetric 255^3, u0 = 0, the seeded bump source; left GMRES(20),
    mixed precision at the benchmark's tolerance, inner tolerance and warm
    start) against the oracle's steps solved to 1e-11 on the host: within
    1e-8 in the relative 2-norm and max-norm.  The float64 solver at the same
    tolerance is held to the same bound.  The oracle takes one to two
    minutes (its DST-I runs on every host core; the worker count does not
    change its results)."""
    Problem, w, orc = setup
    S = workloads.HEADLINE_SOLVER
    steps = 2
    F = _dev(w.F)
    outs = {}
    for precision in ("mixed", "fp64"):
        kw = dict(S)
        if precision == "fp64":
            kw.pop("inner_tol")
            kw.pop("max_outer")
        prob = Problem(3, w.n, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="gmres",
                       precision=precision, **kw)
        u = _dev(w.u0)
        for _ in range(steps):
            u, st = prob.cn_step(u, F)
            assert st["converged"] == 1
        outs[precision] = _host(u)
        del prob
    t0 = time.perf_counter()
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    with sfft.set_workers(min(cores, 16)):
        ref, its = cn.run(orc, w.u0, lambda m: w.F, tol=1e-11, x0_mode="prev", solver="gmres",
                          steps=steps)
    print(f"oracle: {steps} steps, iterations {its}, {time.perf_counter() - t0:.1f} s")
    for precision, u in outs.items():
        _close(u, ref, 1e-8)


def test_mixed_step_residual_sampled(setup):
    Problem, w, orc = setup
    prob = Problem(3, w.n, w.delta, w.kplus, w.kminus, M=w.M, T=w.T, solver="gmres",
                   restart=20, tol=w.tol, precision="mixed", inner_tol=1e-4)
    rng = np.random.default_rng(33)
    u0 = rng.standard_normal(orc.shape)
    F = w.F
    u1, st = prob.cn_step(_dev(u0), _dev(F))
    u1 = _host(u1)
    assert st["status"] == 0
    scale = None
    worst = 0.0
    for idx in _samples(orc.shape, 12, 6):
        b = op.apply_A_at(orc, u0, idx, -1.0) + orc.dt * F[idx]
        r = b - op.apply_A_at(orc, u1, idx)
        worst = max(worst, abs(r))
        scale = max(scale or 0.0, abs(b))
    assert worst <= 1e-7 * scale, (worst, scale)
