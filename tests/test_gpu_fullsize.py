"""Parity at the benchmark's full size, 255^3 (the 3D non-symmetric
workload: the shapes and launch configuration `bench.py` times).

The float64 operator is checked on sampled outputs the oracle computes one
by one (`apply_A_at`: one row per axis contracted with the whole grid), the
preconditioners against the oracle's full sine transforms (scipy DST-I over
the 255^3 grid), and one mixed-precision CN step by a property: its
residual, sampled with the oracle's rows, is at the solver tolerance.

Tolerances: float64 1e-12 relative (round-off of FFTs of length 512);
float32 preconditioner 1e-5 relative 2-norm (float32 round-off over the
transforms); the sampled residual of the step <= 1e-7 of max |b| (the
solves stop at 1e-8 relative in the preconditioned norm, and P^{-1} is
well conditioned, Theorem 3.1).
"""
import numpy as np
import pytest

import workloads
from oracle import operators as op

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
        assert _relerr(z, ref) <= 1e-12
    else:
        z = _host(prob.apply_Pinv32(_dev(X)))
        assert _relerr(z, ref) <= 1e-5


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
