"""Comparator preconditioners of Section 4 on the HIP path (through the C
ABI): no preconditioner, T. Chan's and Strang's circulants (every Toeplitz
factor replaced by its circulant; P^{-1} by Bluestein DFT passes).

Parity: one application of P^{-1} against the oracle's ifftn(fftn(r) /
Lambda) to 1e-12 (relative 2-norm; float64 DFTs of length n by FFTs of
length M <= 2048, round-off about eps log2 M per transform), CN steps
against the stopping test evaluated by the oracle, and the printed
comparator iteration counts of Tables 1-4 in the replication setting
(x0 = 0, tol 1e-9, restart 20), most of them exactly.

Tolerance of the printed counts (iterations summed over the M steps): two,
or 0.1% of the total, for CG and GMRES without preconditioner and for every
GMRES comparator; 4% for the circulant-preconditioned CG rows of the
symmetric tables.  There the preconditioned spectrum has outliers (Strang's
circulant at (alpha, beta) = (0.1, 0.2), n = 63: eigenvalues of P from 1.6
to 6089), CG converges slowly near the threshold, and where the residual of
a step ends within rounding of tol the count moves by one; the paper notes
the slow convergence of PCG(T) and PCG(S) for small and anisotropic orders.
Measured: 168 of the 188 entries exact, the largest difference -3.2%
(PCG(S), (0.1, 0.2), 511^2).

Against the oracle itself at the sizes its own tests do not reach (the
symmetric circulant rows, 128^2 to 511^2 and 32^3, 64^3; the oracle's
counts are within 0.74% of the printed ones there): 25 of 40 rows equal in
every step, all 3D rows among them; every step within 4 iterations and
every total within 2.5% (measured: 2.4%, (0.1, 0.2) PCG(S) at 511^2).
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle import circulant as circ, cn, examples as ex, operators as op

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def fsd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2511_21198_amd.solver import Problem
    return Problem


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def relerr(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))


PINV_CASES = [
    # dim, n, kplus, kminus: symmetric and not, ragged rows (n1 = 95: 96
    # columns), a degenerate axis, the largest line (n = 1023, M = 2048)
    (2, [63, 47], [5, 5], [5, 5]),
    (2, [95, 15], [19, 21], [21, 23]),
    (2, [1023, 7], [1.0, 2.0], [0.5, 1.0]),
    (3, [31, 23, 15], [1, 1, 1], [1, 1, 1]),
    (3, [15, 31, 7], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3]),
    (3, [1, 2, 3], [1, 2, 3], [2, 2, 2]),
    (3, [127, 127, 127], [19, 21, 23], [21, 23, 25]),
    (3, [255, 255, 255], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3]),   # the benchmark grid
]


@pytest.mark.parametrize("kind", ["tchan", "strang"])
@pytest.mark.parametrize("case", PINV_CASES, ids=lambda c: f"{c[0]}d-" + "x".join(map(str, c[1])))
def test_circulant_pinv_vs_oracle(fsd, case, kind):
    dim, n, kp, km = case
    d = [0.3, 0.6, 0.8][:dim]
    prob = fsd(dim, n, d, kp, km, M=4, T=1.0, precond=kind)
    orc = op.Problem(dim, n, d, kp, km, T=1.0, M=4)
    R = workloads.random_grid(orc.shape, 61)
    z = host(prob.apply_Pinv(dev(R)))
    ref = circ.apply_Pinv(orc, R, circ.precond_eigs(orc, kind))
    assert relerr(z, ref) <= 1e-12


def test_no_preconditioner_is_identity(fsd):
    prob = fsd(3, [15, 7, 31], [0.3, 0.6, 0.8], [1, 1, 1], [1, 1, 1], precond="none")
    R = workloads.random_grid((31, 7, 15), 62)
    assert np.array_equal(host(prob.apply_Pinv(dev(R))), R)


@pytest.mark.parametrize("kind", ["none", "tchan", "strang"])
@pytest.mark.parametrize("case", [
    (2, [63, 47], [0.4, 0.7], [5, 5], [5, 5]),
    (2, [31, 63], [0.2, 0.9], [19, 21], [21, 23]),
    (3, [15, 23, 7], [0.3, 0.5, 0.7], [1, 1, 1], [1, 1, 1]),
    (3, [7, 15, 11], [0.4, 0.6, 0.8], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3]),
], ids=lambda c: f"{c[0]}d-" + "x".join(map(str, c[1])))
def test_comparator_cn_steps_vs_oracle(fsd, case, kind):
    """Three CN steps from u^{m-1} (PCG when symmetric, left GMRES(20)
    otherwise).  A Krylov solution is any iterate that meets the stopping
    test, so each GPU step is checked against that test evaluated by the
    oracle from the GPU's own previous state: ||b - A u|| <= tol ||b|| (PCG),
    ||P^{-1}(b - A u)|| <= tol ||P^{-1} b|| (left GMRES; P = I without a
    preconditioner), with 1.5 tol for the gap between the solver's recursive
    residual and the true one.  Iteration counts are within one of the
    oracle's; the final state is within 1e-6 of the oracle's tight solve
    (the error bound kappa(A) tol of an unpreconditioned solve)."""
    dim, n, d, kp, km = case
    M, tol = 3, 1e-11
    orc = op.Problem(dim, n, d, kp, km, T=1.0, M=M)
    u0 = np.random.default_rng(63).standard_normal(orc.shape)
    F = workloads.random_grid(orc.shape, 64)
    prob = fsd(dim, n, d, kp, km, M=M, T=1.0, tol=tol, precond=kind)
    minv = circ.minv(orc, kind)
    u_prev = u0
    its = []
    for _ in range(M):
        u_gpu, st = prob.cn_step(dev(u_prev), dev(F))
        u = host(u_gpu)
        its.append(st["iters"])
        b = op.apply_rhs(orc, u_prev, F)
        r = b - op.apply_A(orc, u)
        if orc.symmetric:
            q = np.linalg.norm(r) / np.linalg.norm(b)
        else:
            q = np.linalg.norm(minv(r)) / np.linalg.norm(minv(b))
        assert q <= 1.5 * tol, (q, st)
        u_prev = u
    _, its_ref = cn.run(orc, u0, lambda m: F, tol=tol, x0_mode="prev", precond=kind)
    assert all(abs(a - b) <= 1 for a, b in zip(its, its_ref)), (its, its_ref)
    u_ref, _ = cn.run(orc, u0, lambda m: F, tol=1e-13, x0_mode="prev", precond=kind)
    assert relerr(u_prev, u_ref) <= 1e-6


def test_circulant_rejects_mixed_and_two_sided(fsd):
    from paper_2511_21198_amd._native import FsdError
    with pytest.raises(FsdError):
        fsd(2, [7, 7], [0.5, 0.5], [1, 1], [1, 1], precision="mixed", precond="tchan")
    with pytest.raises(FsdError):
        fsd(2, [7, 7], [0.5, 0.5], [1, 2], [2, 1], solver="gmres2", precond="strang")


def _rows():
    rows = json.load(open(os.path.join(GOLDEN, "paper_comparator_iterations.json")))["rows"]
    out = []
    for tab, dim, orders, M, n1, none, tchan, strang in rows:
        for kind, it in (("none", none), ("tchan", tchan), ("strang", strang)):
            if it is not None:
                out.append((tab, dim, tuple(orders), M, n1, kind, it))
    return out


_TOTALS = {}
_SOURCE = {}   # the example's initial state and per-step sources of the last problem


def _example(tab, dim, orders, M, n1):
    key = (tab, dim, orders, M, n1)
    if key not in _SOURCE:
        sym = tab in (1, 3)
        kp = [5.0] * dim if sym else [19.0, 21.0, 23.0][:dim]
        km = [5.0] * dim if sym else [21.0, 23.0, 25.0][:dim]
        orc = op.Problem(dim, [n1 - 1] * dim, list(orders), kp, km, T=1.0, M=M)
        h = orc.h
        if dim == 2:
            Fs = [ex.cell_average(lambda X, Y: ex.ex41_source(
                X, Y, (m - 0.5) * orc.dt, orc.delta, kp, km), orc.n, h) for m in range(1, M + 1)]
            u0 = ex.nodal(lambda X, Y: ex.ex41_exact(X, Y, 0.0), orc.n, h)
        else:
            Fs = [ex.cell_average(lambda X, Y, Z: ex.ex42_source(
                X, Y, Z, (m - 0.5) * orc.dt, orc.delta, kp, km), orc.n, h) for m in range(1, M + 1)]
            u0 = ex.nodal(lambda X, Y, Z: ex.ex42_exact(X, Y, Z, 0.0), orc.n, h)
        _SOURCE.clear()
        _SOURCE[key] = (kp, km, u0, Fs)
    return _SOURCE[key]


_STEPS = {}   # (table, dim, orders, M, n + 1, kind) -> iterations of each CN step


def _run_steps(fsd, key):
    if key not in _STEPS:
        tab, dim, orders, M, n1, kind = key
        kp, km, u0, Fs = _example(tab, dim, orders, M, n1)
        prob = fsd(dim, [n1 - 1] * dim, list(orders), kp, km, M=M, T=1.0, tol=1e-9, x0="zero",
                   restart=20, maxit=(n1 - 1) ** 3, precond=kind)
        u = dev(u0)
        its = []
        for m in range(M):
            u, st = prob.cn_step(u, dev(Fs[m]))
            assert st["converged"] == 1
            its.append(int(st["iters"]))
        _STEPS[key] = its
    return _STEPS[key]


def _gpu_total(fsd, row):
    if row not in _TOTALS:
        tab, dim, orders, M, n1, kind, it = row
        total = sum(_run_steps(fsd, (tab, dim, orders, M, n1, kind)))
        _TOTALS[row] = (total, int(round(it * M)))
    return _TOTALS[row]


def _tolerance(row, printed):
    tab, kind = row[0], row[5]
    if tab in (1, 3) and kind != "none":
        return max(2, int(0.04 * printed))
    return max(2, int(0.001 * printed))


@pytest.mark.parametrize("row", _rows(), ids=lambda r: f"T{r[0]}-{r[4]}-{r[5]}-{'_'.join(map(str, r[2]))}")
def test_paper_comparator_counts_gpu(fsd, row):
    """Every printed comparator count of Tables 1-4 (the dagger entries
    excepted) up to the largest grids, 511^2 and 63^3."""
    total, printed = _gpu_total(fsd, row)
    assert abs(total - printed) <= _tolerance(row, printed), (row, total, printed)


def _oracle_rows():
    path = os.path.join(GOLDEN, "oracle_comparator_counts.json")
    return sorted(json.load(open(path))["rows"].items())


def _gpu_steps(fsd, v):
    return _run_steps(fsd, (v["table"], v["dim"], tuple(v["orders"]), v["M"], v["n_plus_1"],
                            v["kind"]))


@pytest.mark.parametrize("name,v", _oracle_rows(), ids=[k for k, _ in _oracle_rows()])
def test_comparator_steps_vs_oracle(fsd, name, v):
    """The circulant-preconditioned CG comparators of the symmetric tables
    at the sizes the oracle's own tests do not reach (128^2 to 511^2, 32^3
    and 64^3), step by step against the oracle's counts
    (golden/oracle_comparator_counts.json, written by the oracle).  Both
    are float64 CG with the same preconditioner (its application agrees to
    1e-12 above); where the preconditioned system is ill-conditioned the
    step at which the residual crosses tol moves with the rounding order:
    every step within 4 iterations, the total within 2.5%."""
    its = _gpu_steps(fsd, v)
    ref = v["iters"]
    assert len(its) == len(ref)
    worst = max(abs(a - b) for a, b in zip(its, ref))
    assert worst <= 4, (name, worst)
    assert abs(sum(its) - sum(ref)) <= max(2, 0.025 * sum(ref)), (name, sum(its), sum(ref))


def test_comparator_steps_vs_oracle_mostly_exact(fsd):
    """Most of those rows agree with the oracle in every step (every 3D
    row does)."""
    rows = _oracle_rows()
    exact = [k for k, v in rows if _gpu_steps(fsd, v) == v["iters"]]
    assert len(exact) >= int(0.6 * len(rows)), (len(exact), len(rows))
    assert all(k in exact for k, v in rows if v["dim"] == 3)


def test_paper_comparator_counts_gpu_mostly_exact(fsd):
    rows = _rows()
    exact = sum(1 for r in rows if _gpu_total(fsd, r)[0] == _gpu_total(fsd, r)[1])
    assert exact >= int(0.85 * len(rows)), (exact, len(rows))
