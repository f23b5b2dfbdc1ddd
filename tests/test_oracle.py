"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics (closed forms, brute force on tiny grids, the paper's printed
iteration counts, invariants).  CPU only."""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import circulant as circ, coeffs, cn, examples as ex, krylov, operators as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- coefficients

@pytest.mark.parametrize("delta", [0.1, 0.3, 0.5, 0.7, 0.9])
def test_coef_lemma_2_1_and_2_2(delta):
    """Lemma 2.1 (signs, zero sum via telescoping, positive partial sums) and
    Lemma 2.2 (q_0+q_2 < q_3 < q_4 < ...)."""
    n = 400
    q = coeffs.q_coeffs(delta, n)
    s = coeffs.s_coeffs(delta, n)
    assert q[1] > 0 and q[0] + q[2] < 0
    assert np.all(q[3:] < 0)
    # sum_{k=0}^{K} q_k = -s_K exactly (telescoping), and s_K -> 0
    qm = coeffs.q_coeffs_mp(delta, n)
    sm = coeffs.s_coeffs_mp(delta, n)
    with mp.workdps(50):
        for K in (1, 2, 5, 50, n):
            assert abs(mp.fsum(qm[:K + 1]) + sm[K]) < mp.mpf(10) ** -40
    assert abs(s[n]) < 1e-3 and abs(s[n]) < abs(s[n // 2])
    # (iii) q_1 + sum_{k != 1, k <= s} q_k > 0 for s >= 2
    assert np.all(np.cumsum(q)[2:] > 0)
    # Lemma 2.2
    assert q[0] + q[2] < q[3]
    assert np.all(np.diff(q[3:]) > 0)


def test_coef_mp_vs_naive_small_k():
    """The float64 rounding of the 50-digit values agrees with the naive
    float64 formula where cancellation is harmless (small k)."""
    d = 0.37
    s = coeffs.s_coeffs(d, 10)
    naive = [0.5 ** d, 1.5 ** d - 2 * 0.5 ** d] + [
        (k + 0.5) ** d - 2 * (k - 0.5) ** d + (k - 1.5) ** d for k in range(2, 11)]
    np.testing.assert_allclose(s, naive, rtol=1e-13, atol=0)


def test_delta_zero_gives_laplacian():
    """At delta = 0 (outside the method's range) T_n = tridiag(-1, 2, -1)."""
    q = coeffs.q_coeffs(0.0, 6)
    T = op.T_mat(q, 6)
    ref = 2 * np.eye(6) - np.eye(6, k=1) - np.eye(6, k=-1)
    np.testing.assert_array_equal(T, ref)


@pytest.mark.parametrize("n", [1, 2, 5, 9])
@pytest.mark.parametrize("delta,kp,km", [(0.2, 1.0, 1.0), (0.65, 19.0, 21.0), (0.9, 0.3, 1.7)])
def test_B_from_hat_functions(n, delta, kp, km):
    """B_n from q_k equals the entry-wise finite-volume assembly from the
    Riemann-Liouville derivatives of the hat functions (Section 2)."""
    q = coeffs.q_coeffs(delta, n)
    np.testing.assert_allclose(op.B_mat(q, n, kp, km),
                               op.B_from_hat_functions(delta, n, kp, km),
                               rtol=0, atol=1e-14 * max(kp, km))


@pytest.mark.parametrize("n", [1, 2, 3, 8, 17])
def test_a_eigs(n):
    """Lemma 3.1: A_n is SPD with eigenvalues in (1/2, 1); closed form in the
    DST-I basis."""
    A = op.A_mat(n)
    S = op.dst1_mat(n)
    D = S @ A @ S
    np.testing.assert_allclose(D, np.diag(coeffs.a_eigs(n)), atol=1e-14)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > 0.5 and ev.max() < 1.0


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 16])
def test_dst_orthogonal_symmetric(n):
    S = op.dst1_mat(n)
    np.testing.assert_allclose(S, S.T, atol=1e-15)
    np.testing.assert_allclose(S @ S, np.eye(n), atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 9, 20])
@pytest.mark.parametrize("delta", [0.1, 0.5, 0.9])
def test_tau_eigs_diagonalise(n, delta):
    """Lemma 3.2 eigenvalue formula (index read as j): S tau(H(T)) S is
    diagonal with those entries; tau(H(T)) and H(T) are SPD; Lemma 3.5
    bound 1/2 < lambda(tau^{-1} H(T)) < 3/2."""
    q = coeffs.q_coeffs(delta, n)
    t = coeffs.sym_first_column(q, n)
    tau = op.tau_of_symmetric_toeplitz(t)
    S = op.dst1_mat(n)
    D = S @ tau @ S
    lam = coeffs.tau_eigs(q, n)
    np.testing.assert_allclose(D, np.diag(lam), atol=1e-14)
    assert lam.min() > 0
    T = op.T_mat(q, n)
    H = 0.5 * (T + T.T)
    assert np.linalg.eigvalsh(H).min() > 0
    if n >= 3:
        ev = np.linalg.eigvals(np.linalg.solve(tau, H)).real
        assert ev.min() > 0.5 and ev.max() < 1.5


# ---------------------------------------------------------------- operators

def _prob(dim, n, delta, kp, km, M=4):
    return op.Problem(dim, n, delta, kp, km, T=1.0, M=M)


PROBS = [
    _prob(2, [5, 7], [0.3, 0.8], [1.0, 1.0], [1.0, 1.0]),
    _prob(2, [6, 4], [0.4, 0.6], [19.0, 21.0], [21.0, 23.0]),
    _prob(3, [3, 4, 5], [0.3, 0.5, 0.7], [1.0] * 3, [1.0] * 3),
    _prob(3, [4, 3, 2], [0.4, 0.6, 0.8], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3]),
]


@pytest.mark.parametrize("prob", PROBS)
def test_dense_kron_equals_hat_assembly(prob):
    A1, R1 = op.dense_system(prob, "q")
    A2, R2 = op.dense_system(prob, "hat")
    scale = np.abs(A1).max()
    np.testing.assert_allclose(A1, A2, atol=1e-14 * scale)
    np.testing.assert_allclose(R1, R2, atol=1e-14 * scale)
    if prob.symmetric:
        np.testing.assert_allclose(A1, A1.T, atol=1e-15 * scale)
        assert np.linalg.eigvalsh(A1).min() > 0


@pytest.mark.parametrize("prob", PROBS)
def test_structured_vs_dense(prob):
    A, R = op.dense_system(prob)
    rng = np.random.default_rng(3)
    X = rng.standard_normal(prob.shape)
    F = rng.standard_normal(prob.shape)
    y = op.apply_A(prob, X)
    np.testing.assert_allclose(y.reshape(-1), A @ X.reshape(-1), rtol=0,
                               atol=1e-13 * np.abs(A).max() * np.abs(X).max())
    b = op.apply_rhs(prob, X, F)
    np.testing.assert_allclose(b.reshape(-1), R @ X.reshape(-1) + prob.dt * F.reshape(-1),
                               rtol=0, atol=1e-13 * np.abs(R).max() * 3)
    # independent route: multilevel circulant embedding + real FFT
    yc = op.apply_A_circulant(prob, X)
    np.testing.assert_allclose(yc, y, rtol=0, atol=1e-12 * np.abs(y).max())
    bc = op.apply_A_circulant(prob, X, sign=-1.0) + prob.dt * F
    np.testing.assert_allclose(bc, b, rtol=0, atol=1e-12 * np.abs(b).max())


@pytest.mark.parametrize("prob", PROBS)
def test_preconditioner(prob):
    """P = S_N Lambda S_N equals the explicit tau-matrix preconditioner;
    Lemma 3.3 lambda_min(P) > 1/8."""
    P = op.dense_preconditioner(prob)
    np.testing.assert_allclose(P, P.T, atol=1e-14 * np.abs(P).max())
    rng = np.random.default_rng(5)
    R = rng.standard_normal(prob.shape)
    z = op.apply_Pinv(prob, R)
    np.testing.assert_allclose(z.reshape(-1), np.linalg.solve(P, R.reshape(-1)),
                               rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(op.apply_P(prob, z), R, atol=1e-11 * np.abs(R).max())
    assert np.linalg.eigvalsh(P).min() > 1.0 / 8.0
    Lam = op.precond_eigs(prob)
    np.testing.assert_allclose(np.sort(Lam.reshape(-1)), np.linalg.eigvalsh(P),
                               rtol=1e-12)


def test_theorem_3_1_spectrum():
    """Theorem 3.1: symmetric case, lambda(P^{-1} A) in (1/2, 3/2)."""
    for delta in ([0.3, 0.5, 0.7], [0.1, 0.2, 0.3], [0.7, 0.8, 0.9]):
        prob = _prob(3, [7, 7, 7], delta, [1.0] * 3, [1.0] * 3)
        A, _ = op.dense_system(prob)
        P = op.dense_preconditioner(prob)
        ev = np.linalg.eigvals(np.linalg.solve(P, A))
        assert np.abs(ev.imag).max() < 1e-10
        assert ev.real.min() > 0.5 and ev.real.max() < 1.5


def test_lemmas_3_7_3_10_nonsymmetric():
    """Lemma 3.7: lambda(P^{-1/2} H(A) P^{-1/2}) in (1/2, 3/2); Lemma 3.10:
    rho(P^{-1/2} S(A) P^{-1/2}) <= (3/2) max_i tan(delta_i pi/2)
    |k+ - k-|/(k+ + k-); Theorem 3.2 rate omega < 1."""
    prob = _prob(3, [7, 7, 7], [0.4, 0.6, 0.8], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3])
    A, _ = op.dense_system(prob)
    P = op.dense_preconditioner(prob)
    w, V = np.linalg.eigh(P)
    Pmh = V @ np.diag(w ** -0.5) @ V.T
    H = 0.5 * (A + A.T)
    S = 0.5 * (A - A.T)
    evH = np.linalg.eigvalsh(Pmh @ H @ Pmh)
    assert evH.min() > 0.5 and evH.max() < 1.5
    rho = np.abs(np.linalg.eigvals(Pmh @ S @ Pmh)).max()
    vs = 1.5 * max(math.tan(prob.delta[i] * math.pi / 2) * abs(prob.kplus[i] - prob.kminus[i])
                   / (prob.kplus[i] + prob.kminus[i]) for i in range(3))
    assert rho <= vs
    omega = math.sqrt((2 + 4 * vs ** 2) / (3 + 4 * vs ** 2))
    assert omega < 1


# ---------------------------------------------------------------- solvers

@pytest.mark.parametrize("prob", PROBS)
def test_krylov_vs_lu(prob):
    A, _ = op.dense_system(prob)
    rng = np.random.default_rng(11)
    b = rng.standard_normal(prob.shape)
    x_ref = np.linalg.solve(A, b.reshape(-1)).reshape(prob.shape)
    x, info = cn.solve_step(prob, b, None, 1e-13)
    assert info.converged
    np.testing.assert_allclose(x, x_ref, rtol=0, atol=1e-11 * np.abs(x_ref).max())
    # with a nonzero initial guess
    x2, info2 = cn.solve_step(prob, b, rng.standard_normal(prob.shape), 1e-13)
    np.testing.assert_allclose(x2, x_ref, rtol=0, atol=1e-11 * np.abs(x_ref).max())
    # both solvers on the same (possibly non-symmetric) system: GMRES always
    # applies; PCG only in the symmetric case
    x3, _ = cn.solve_step(prob, b, None, 1e-13, solver="gmres", restart=3)
    np.testing.assert_allclose(x3, x_ref, rtol=0, atol=1e-10 * np.abs(x_ref).max())


def test_delta_zero_one_iteration():
    """At delta = 0, tau(H(T)) = T, so P = A and both solvers converge in one
    iteration (classical heat-equation limit; a test case outside (0,1))."""
    for kp, km in (([1.0, 1.0, 1.0], [1.0, 1.0, 1.0]), ([1.0, 2.0, 0.5], [3.0, 1.0, 0.7])):
        prob = _prob(3, [6, 5, 7], [0.0, 0.0, 0.0], kp, km)
        b = np.random.default_rng(1).standard_normal(prob.shape)
        x, info = cn.solve_step(prob, b, None, 1e-12)
        assert info.iters == 1
        A, _ = op.dense_system(prob)
        np.testing.assert_allclose(x.reshape(-1), np.linalg.solve(A, b.reshape(-1)), atol=1e-12)


def test_cn_run_vs_lu():
    for prob in PROBS:
        rng = np.random.default_rng(2)
        u0 = rng.standard_normal(prob.shape)
        F = rng.standard_normal(prob.shape)
        u, its = cn.run(prob, u0, lambda m: F * m, tol=1e-13)
        u_ref = cn.run_direct(prob, u0, lambda m: F * m)
        np.testing.assert_allclose(u, u_ref, rtol=0, atol=1e-11 * np.abs(u_ref).max())
        assert len(its) == prob.M


# ---------------------------------------------------------------- examples

def test_example_sources_match_printed():
    x = np.linspace(0.01, 0.99, 17)
    y = np.linspace(0.03, 0.97, 13)[:, None]
    for d, kp, km in (([0.1, 0.9], [5, 5], [5, 5]), ([0.4, 0.5], [19, 21], [21, 23])):
        a = ex.ex41_source(x, y, 0.3, d, kp, km)
        b = ex.ex41_source_printed(x, y, 0.3, d, kp, km)
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("delta,kp,km,x", [(0.3, 1.0, 0.0, 0.37), (0.7, 0.0, 1.0, 0.61),
                                          (0.5, 19.0, 21.0, 0.2)])
def test_flux_derivative_vs_quadrature(delta, kp, km, x):
    """d/dx D^delta p from the Riemann-Liouville integrals (Section 1),
    evaluated by mpmath quadrature.  Since p(0) = p'(0) = p(1) = p'(1) = 0 the
    two x-derivatives move under the integral sign:
    d/dx D^delta p = (1/Gamma(delta)) int_0^x w^(delta-1) [k+ p''(x-w)] dw
                   + (1/Gamma(delta)) int_0^(1-x) w^(delta-1) [k- p''(x+w)] dw."""
    with mp.workdps(30):
        d = mp.mpf(delta)
        xx = mp.mpf(x)
        p2 = lambda s: 2 - 12 * s + 12 * s ** 2      # (s^2 (1-s)^2)''
        left = mp.quad(lambda w: w ** (d - 1) * p2(xx - w), [0, xx])
        right = mp.quad(lambda w: w ** (d - 1) * p2(xx + w), [0, 1 - xx])
        ref = float((kp * left + km * right) / mp.gamma(d))
    got = float(ex.flux_derivative(np.array(x), delta, kp, km))
    assert abs(got - ref) <= 1e-9 * max(1.0, abs(ref))


def test_second_order_convergence_2d():
    """Remark 2.1: symmetric case, second order in space and time; the max
    relative error at T=1 drops about 4x per halving of h and dt."""
    errs = []
    for n1 in (16, 32, 64):
        prob = op.Problem(2, [n1 - 1] * 2, [0.4, 0.5], [5, 5], [5, 5], T=1.0, M=n1 // 4)
        h = prob.h
        F = lambda m: ex.cell_average(lambda X, Y: ex.ex41_source(
            X, Y, (m - 0.5) * prob.dt, prob.delta, prob.kplus, prob.kminus), prob.n, h)
        u0 = ex.nodal(lambda X, Y: ex.ex41_exact(X, Y, 0.0), prob.n, h)
        u, _ = cn.run(prob, u0, F, tol=1e-12)
        ue = ex.nodal(lambda X, Y: ex.ex41_exact(X, Y, 1.0), prob.n, h)
        errs.append(np.abs(u - ue).max() / np.abs(ue).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.5 and 3.0 < r2 < 5.5, errs


# ---------------------------------------------------------------- paper tables

def _golden_rows(max_2d=128, max_3d=32):
    rows = json.load(open(os.path.join(GOLDEN, "paper_iterations.json")))["rows"]
    out = []
    for tab, dim, orders, M, n1, it in rows:
        if (dim == 2 and n1 <= max_2d) or (dim == 3 and n1 <= max_3d):
            out.append((tab, dim, tuple(orders), M, n1, it))
    return out


@pytest.mark.parametrize("row", _golden_rows())
def test_paper_iteration_counts(row):
    """The oracle with the replication settings (x0 = 0, tol 1e-9, restart
    20) reproduces the printed average iteration counts of Tables 1-4."""
    tab, dim, orders, M, n1, it = row
    sym = tab in (1, 3)
    kp = [5.0] * dim if sym else [19.0, 21.0, 23.0][:dim]
    km = [5.0] * dim if sym else [21.0, 23.0, 25.0][:dim]
    prob = op.Problem(dim, [n1 - 1] * dim, list(orders), kp, km, T=1.0, M=M)
    h = prob.h
    if dim == 2:
        F = lambda m: ex.cell_average(lambda X, Y: ex.ex41_source(
            X, Y, (m - 0.5) * prob.dt, prob.delta, kp, km), prob.n, h)
        u0 = ex.nodal(lambda X, Y: ex.ex41_exact(X, Y, 0.0), prob.n, h)
    else:
        F = lambda m: ex.cell_average(lambda X, Y, Z: ex.ex42_source(
            X, Y, Z, (m - 0.5) * prob.dt, prob.delta, kp, km), prob.n, h)
        u0 = ex.nodal(lambda X, Y, Z: ex.ex42_exact(X, Y, Z, 0.0), prob.n, h)
    _, its = cn.run(prob, u0, F, tol=1e-9, x0_mode="zero",
                    maxit=(n1 - 1) ** 3, restart=20)
    assert round(float(np.mean(its)), 2) == it


@pytest.mark.parametrize("prob", PROBS)
def test_apply_A_at_sampled_entries(prob):
    """Single entries of A X and of the right-hand-side operator from the
    Kronecker rows agree with the full structured application."""
    X = np.random.default_rng(8).standard_normal(prob.shape)
    Y = op.apply_A(prob, X)
    R = op.apply_rhs(prob, X, None)
    for idx in np.ndindex(*prob.shape):
        assert abs(op.apply_A_at(prob, X, idx) - Y[idx]) <= 1e-13 * np.abs(Y).max()
        assert abs(op.apply_A_at(prob, X, idx, -1.0) - R[idx]) <= 1e-13 * np.abs(R).max()


# ------------------------------------------------ two-sided system (NEXT row)

NONSYM = [
    _prob(3, [7, 7, 7], [0.4, 0.6, 0.8], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3]),
    _prob(3, [5, 6, 7], [0.1, 0.5, 0.9], [19.0, 21.0, 23.0], [21.0, 23.0, 25.0]),
    _prob(2, [15, 9], [0.8, 0.9], [1.0, 2.0], [2.0, 0.5]),
]


def _dense_half(prob):
    """P^{-1/2} and P^{1/2} from the eigendecomposition of the dense tau
    preconditioner (an independent route to the sine-transform forms)."""
    P = op.dense_preconditioner(prob)
    w, V = np.linalg.eigh(P)
    return V @ np.diag(w ** -0.5) @ V.T, V @ np.diag(w ** 0.5) @ V.T


@pytest.mark.parametrize("prob", NONSYM[:2] + PROBS[:3])
def test_half_preconditioner_dense(prob):
    """S_N Lambda^{-1/2} S_N and S_N Lambda^{1/2} S_N equal the symmetric
    square roots of P^{-1} and P; applied twice they give P^{-1}."""
    Pmh, Ph = _dense_half(prob)
    R = np.random.default_rng(21).standard_normal(prob.shape)
    z = op.apply_Pinv_half(prob, R)
    np.testing.assert_allclose(z.reshape(-1), Pmh @ R.reshape(-1), rtol=1e-11,
                               atol=1e-12 * np.abs(z).max())
    np.testing.assert_allclose(op.apply_P_half(prob, R).reshape(-1), Ph @ R.reshape(-1),
                               rtol=1e-11, atol=1e-12 * np.abs(R).max())
    np.testing.assert_allclose(op.apply_Pinv_half(prob, z), op.apply_Pinv(prob, R),
                               atol=1e-13 * np.abs(z).max())


@pytest.mark.parametrize("prob", NONSYM)
def test_two_sided_gmres_vs_lu(prob):
    A, _ = op.dense_system(prob)
    b = np.random.default_rng(22).standard_normal(prob.shape)
    x_ref = np.linalg.solve(A, b.reshape(-1)).reshape(prob.shape)
    for x0 in (None, np.random.default_rng(23).standard_normal(prob.shape)):
        x, info = cn.solve_step(prob, b, x0, 1e-13, solver="gmres2")
        assert info.converged
        assert np.linalg.norm(x - x_ref) <= 1e-11 * np.linalg.norm(x_ref)


def _varsigma(prob):
    d = prob.dim
    return 1.5 * max(math.tan(prob.delta[i] * math.pi / 2) * abs(prob.kplus[i] - prob.kminus[i])
                     / (prob.kplus[i] + prob.kminus[i]) for i in range(d))


@pytest.mark.parametrize("prob", NONSYM)
def test_theorem_3_2_rate(prob):
    """Theorem 3.2: GMRES on P^{-1/2} A P^{-1/2} v = P^{-1/2} b has
    ||r_k|| <= omega^k ||r_0||, omega = sqrt((2 + 4 s^2) / (3 + 4 s^2)) with
    s the Lemma 3.10 bound; checked at every iteration, restarted (restart 5)
    and not."""
    vs = _varsigma(prob)
    omega = math.sqrt((2 + 4 * vs ** 2) / (3 + 4 * vs ** 2))
    A = lambda v: op.apply_A(prob, v)
    Mh = lambda v: op.apply_Pinv_half(prob, v)
    b = np.random.default_rng(24).standard_normal(prob.shape)
    for restart in (100, 5):
        _, info = krylov.gmres_two_sided(A, Mh, b, None, 1e-12, restart, 100)
        h = np.array(info.history)
        k = np.arange(len(h))
        assert np.all(h <= omega ** k * h[0] * (1 + 1e-10)), (restart, h, omega)


@pytest.mark.parametrize("prob", NONSYM)
def test_theorem_3_3_one_vs_two_sided(prob):
    """Theorem 3.3: from corresponding initial guesses (here zero) the
    one-sided GMRES residual ||P^{-1} b - P^{-1} A u_j|| is at most 2 sqrt(2)
    times the two-sided one ||P^{-1/2} b - P^{-1/2} A P^{-1/2} v_j||, at
    every iteration j >= 1 (both runs inside their first restart cycle)."""
    Lam = op.precond_eigs(prob)
    A = lambda v: op.apply_A(prob, v)
    Minv = lambda v: op.apply_Pinv(prob, v, Lam)
    Mh = lambda v: op.apply_Pinv_half(prob, v, Lam)
    b = np.random.default_rng(25).standard_normal(prob.shape)
    _, one = krylov.gmres_left(A, Minv, b, None, 1e-12, 200, 200)
    _, two = krylov.gmres_two_sided(A, Mh, b, None, 1e-12, 200, 200)
    r1 = np.array(one.history) * np.linalg.norm(Minv(b))
    r2 = np.array(two.history) * np.linalg.norm(Mh(b))
    k = min(len(r1), len(r2))
    assert k > 3
    assert np.all(r1[1:k] <= 2 * math.sqrt(2) * r2[1:k] * (1 + 1e-10)), (r1[:k], r2[:k])


# ---------------------------------------------------------------- comparators



def _random_toeplitz(n, rng):
    t = rng.standard_normal(2 * n - 1)          # t[o + n - 1] = t_o, o = -(n-1)..n-1
    return np.array([[t[j - k + n - 1] for k in range(n)] for j in range(n)])


@pytest.mark.parametrize("n", [1, 2, 7, 8, 15])
def test_strang_keeps_central_diagonals(n):
    """Strang's circulant equals T on every diagonal with |j - k| < n/2
    (and on |j - k| = n//2 below the main diagonal)."""
    T = _random_toeplitz(n, np.random.default_rng(n))
    C = sla.circulant(circ.first_column(T, "strang"))
    for j in range(n):
        for k in range(n):
            o = j - k
            if abs(o) < n / 2 or o == n // 2:
                assert C[j, k] == T[j, k]


@pytest.mark.parametrize("n", [1, 2, 7, 8, 15])
def test_tchan_is_the_frobenius_nearest_circulant(n):
    """T. Chan's circulant minimises ||C - T||_F over circulants: solve that
    least-squares problem over the basis of n circulant permutations."""
    T = _random_toeplitz(n, np.random.default_rng(100 + n))
    E = [sla.circulant(np.eye(n)[j]) for j in range(n)]
    Amat = np.stack([e.ravel() for e in E], axis=1)
    c_ls, *_ = np.linalg.lstsq(Amat, T.ravel(), rcond=None)
    assert np.allclose(circ.first_column(T, "tchan"), c_ls, rtol=0, atol=1e-13)


CIRC_PROBS = [
    op.Problem(2, [7, 5], [0.3, 0.7], [1.0, 2.0], [1.0, 2.0], T=1.0, M=4),
    op.Problem(2, [6, 9], [0.2, 0.9], [19.0, 21.0], [21.0, 23.0], T=1.0, M=3),
    op.Problem(3, [5, 4, 3], [0.1, 0.5, 0.9], [5.0, 5.0, 5.0], [5.0, 5.0, 5.0], T=1.0, M=2),
    op.Problem(3, [3, 5, 4], [0.4, 0.6, 0.8], [1.0, 0.8, 1.2], [0.5, 1.0, 0.3], T=1.0, M=2),
]


@pytest.mark.parametrize("kind", ["tchan", "strang"])
@pytest.mark.parametrize("prob", CIRC_PROBS)
def test_circulant_pinv_against_dense(prob, kind):
    """ifftn(fftn(R) / Lambda) equals the dense solve with P assembled from
    dense circulants and Kronecker products; P is real, and symmetric when
    every axis is."""
    P = circ.dense_precond(prob, kind)
    R = np.random.default_rng(3).standard_normal(prob.shape)
    Z = circ.apply_Pinv(prob, R, circ.precond_eigs(prob, kind))
    ref = np.linalg.solve(P, R.ravel()).reshape(prob.shape)
    assert np.abs(Z - ref).max() <= 1e-12 * np.abs(ref).max()
    if prob.symmetric:
        assert np.allclose(P, P.T, rtol=0, atol=1e-14 * np.abs(P).max())


def test_tchan_preserves_positive_definiteness():
    """T. Chan's circulant of a symmetric positive definite Toeplitz matrix
    is positive definite, so PCG(T) is well defined in the symmetric case."""
    prob = op.Problem(3, [7, 15, 3], [0.1, 0.5, 0.9], [5.0] * 3, [5.0] * 3, T=1.0, M=8)
    Lam = circ.precond_eigs(prob, "tchan")
    assert np.abs(Lam.imag).max() <= 1e-12 * np.abs(Lam).max()
    assert Lam.real.min() > 0


def _comparator_rows(max_2d=64, max_3d=16):
    rows = json.load(open(os.path.join(GOLDEN, "paper_comparator_iterations.json")))["rows"]
    out = []
    for tab, dim, orders, M, n1, none, tchan, strang in rows:
        if (dim == 2 and n1 <= max_2d) or (dim == 3 and n1 <= max_3d):
            for kind, it in (("none", none), ("tchan", tchan), ("strang", strang)):
                out.append((tab, dim, tuple(orders), M, n1, kind, it))
    return out


def _paper_problem(tab, dim, orders, M, n1):
    sym = tab in (1, 3)
    kp = [5.0] * dim if sym else [19.0, 21.0, 23.0][:dim]
    km = [5.0] * dim if sym else [21.0, 23.0, 25.0][:dim]
    prob = op.Problem(dim, [n1 - 1] * dim, list(orders), kp, km, T=1.0, M=M)
    h = prob.h
    if dim == 2:
        F = lambda m: ex.cell_average(lambda X, Y: ex.ex41_source(
            X, Y, (m - 0.5) * prob.dt, prob.delta, kp, km), prob.n, h)
        u0 = ex.nodal(lambda X, Y: ex.ex41_exact(X, Y, 0.0), prob.n, h)
    else:
        F = lambda m: ex.cell_average(lambda X, Y, Z: ex.ex42_source(
            X, Y, Z, (m - 0.5) * prob.dt, prob.delta, kp, km), prob.n, h)
        u0 = ex.nodal(lambda X, Y, Z: ex.ex42_exact(X, Y, Z, 0.0), prob.n, h)
    return prob, F, u0


_COMPARATOR_TOTALS = {}


def _comparator_total(row):
    """(iterations summed over the M steps, the printed average times M)."""
    if row not in _COMPARATOR_TOTALS:
        tab, dim, orders, M, n1, kind, it = row
        prob, F, u0 = _paper_problem(tab, dim, orders, M, n1)
        _, its = cn.run(prob, u0, F, tol=1e-9, x0_mode="zero", maxit=(n1 - 1) ** 3,
                        restart=20, precond=kind)
        _COMPARATOR_TOTALS[row] = (int(np.sum(its)), int(round(it * M)))
    return _COMPARATOR_TOTALS[row]


@pytest.mark.parametrize("row", _comparator_rows())
def test_paper_comparator_iteration_counts(row):
    """The oracle's comparators with the replication settings reproduce the
    printed average iteration counts of CG/GMRES, PCG(T)/PGMRES(T) and
    PCG(S)/PGMRES(S) (Tables 1-4), to within two iterations summed over the
    M steps: without a preconditioner CG and GMRES run hundreds of
    iterations per step, and where a step ends right at the threshold a
    different rounding order moves its count by one."""
    total, printed = _comparator_total(row)
    assert abs(total - printed) <= 2, (row, total, printed)


def test_paper_comparator_counts_mostly_exact():
    """Most comparator entries match the printed average exactly (the
    tolerance above is for the few rounding-sensitive ones)."""
    rows = _comparator_rows()
    exact = sum(1 for r in rows if _comparator_total(r)[0] == _comparator_total(r)[1])
    assert exact >= int(0.85 * len(rows)), (exact, len(rows))


def test_oracle_comparator_golden_matches_paper():
    """The oracle's stored comparator counts at the larger grids
    (golden/oracle_comparator_counts.json, written by
    make_oracle_comparator_counts.py from oracle/ alone) reproduce the
    printed averages of Tables 1 and 3 to 1% of the total (measured: 0.74%
    at most, PCG(S) with orders (0.1, 0.2) at 511^2), and every stored row
    has one count per time step."""
    rows = json.load(open(os.path.join(GOLDEN, "oracle_comparator_counts.json")))["rows"]
    printed = {}
    for tab, dim, orders, M, n1, none, tchan, strang in json.load(
            open(os.path.join(GOLDEN, "paper_comparator_iterations.json")))["rows"]:
        printed[(tab, tuple(orders), n1, "tchan")] = (M, tchan)
        printed[(tab, tuple(orders), n1, "strang")] = (M, strang)
    assert len(rows) == 40
    for name, v in rows.items():
        M, avg = printed[(v["table"], tuple(v["orders"]), v["n_plus_1"], v["kind"])]
        assert v["M"] == M and len(v["iters"]) == M, name
        total = sum(v["iters"])
        assert abs(total - avg * M) <= max(2, 0.01 * avg * M), (name, total, avg * M)


def test_example_sources_separate_in_time():
    """Example 4.1's source is e^t f(x, y, 0); Example 4.2's is
    cos(t+1) P - sin(t+1) D with (P, D) from ex42_source_parts, at random
    points and times (the form the large-grid GPU runs use)."""
    rng = np.random.default_rng(5)
    x, y, z = (rng.uniform(0.01, 0.99, 200) for _ in range(3))
    d, kp, km = [0.1, 0.5, 0.9], [19.0, 21.0, 23.0], [21.0, 23.0, 25.0]
    P, D = ex.ex42_source_parts(x, y, z, d, kp, km)
    for t in (0.0, 0.3, 1.0):
        f2 = ex.ex41_source(x, y, t, d, kp, km)
        assert np.allclose(f2, math.exp(t) * ex.ex41_source(x, y, 0.0, d, kp, km), rtol=1e-14, atol=0)
        f3 = ex.ex42_source(x, y, z, t, d, kp, km)
        g3 = math.cos(t + 1.0) * P - math.sin(t + 1.0) * D
        assert np.abs(f3 - g3).max() <= 1e-14 * np.abs(f3).max()


def test_separable_cell_averages():
    """The one-dimensional Gauss average is exact for polynomials of degree
    up to 7 (closed-form cell averages of x^2 and x^7), and the sources
    assembled from one-dimensional averages equal the tensor-product cell
    averages of the full sources (Examples 4.1 and 4.2)."""
    n, h = 9, 0.1
    lo = h * np.arange(1, n + 1) - 0.5 * h
    hi = lo + h
    for k in (2, 7):
        exact = (hi ** (k + 1) - lo ** (k + 1)) / ((k + 1) * h)
        got = ex.cell_average_1d(lambda x: x ** k, n, h)
        assert np.abs(got - exact).max() <= 1e-15 * np.abs(exact).max()
    d, kp, km = [0.3, 0.7, 0.45], [19.0, 1.0, 5.0], [21.0, 2.5, 5.0]
    n2 = [31, 23]
    h2 = [1.0 / 32, 1.0 / 24]
    full = ex.cell_average(lambda X, Y: ex.ex41_source(X, Y, 0.0, d, kp, km), n2, h2)
    sep = ex.ex41_source_cells(n2, h2, d, kp, km)
    assert sep.shape == full.shape
    assert np.abs(sep - full).max() <= 1e-13 * np.abs(full).max()
    n3 = [7, 9, 5]
    h3 = [1.0 / 8, 1.0 / 10, 1.0 / 6]
    P, D = ex.ex42_source_parts_cells(n3, h3, d, kp, km)
    Pf = ex.cell_average(lambda X, Y, Z: ex.ex42_source_parts(X, Y, Z, d, kp, km)[0], n3, h3)
    Df = ex.cell_average(lambda X, Y, Z: ex.ex42_source_parts(X, Y, Z, d, kp, km)[1], n3, h3)
    assert np.abs(P - Pf).max() <= 1e-13 * np.abs(Pf).max()
    assert np.abs(D - Df).max() <= 1e-13 * np.abs(Df).max()


@pytest.mark.parametrize("n,delta", [(1023, 0.35), (4095, 0.35), (4095, 0.8)])
def test_tau_eigs_extended_precision(n, delta):
    """The Lemma 3.2 sum cancels for the smallest eigenvalues (the q_j sum
    to zero, Lemma 2.1).  The oracle's value from the split q_j agrees with
    a 40-digit mpmath evaluation of the same sum over the 50-digit q_j at
    the smallest, middle and largest k.  Bound: extended precision (unit
    roundoff 1.1e-19) over terms whose magnitudes sum to S = sum |q_j|
    (they decay like j^(delta-2), so a few dozen dominate the partial sums):
    20 * 1.1e-19 * S, plus the final rounding to float64 (measured: 1.5e-19
    absolute, 2.8e-14 relative to the smallest eigenvalue at n = 4095,
    delta = 0.35).  From the float64 q_j alone that eigenvalue is off by
    5e-17 absolute (1e-11 relative)."""
    import mpmath as mp
    hi, lo = coeffs.q_coeffs_split(delta, n)
    lam = coeffs.tau_eigs(hi, n, lo)
    S = float(np.abs(hi).sum())
    qmp = coeffs.q_coeffs_mp(delta, n)
    with mp.workdps(40):
        for k in (1, 2, 3, n // 2, n):
            th = mp.mpf(k) * mp.pi / (n + 1)
            ref = qmp[1] + (qmp[0] + qmp[2]) * mp.cos(th)
            ref += mp.fsum(qmp[j + 1] * mp.cos(j * th) for j in range(2, n))
            r = float(ref)
            bound = 20 * 1.1e-19 * S + 1.2e-16 * abs(r)
            assert abs(lam[k - 1] - r) <= bound, (k, lam[k - 1], r, bound)
            if k == 1 and n == 4095:
                # the float64 rounding of the q_j alone moves it far more
                assert abs(coeffs.tau_eigs(hi, n)[0] - r) > 3 * bound
