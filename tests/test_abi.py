"""The C-ABI library: it loads, exports every symbol include/*.h declares,
validates parameters, and its host-side coefficients match the oracle.
CPU only: no call here touches a GPU (fsd_init_problem and
fsd_get_coefficients are host-only)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("fsd.h", "fsd_nn.h", "fsd_batch.h")]


def header_functions():
    names = set()
    for h in HEADERS:
        text = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(fsd_[A-Za-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_headers_listed():
    assert sorted(os.listdir(os.path.join(ROOT, "include"))) == sorted(os.path.basename(h) for h in HEADERS)


@pytest.fixture(scope="module")
def nat():
    from paper_2511_21198_amd import _native
    return _native


def test_header_symbols_exported(nat):
    names = header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(nat.lib, name), name
        assert name in nat.SIGNATURES, f"binding lacks {name}"
    assert set(nat.SIGNATURES) == set(names)


def test_struct_sizes(nat):
    # fsd_params / fsd_stats as laid out by the C compiler (x86-64 SysV)
    # dim, n[3], 5 double[3], M, (pad), T, solver, restart, tol, maxit, precision,
    # (pad), inner_tol, max_outer, x0_mode, allow_delta_zero, dst_mfma, reorth_eta2,
    # precond, (pad)
    assert C.sizeof(nat.Params) == (4 + 12 + 5 * 24 + 4 + 4 + 8 + 4 + 4 + 8 + 8 + 4 + 4 + 8 + 4 + 4
                                    + 4 + 4 + 8 + 4 + 4)
    assert C.sizeof(nat.Stats) == 40


def _params(nat, **kw):
    p = nat.Params()
    assert nat.lib.fsd_default_params(C.byref(p)) == nat.OK
    for k, v in kw.items():
        if isinstance(v, (list, tuple)):
            arr = getattr(p, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(p, k, v)
    return p


def _init(nat, p):
    h = C.c_void_p()
    s = nat.lib.fsd_init_problem(C.byref(p), C.byref(h))
    return s, h


@pytest.mark.parametrize("kw,status", [
    (dict(dim=4), 1), (dict(n=[0, 7, 7]), 1), (dict(delta=[1.0, 0.5, 0.5]), 1),
    (dict(delta=[0.0, 0.5, 0.5]), 1), (dict(kplus=[-1.0, 1.0, 1.0]), 1), (dict(T=0.0), 1),
    (dict(M=0), 1), (dict(tol=0.0), 1), (dict(restart=0), 1), (dict(restart=65), 1),
    (dict(solver=4), 1), (dict(solver=-1), 1), (dict(precond=4), 1), (dict(precond=-1), 1),
    (dict(precond=2, precision=1), 1), (dict(precond=3, solver=3), 1),
    (dict(n=[9, 7, 7]), 7), (dict(n=[8191, 7, 7]), 7), (dict(n=[100, 7, 7]), 7),
    (dict(n=[5000, 7, 7]), 7), (dict(n=[2047, 7, 7], precond=2), 7),
])
def test_init_validation(nat, kw, status):
    s, h = _init(nat, _params(nat, **kw))
    assert s == status
    assert not h.value
    assert len(nat.lib.fsd_last_error()) > 0


def test_two_sided_gmres_accepted(nat):
    s, h = _init(nat, _params(nat, n=[7, 7, 7], solver=nat.SOLVER_PGMRES2, precision=1))
    assert s == nat.OK
    assert nat.lib.fsd_workspace_bytes(h) > 0
    nat.lib.fsd_destroy(h)


@pytest.mark.parametrize("precond,solver,prec", [(1, 1, 1), (1, 3, 0), (2, 2, 0), (3, 1, 0)])
def test_comparator_preconditioners_accepted(nat, precond, solver, prec):
    """No preconditioner runs with every solver and precision; the circulant
    ones in float64 with the one-sided solvers.  The circulant workspace
    holds one complex work vector more."""
    kw = dict(n=[255, 255, 255], solver=solver, precision=prec)
    s, h = _init(nat, _params(nat, precond=precond, **kw))
    assert s == nat.OK
    s0, h0 = _init(nat, _params(nat, **kw))
    assert s0 == nat.OK
    extra = nat.lib.fsd_workspace_bytes(h) - nat.lib.fsd_workspace_bytes(h0)
    Np = 256 * 255 * 255
    if precond in (2, 3):
        assert 16 * Np <= extra < 16 * Np + (1 << 20)
    else:
        assert extra == 0
    nat.lib.fsd_destroy(h)
    nat.lib.fsd_destroy(h0)


def test_delta_zero_allowed_in_test_mode(nat):
    s, h = _init(nat, _params(nat, delta=[0.0, 0.0, 0.0], allow_delta_zero=1, n=[7, 7, 7]))
    assert s == nat.OK
    nat.lib.fsd_destroy(h)


def test_null_and_unbound(nat):
    assert nat.lib.fsd_workspace_bytes(None) == 0
    s, h = _init(nat, _params(nat, n=[7, 7, 7]))
    assert s == nat.OK
    x = C.c_void_p(16)
    assert nat.lib.fsd_apply_A(h, x, x) == nat.ENOTBOUND
    assert nat.lib.fsd_apply_A_noalloc(h, x, x) == nat.ENOTBOUND
    assert nat.lib.fsd_apply_A32(h, x, x) == nat.ENOTBOUND
    assert nat.lib.fsd_noalloc_scratch_bytes() == 64 << 20
    # argument checks of the stream copy come before any device work
    assert nat.lib.fsd_hbm_copy(None, x, 16, None) == nat.EINVAL
    assert nat.lib.fsd_hbm_copy(C.c_void_p(16), C.c_void_p(4096), 24, None) == nat.EINVAL
    assert nat.lib.fsd_hbm_copy(C.c_void_p(16), C.c_void_p(32), 64, None) == nat.EINVAL
    assert nat.lib.fsd_bind(h, None, 0, None) == nat.EINVAL
    assert nat.lib.fsd_bind(h, C.c_void_p(256), 16, None) == nat.ESMALLWS
    assert nat.lib.fsd_bind(h, C.c_void_p(257), 1 << 40, None) == nat.EINVAL
    nat.lib.fsd_destroy(h)


@pytest.mark.parametrize("dim,n,solver,prec", [
    (3, [255, 255, 255], 1, 0), (3, [255, 255, 255], 2, 1), (2, [1023, 1023, 1], 1, 1),
    (3, [1, 2, 3], 2, 0)])
def test_workspace_size(nat, dim, n, solver, prec):
    s, h = _init(nat, _params(nat, dim=dim, n=n, solver=solver, precision=prec))
    assert s == nat.OK
    ws = nat.lib.fsd_workspace_bytes(h)
    P1 = (n[0] + 31) // 32 * 32
    Np = P1 * n[1] * (n[2] if dim == 3 else 1)
    nvec = 10 + (22 if solver == 2 and prec == 0 else 0)
    assert ws >= Np * 8 * nvec
    assert ws < Np * 8 * (nvec + 2) + Np * 4 * (10 + (22 if solver == 2 else 0)) * prec + (64 << 20)
    nat.lib.fsd_destroy(h)


@pytest.mark.parametrize("n", [1, 2, 7, 63, 255, 1023, 4095])
@pytest.mark.parametrize("delta", [0.05, 0.3, 0.5, 0.8, 0.97])
def test_host_coefficients_match_oracle(nat, n, delta):
    """q_k (cancellation-safe evaluation in the library) and the tau
    eigenvalues agree with the oracle's 50-digit values."""
    from oracle import coeffs, operators as op
    s, h = _init(nat, _params(nat, dim=2, n=[n, 3, 1], delta=[delta, 0.5, 0.5],
                              kplus=[1.3, 1, 1], kminus=[0.7, 1, 1], M=7, T=0.9))
    assert s == nat.OK
    q = (C.c_double * (n + 1))()
    lam = (C.c_double * n)()
    eta = C.c_double()
    assert nat.lib.fsd_get_coefficients(h, 0, q, lam, C.byref(eta)) == nat.OK
    qo, qlo = coeffs.q_coeffs_split(delta, n)
    np.testing.assert_allclose(np.array(q), qo, rtol=1.2e-15, atol=0)
    lo = coeffs.tau_eigs(qo, n, qlo)
    np.testing.assert_allclose(np.array(lam), lo, rtol=1e-13, atol=1e-15 * np.abs(lo).max())
    pr = op.Problem(2, [n, 3], [delta, 0.5], [1.3, 1], [0.7, 1], T=0.9, M=7)
    assert abs(eta.value - pr.eta[0]) <= 1e-15 * pr.eta[0]
    assert nat.lib.fsd_get_coefficients(h, 2, None, None, None) == nat.EINVAL
    nat.lib.fsd_destroy(h)


def test_engine_selection_host(nat):
    """fsd_set_engine validates pass, engine and length on the host (no
    device work); fsd_engines reports the choice; fsd_autotune needs a bound
    workspace."""
    s, h = _init(nat, _params(nat, dim=3, n=[255, 95, 63], precision=1))
    assert s == nat.OK
    assert nat.lib.fsd_autotune(h) == nat.ENOTBOUND
    # float32 strided pass of length 512 on the x axis is not a column pass
    assert nat.lib.fsd_set_engine(h, 1, nat.PASSES["toep_x"], nat.ENGINES["col"]) == nat.EUNSUPPORTED
    assert nat.lib.fsd_set_engine(h, 0, 9, 0) == nat.EINVAL
    assert nat.lib.fsd_set_engine(h, 0, nat.PASSES["toep_x"], 7) == nat.EINVAL
    assert nat.lib.fsd_set_engine(h, 0, nat.PASSES["toep_x"], nat.ENGINES["stage"]) == nat.OK
    assert nat.lib.fsd_set_engine(h, 1, nat.PASSES["dst_x"], nat.ENGINES["stage_half"]) == nat.OK
    # y axis: n = 95 (length 192): stage engine only
    assert nat.lib.fsd_set_engine(h, 0, nat.PASSES["toep_y"], nat.ENGINES["wave"]) == nat.EUNSUPPORTED
    assert nat.lib.fsd_set_engine(h, 1, nat.PASSES["toep_y"], nat.ENGINES["wave1"]) == nat.EUNSUPPORTED
    # one line per lane group: float32 wave-engine lengths only
    assert nat.lib.fsd_set_engine(h, 0, nat.PASSES["dst_x"], nat.ENGINES["wave1"]) == nat.EUNSUPPORTED
    assert nat.lib.fsd_set_engine(h, 1, nat.PASSES["toep_z"], nat.ENGINES["wave1"]) == nat.OK
    n = nat.lib.fsd_engines(h, None, 0)
    buf = C.create_string_buffer(n + 1)
    assert nat.lib.fsd_engines(h, buf, n + 1) == n
    txt = buf.value.decode()
    assert "toep_x_f64(L=512)=stage" in txt and "dst_x_f32(L=512)=stage_half" in txt
    assert "toep_y_f64(L=192)=auto" in txt and "dsts_last_f32(L=128)=auto" in txt
    assert "toep_z_f32(L=128)=wave1" in txt
    nat.lib.fsd_destroy(h)
    s, h = _init(nat, _params(nat, dim=2, n=[255, 63]))
    assert nat.lib.fsd_set_engine(h, 0, nat.PASSES["toep_z"], 0) == nat.EINVAL   # 2D: no z pass
    nat.lib.fsd_destroy(h)
