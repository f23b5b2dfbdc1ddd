"""Host-side checks of the batch ABI (no GPU work): creation validates every
parameter set and reports the failing index; the workspace is the sum of
the per-problem workspaces, each 256-byte aligned."""
import ctypes as C

import pytest


@pytest.fixture(scope="module")
def nat():
    from paper_2511_21198_amd import _native
    return _native


def _params(nat, items):
    from paper_2511_21198_amd.solver import make_params
    arr = (nat.Params * len(items))()
    for i, kw in enumerate(items):
        arr[i] = make_params(**kw)
    return arr


KW = [dict(dim=2, n=(127, 63), delta=(0.3, 0.6), kplus=(1, 1), kminus=(1, 1), M=8),
      dict(dim=3, n=(31, 15, 63), delta=(0.3, 0.6, 0.8), kplus=(1, 2, 1), kminus=(2, 1, 1), M=8,
           solver="gmres", precision="mixed"),
      dict(dim=3, n=(95, 95, 95), delta=(0.5, 0.5, 0.5), kplus=(1, 1, 1), kminus=(1, 1, 1), M=8)]


def test_workspace_is_sum_of_parts(nat):
    p = _params(nat, KW)
    h = C.c_void_p()
    assert nat.lib.fsd_batch_create(p, len(KW), C.byref(h)) == nat.OK
    total = 0
    for i, kw in enumerate(KW):
        q = C.c_void_p()
        assert nat.lib.fsd_init_problem(C.byref(p[i]), C.byref(q)) == nat.OK
        assert nat.lib.fsd_batch_offset(h, i) == total
        total += (nat.lib.fsd_workspace_bytes(q) + 255) // 256 * 256
        nat.lib.fsd_destroy(q)
    assert nat.lib.fsd_batch_workspace_bytes(h) == total
    assert nat.lib.fsd_batch_problem(h, 1) is not None and nat.lib.fsd_batch_problem(h, 3) is None
    assert nat.lib.fsd_batch_cn_step(h, None, None, None, None, None) == nat.ENOTBOUND
    nat.lib.fsd_batch_destroy(h)


def test_invalid_member_reported(nat):
    bad = KW + [dict(dim=3, n=(100, 15, 15), delta=(0.3, 0.6, 0.8), kplus=(1, 1, 1),
                     kminus=(1, 1, 1))]
    h = C.c_void_p()
    assert nat.lib.fsd_batch_create(_params(nat, bad), len(bad), C.byref(h)) == nat.EUNSUPPORTED
    assert "problem 3" in nat.lib.fsd_last_error().decode()
    assert nat.lib.fsd_batch_create(None, 0, C.byref(h)) == nat.EINVAL
