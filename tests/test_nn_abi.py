"""Host-side checks of the warm-start network ABI (no GPU work): the layer
table and parameter count agree with the oracle's network definition,
sizes are validated, workspace sizes grow with the grid."""
import ctypes as C

import pytest

from oracle import nn as onn


@pytest.fixture(scope="module")
def nat():
    from paper_2511_21198_amd import _native
    return _native


def test_layers_match_oracle(nat):
    assert nat.lib.fsd_nn_param_count() == onn.param_count()
    for k, (_, ci, co, lv, _) in enumerate(onn.LAYERS):
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        assert nat.lib.fsd_nn_layer(k, C.byref(a), C.byref(b), C.byref(c)) == nat.OK
        assert (a.value, b.value, c.value) == (ci, co, lv)
    assert nat.lib.fsd_nn_layer(7, None, None, None) == nat.EINVAL


@pytest.mark.parametrize("dims,status", [((0, 4, 4, 1), 1), ((4, 4, 4, 0), 1), ((4, 4, 4, 1), 0)])
def test_create_validation(nat, dims, status):
    h = C.c_void_p()
    assert nat.lib.fsd_nn_create(*dims, 0, C.byref(h)) == status
    if status == 0:
        nat.lib.fsd_nn_destroy(h)


def test_workspace_and_unbound(nat):
    sizes = []
    for training in (0, 1):
        for n in (8, 16):
            h = C.c_void_p()
            assert nat.lib.fsd_nn_create(n, n, n, 1, training, C.byref(h)) == nat.OK
            sizes.append(nat.lib.fsd_nn_workspace_bytes(h))
            if n == 8:
                assert nat.lib.fsd_nn_forward(h, None, None, None) == nat.ENOTBOUND
            nat.lib.fsd_nn_destroy(h)
    assert sizes[0] < sizes[1] and sizes[2] < sizes[3] and sizes[0] < sizes[2]
