"""The device-pointer entry points of the binding reject tensors the kernels would misread (wrong
dtype, not contiguous, too short, not on the GPU) with ValueError before the library is called.
CPU only: the library entry is replaced by one that fails if reached."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1510_04068_amd.nbx as nbx  # noqa: E402


@pytest.fixture
def no_library(monkeypatch):
    def refuse(*a, **k):
        raise AssertionError("the library was called")

    monkeypatch.setattr(nbx, "load", refuse)


def _f64(*shape):
    return torch.zeros(shape, dtype=torch.float64)


def _force_args(ni, **over):
    args = dict(d_i_addr=torch.zeros(ni, dtype=torch.int32), d_h2=None, d_acc=_f64(ni, 3), d_jerk=_f64(ni, 3),
                d_snap=None, d_pot=_f64(ni), d_nn_id=torch.zeros(ni, dtype=torch.int64), d_nn_r2=_f64(ni))
    args.update(over)
    return args


def _call_force(ni, **over):
    a = _force_args(ni, **over)
    return nbx.nbx_force_dev(None, 0, ni, a["d_i_addr"], 1e-4, a["d_h2"], a["d_acc"], a["d_jerk"], a["d_snap"],
                             a["d_pot"], a["d_nn_id"], a["d_nn_r2"])


def test_float32_output_rejected(no_library):
    with pytest.raises(ValueError, match="d_acc: dtype torch.float32"):
        _call_force(8, d_acc=torch.zeros((8, 3), dtype=torch.float32))


def test_int64_addresses_rejected(no_library):
    with pytest.raises(ValueError, match="d_i_addr: dtype torch.int64"):
        _call_force(8, d_i_addr=torch.zeros(8, dtype=torch.int64))


def test_non_contiguous_rejected(no_library):
    with pytest.raises(ValueError, match="d_jerk: tensor is not contiguous"):
        _call_force(8, d_jerk=_f64(3, 8).t())


def test_short_tensor_rejected(no_library):
    with pytest.raises(ValueError, match="d_pot: 7 elements, the call needs 8"):
        _call_force(8, d_pot=_f64(7))


def test_cpu_tensor_rejected(no_library):
    with pytest.raises(ValueError, match="d_i_addr: tensor is on cpu, not on a GPU"):
        _call_force(8)


def test_set_j_and_vjp_and_batch_checked(no_library):
    n = 5
    i32, i64 = torch.zeros(n, dtype=torch.int32), torch.zeros(n, dtype=torch.int64)
    with pytest.raises(ValueError, match="d_x: dtype torch.float32"):
        nbx.nbx_set_j_dev(None, 0, n, i32, i64, _f64(n), _f64(n), torch.zeros((n, 3)), _f64(n, 3), _f64(n, 3),
                          _f64(n, 3))
    with pytest.raises(ValueError, match="d_g_jerk: 12 elements, the call needs 15"):
        nbx.nbx_force_vjp_dev(None, 0, n, _f64(n), _f64(n, 3), _f64(n, 3), 0.0, _f64(n, 3), _f64(4, 3), _f64(n),
                              _f64(n, 3), _f64(n, 3), _f64(n))
    with pytest.raises(ValueError, match="d_m: tensor is on cpu"):
        nbx.nbx_batch_force_dev(None, 0, _f64(n), _f64(n, 3), _f64(n, 3), 0.0, _f64(n, 3), _f64(n, 3), _f64(n))


def test_neighbour_arrays_checked_against_capacity(no_library):
    # a context the binding opened with nbr_max = 4: the id array must hold ni * 4 entries
    key = 0x1234
    nbx._CTX_INFO[key] = {"device": 0, "order": 4, "nbr_max": 4, "batch_n": 0}
    try:
        ctx = nbx.ctypes.c_void_p(key)
        a = _force_args(6)
        with pytest.raises(ValueError, match="d_nbr_ids: 20 elements, the call needs 24"):
            nbx.nbx_force_dev(ctx, 0, 6, a["d_i_addr"], 1e-4, _f64(6), a["d_acc"], a["d_jerk"], None, a["d_pot"],
                              a["d_nn_id"], a["d_nn_r2"], torch.zeros(6, dtype=torch.int32),
                              torch.zeros(20, dtype=torch.int64))
    finally:
        del nbx._CTX_INFO[key]


def test_raw_pointers_pass_through():
    # integers are taken as device addresses as given (the caller's responsibility)
    assert nbx._dptr(12345, "f64", 10**9) == 12345
    assert nbx._dptr(None, "f64", 10) is None
    assert np.dtype(np.float64).itemsize == 8
