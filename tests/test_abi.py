"""C-ABI checks that need no GPU: the library loads, exports every symbol include/nbx.h declares,
and reports the absence of a device as an error code (no abort, no exception across the ABI)."""

import ctypes
import os
import re

import pytest

import paper_1510_04068_amd as nbx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbx.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nbx_[a-z0-9_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(nbx.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(nbx.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name


def test_version():
    assert nbx.nbx_version() == 10300


def test_argument_errors_without_device():
    lib = nbx.load()
    assert lib.nbx_open(None, None) == nbx.NBX_ERR_ARG
    ctx = ctypes.c_void_p()
    assert lib.nbx_open(ctypes.byref(ctx), None) == nbx.NBX_ERR_ARG
    bad = nbx.nbx_config(0, 5, nbx.NBX_FP64, 10, 10, 0)
    assert lib.nbx_open(ctypes.byref(ctx), ctypes.byref(bad)) == nbx.NBX_ERR_ARG
    assert b"order" in lib.nbx_last_error(None)
    bad = nbx.nbx_config(0, 4, 7, 10, 10, 0)
    assert lib.nbx_open(ctypes.byref(ctx), ctypes.byref(bad)) == nbx.NBX_ERR_ARG
    bad = nbx.nbx_config(0, 4, nbx.NBX_FP64, 0, 10, 0)
    assert lib.nbx_open(ctypes.byref(ctx), ctypes.byref(bad)) == nbx.NBX_ERR_ARG
    # entry points reject a NULL context instead of crashing
    assert lib.nbx_close(None) == nbx.NBX_OK
    assert lib.nbx_predict(None, 0.0) == nbx.NBX_ERR_ARG
    assert lib.nbx_set_nj(None, 1) == nbx.NBX_ERR_ARG
    assert lib.nbx_force(None, 0, None, 0.0, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_get_force(None, None, None, None, None, None, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_set_precision(None, 0) == nbx.NBX_ERR_ARG
    assert lib.nbx_launch_shape(None, 1, None, None, None, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_bs_init(None, 1, None, None, None, None, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_bs_step(None, 1.0, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_bs_run(None, 1.0, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_bs_get_state(None, None, None, None, None, None, None) == nbx.NBX_ERR_ARG
    assert lib.nbx_bs_energy(None, None, None) == nbx.NBX_ERR_ARG


def test_no_device_is_an_error_code():
    if nbx.nbx_device_count() > 0:
        pytest.skip("a GPU is visible")
    with pytest.raises(nbx.NbxError) as e:
        nbx.nbx_open(0, 4, nbx.NBX_FP64, 128, 128, 0)
    assert e.value.code == nbx.NBX_ERR_NO_DEVICE
