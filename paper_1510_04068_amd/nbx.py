"""ctypes binding of libnbx (include/nbx.h): same entry-point names, argument marshalling only.

Every computation happens in the HIP library.  If ``libnbx.so`` has not been built, loading
fails with a RuntimeError: there is no CPU fallback.

Host-array entry points take numpy arrays; the ``*_dev`` entry points take torch device tensors
(or raw device pointers) and a stream (``torch.cuda.Stream``, a raw hipStream_t integer, or None
for torch's current stream).
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnbx.so")

NBX_OK = 0
NBX_WARN_NBR_OVERFLOW = 1
NBX_WARN_DT_MIN = 2
NBX_ERR_ARG = -1
NBX_ERR_CAPACITY = -2
NBX_ERR_STATE = -3
NBX_ERR_DEVICE = -4
NBX_ERR_NO_DEVICE = -5
NBX_ERR_OOM = -6
NBX_FP64 = 0
NBX_MIXED = 1
NBX_DS = 2

_ERR_NAMES = {
    NBX_ERR_ARG: "NBX_ERR_ARG",
    NBX_ERR_CAPACITY: "NBX_ERR_CAPACITY",
    NBX_ERR_STATE: "NBX_ERR_STATE",
    NBX_ERR_DEVICE: "NBX_ERR_DEVICE",
    NBX_ERR_NO_DEVICE: "NBX_ERR_NO_DEVICE",
    NBX_ERR_OOM: "NBX_ERR_OOM",
}

# Every symbol include/nbx.h declares.
EXPORTS = (
    "nbx_version", "nbx_device_count", "nbx_open", "nbx_close", "nbx_last_error", "nbx_set_precision",
    "nbx_set_nj", "nbx_set_j", "nbx_predict", "nbx_force", "nbx_force_ext", "nbx_get_force", "nbx_get_nbr",
    "nbx_get_predicted", "nbx_get_j", "nbx_set_j_dev", "nbx_force_dev", "nbx_sync", "nbx_launch_shape",
    "nbx_batch_setup", "nbx_batch_tune", "nbx_batch_force_dev", "nbx_force_vjp_dev",
    "nbx_bs_init", "nbx_bs_step", "nbx_bs_run", "nbx_bs_get_state", "nbx_bs_energy", "nbx_tune",
    "nbx_get_crackle", "nbx_force8_dev", "nbx_force_ext8", "nbx_clock_sample", "nbx_clock_rates",
    "nbx_force_dev_noalloc",
)
NBX_NOALLOC_SCRATCH_BYTES = 64 << 20
NBX_BATCH_NMAX = 128


class nbx_config(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int),
        ("order", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("nj_max", ctypes.c_int),
        ("ni_max", ctypes.c_int),
        ("nbr_max", ctypes.c_int),
        ("want_nn", ctypes.c_int),
    ]


class nbx_bs_params(ctypes.Structure):
    _fields_ = [
        ("eps2", ctypes.c_double),
        ("eta4", ctypes.c_double),
        ("eta6", ctypes.c_double),
        ("eta_start", ctypes.c_double),
        ("dt_max", ctypes.c_double),
        ("dt_min", ctypes.c_double),
    ]


class nbx_bs_stats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("block_steps", ctypes.c_int64),
        ("particle_steps", ctypes.c_int64),
    ]


class NbxError(RuntimeError):
    def __init__(self, code, message):
        super().__init__("%s (%d): %s" % (_ERR_NAMES.get(code, "NBX_ERR"), code, message))
        self.code = code


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double


def load(path: str = LIB_PATH):
    """Load libnbx.so and declare the signatures of every exported function."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libnbx.so is not built (%s); run __graft_entry__.build()" % path)
    # torch ships its own HIP runtime with the same SONAME (libamdhip64.so.7) as the one libnbx
    # links against.  Importing torch first makes the dynamic loader bind libnbx to torch's copy,
    # so the process has one HIP runtime and torch tensors/streams are valid in libnbx calls.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    sig = {
        "nbx_version": ([], _I),
        "nbx_device_count": ([_P], _I),
        "nbx_open": ([_P, ctypes.POINTER(nbx_config)], _I),
        "nbx_close": ([_P], _I),
        "nbx_last_error": ([_P], ctypes.c_char_p),
        "nbx_set_precision": ([_P, _I], _I),
        "nbx_set_nj": ([_P, _I], _I),
        "nbx_set_j": ([_P, _I] + [_P] * 10, _I),
        "nbx_predict": ([_P, _D], _I),
        "nbx_force": ([_P, _I, _P, _D, _P], _I),
        "nbx_force_ext": ([_P, _I, _P, _P, _P, _P, _D, _P], _I),
        "nbx_get_force": ([_P] * 7, _I),
        "nbx_get_nbr": ([_P, _P, _P], _I),
        "nbx_get_predicted": ([_P, _I, _P, _P, _P, _P], _I),
        "nbx_get_j": ([_P, _I] + [_P] * 10, _I),
        "nbx_set_j_dev": ([_P, _P, _I] + [_P] * 10, _I),
        "nbx_force_dev": ([_P, _P, _I, _P, _D] + [_P] * 9, _I),
        "nbx_sync": ([_P, _P], _I),
        "nbx_launch_shape": ([_P, _I, _P, _P, _P, _P], _I),
        "nbx_batch_setup": ([_P, _I, _P], _I),
        "nbx_batch_tune": ([_P, _P, _P, _P, _P, _D, _P, _P, _P, _P], _I),
        "nbx_batch_force_dev": ([_P, _P, _P, _P, _P, _D, _P, _P, _P], _I),
        "nbx_force_vjp_dev": ([_P, _P, _I, _P, _P, _P, _D, _P, _P, _P, _P, _P, _P], _I),
        "nbx_bs_init": ([_P, _I, _P, _P, _P, _P, ctypes.POINTER(nbx_bs_params)], _I),
        "nbx_bs_step": ([_P, _D, _P], _I),
        "nbx_bs_run": ([_P, _D, ctypes.POINTER(nbx_bs_stats)], _I),
        "nbx_bs_get_state": ([_P, _P, _P, _P, _P, _P, ctypes.POINTER(nbx_bs_stats)], _I),
        "nbx_bs_energy": ([_P, _P, _P], _I),
        "nbx_tune": ([_P, _I, _P, _I], _I),
        "nbx_get_crackle": ([_P, _P], _I),
        "nbx_force8_dev": ([_P, _P, _I, _P, _D] + [_P] * 10, _I),
        "nbx_force_ext8": ([_P, _I, _P, _P, _P, _P, _P, _D, _P], _I),
        "nbx_clock_sample": ([_P, _P, _I, _P], _I),
        "nbx_clock_rates": ([_P, _P, _P], _I),
        "nbx_force_dev_noalloc": ([_P, _P, _I, _P, _D] + [_P] * 9, _I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(ctx, rc):
    if rc < 0:
        msg = load().nbx_last_error(ctx)
        raise NbxError(rc, msg.decode() if msg else "")
    return rc


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def _f64(a, n=None, width=3):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        want = (n, width) if width else (n,)
        if a.shape != want:
            raise ValueError("expected shape %s, got %s" % (want, a.shape))
    return a


# What the binding knows about each open context (keyed by the handle's value): the device and
# order it was opened with, its neighbour-list capacity, and the particle count of its batch.
_CTX_INFO = {}

_DTYPE_NAMES = {"f64": "float64", "i32": "int32", "i64": "int64"}


_TORCH_DTYPES = {}


def _torch_dtype(kind):
    if not _TORCH_DTYPES:
        import torch

        _TORCH_DTYPES.update({"f64": torch.float64, "i32": torch.int32, "i64": torch.int64})
    return _TORCH_DTYPES[kind]


def _dptr(t, kind=None, numel=0, ctx=None, name="array"):
    """Device pointer of one torch tensor (see _dptrs); an int passes through as a raw device
    address, None as NULL."""
    return _dptrs(ctx, [(name, t, kind, numel)])[0]


def _dptrs(ctx, specs):
    """Device pointers of the tensors in specs, a list of (name, tensor, kind, numel).  A tensor must
    have the dtype the C ABI reads (kind: "f64", "i32" or "i64"), be contiguous, hold at least numel
    elements and live on the context's GPU; otherwise ValueError is raised before any library call,
    because the kernels would read or write past the tensor.  The layout checks run over every
    tensor before the placement checks.  Ints pass through as raw device addresses, None as NULL.
    (The checks use the cheap tensor queries, dtype identity, is_cuda and get_device: at small N_i
    a force call's host time is on the critical path of the step.)"""
    for name, t, kind, numel in specs:
        if t is None or isinstance(t, int):
            continue
        if kind is not None and t.dtype is not _torch_dtype(kind):
            raise ValueError("%s: dtype %s, the library reads %s" % (name, t.dtype, _DTYPE_NAMES[kind]))
        if not t.is_contiguous():
            raise ValueError("%s: tensor is not contiguous" % name)
        if t.numel() < numel:
            raise ValueError("%s: %d elements, the call needs %d" % (name, t.numel(), numel))
    info = _CTX_INFO.get(getattr(ctx, "value", None))
    dev = info["device"] if info is not None else None
    out = []
    for name, t, kind, numel in specs:
        if t is None or isinstance(t, int):
            out.append(t)
            continue
        if not t.is_cuda:
            raise ValueError("%s: tensor is on %s, not on a GPU" % (name, t.device))
        if dev is not None and t.get_device() != dev:
            raise ValueError("%s: tensor is on cuda:%d, the context on cuda:%d" % (name, t.get_device(), dev))
        out.append(t.data_ptr())
    return out


def _ctx_order(ctx, default=4):
    info = _CTX_INFO.get(getattr(ctx, "value", None))
    return info["order"] if info is not None else default


def _stream(s):
    if s is None:
        import torch

        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


# ------------------------------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ------------------------------------------------------------------------------------------------
def nbx_version() -> int:
    return load().nbx_version()


def nbx_device_count() -> int:
    n = ctypes.c_int(0)
    rc = load().nbx_device_count(ctypes.byref(n))
    return n.value if rc == NBX_OK else 0


def nbx_open(device=0, order=4, precision=NBX_FP64, nj_max=1, ni_max=1, nbr_max=0, want_nn=True):
    cfg = nbx_config(device, order, precision, nj_max, ni_max, nbr_max, 1 if want_nn else 0)
    ctx = ctypes.c_void_p()
    rc = load().nbx_open(ctypes.byref(ctx), ctypes.byref(cfg))
    if rc < 0:
        raise NbxError(rc, load().nbx_last_error(None).decode())
    _CTX_INFO[ctx.value] = {"device": int(device), "order": int(order), "nbr_max": int(nbr_max), "batch_n": 0,
                            "want_nn": bool(want_nn)}
    return ctx


def nbx_close(ctx):
    _CTX_INFO.pop(getattr(ctx, "value", None), None)
    return load().nbx_close(ctx)


def nbx_last_error(ctx) -> str:
    return load().nbx_last_error(ctx).decode()


def nbx_set_precision(ctx, precision):
    return _check(ctx, load().nbx_set_precision(ctx, precision))


def nbx_set_nj(ctx, nj):
    return _check(ctx, load().nbx_set_nj(ctx, int(nj)))


def nbx_set_j(ctx, addr, id, m, t, x, v, a, jerk, snap=None, crackle=None):
    addr = np.ascontiguousarray(addr, dtype=np.int32)
    n = addr.shape[0]
    id = np.ascontiguousarray(id, dtype=np.int64)
    m, t = _f64(m, n, 0), _f64(t, n, 0)
    x, v, a, jerk = _f64(x, n), _f64(v, n), _f64(a, n), _f64(jerk, n)  # v, a, jerk: None allowed for order 2
    snap, crackle = _f64(snap, n), _f64(crackle, n)
    if id.shape != (n,):
        raise ValueError("id must have shape (n,)")
    rc = load().nbx_set_j(ctx, n, _ptr(addr), _ptr(id), _ptr(m), _ptr(t), _ptr(x), _ptr(v), _ptr(a), _ptr(jerk),
                          _ptr(snap), _ptr(crackle))
    return _check(ctx, rc)


def nbx_predict(ctx, t):
    return _check(ctx, load().nbx_predict(ctx, float(t)))


def nbx_force(ctx, i_addr, eps2, h2=None):
    i_addr = np.ascontiguousarray(i_addr, dtype=np.int32)
    n = i_addr.shape[0]
    h2 = None if h2 is None else _f64(np.broadcast_to(np.asarray(h2, dtype=np.float64), (n,)), n, 0)
    return _check(ctx, load().nbx_force(ctx, n, _ptr(i_addr), float(eps2), _ptr(h2)))


def nbx_force_ext(ctx, id, x, v, a, eps2, h2=None):
    x = _f64(x)
    n = x.shape[0]
    id = np.ascontiguousarray(id, dtype=np.int64)
    v = None if v is None else _f64(v, n)
    a = None if a is None else _f64(a, n)
    h2 = None if h2 is None else _f64(np.broadcast_to(np.asarray(h2, dtype=np.float64), (n,)), n, 0)
    return _check(ctx, load().nbx_force_ext(ctx, n, _ptr(id), _ptr(x), _ptr(v), _ptr(a), float(eps2), _ptr(h2)))


def nbx_force_ext8(ctx, id, x, v, a, jerk, eps2, h2=None):
    x = _f64(x)
    n = x.shape[0]
    id = np.ascontiguousarray(id, dtype=np.int64)
    v, a, jerk = _f64(v, n), _f64(a, n), _f64(jerk, n)
    h2 = None if h2 is None else _f64(np.broadcast_to(np.asarray(h2, dtype=np.float64), (n,)), n, 0)
    return _check(ctx, load().nbx_force_ext8(ctx, n, _ptr(id), _ptr(x), _ptr(v), _ptr(a), _ptr(jerk), float(eps2),
                                              _ptr(h2)))


def nbx_get_force(ctx, ni, order=4):
    """Results of the last force call on ni sinks, as a dict of numpy arrays (plus 'status');
    order 8 adds 'crackle' (read by nbx_get_crackle).  nn_id and nn_r2 are None for a context
    opened with want_nn=False."""
    info = _CTX_INFO.get(getattr(ctx, "value", None))
    nn = info is None or info.get("want_nn", True)
    out = {
        "acc": np.empty((ni, 3)),
        "jerk": np.empty((ni, 3)) if order != 2 else None,
        "snap": np.empty((ni, 3)) if order >= 6 else None,
        "pot": np.empty(ni),
        "nn_id": np.empty(ni, dtype=np.int64) if nn else None,
        "nn_r2": np.empty(ni) if nn else None,
    }
    rc = load().nbx_get_force(ctx, _ptr(out["acc"]), _ptr(out["jerk"]), _ptr(out["snap"]), _ptr(out["pot"]),
                              _ptr(out["nn_id"]), _ptr(out["nn_r2"]))
    out["status"] = _check(ctx, rc)
    if order == 8:
        out["crackle"] = nbx_get_crackle(ctx, ni)
    return out


def nbx_get_crackle(ctx, ni):
    crackle = np.empty((ni, 3))
    _check(ctx, load().nbx_get_crackle(ctx, _ptr(crackle)))
    return crackle


def nbx_get_nbr(ctx, ni, nbr_max):
    count = np.empty(ni, dtype=np.int32)
    ids = np.empty((ni, nbr_max), dtype=np.int64)
    rc = _check(ctx, load().nbx_get_nbr(ctx, _ptr(count), _ptr(ids)))
    return count, ids, rc


def nbx_get_predicted(ctx, addr, order=4):
    addr = np.ascontiguousarray(addr, dtype=np.int32)
    n = addr.shape[0]
    xp, vp, ap = np.empty((n, 3)), np.empty((n, 3)), np.empty((n, 3))
    _check(ctx, load().nbx_get_predicted(ctx, n, _ptr(addr), _ptr(xp), _ptr(vp), _ptr(ap)))
    return xp, vp, ap


def nbx_get_j(ctx, addr, order=4):
    addr = np.ascontiguousarray(addr, dtype=np.int32)
    n = addr.shape[0]
    out = {"id": np.empty(n, dtype=np.int64), "m": np.empty(n), "t": np.empty(n)}
    for k in ("x", "v", "a", "jerk") + (("snap", "crackle") if order >= 6 else ()):
        out[k] = np.empty((n, 3))
    rc = load().nbx_get_j(ctx, n, _ptr(addr), _ptr(out["id"]), _ptr(out["m"]), _ptr(out["t"]), _ptr(out["x"]),
                          _ptr(out["v"]), _ptr(out["a"]), _ptr(out["jerk"]), _ptr(out.get("snap")),
                          _ptr(out.get("crackle")))
    _check(ctx, rc)
    return out


def nbx_set_j_dev(ctx, stream, n, d_addr, d_id, d_m, d_t, d_x, d_v, d_a, d_jerk, d_snap=None, d_crackle=None):
    n = int(n)
    args = _dptrs(ctx, [("d_addr", d_addr, "i32", n), ("d_id", d_id, "i64", n), ("d_m", d_m, "f64", n),
                        ("d_t", d_t, "f64", n), ("d_x", d_x, "f64", 3 * n), ("d_v", d_v, "f64", 3 * n),
                        ("d_a", d_a, "f64", 3 * n), ("d_jerk", d_jerk, "f64", 3 * n),
                        ("d_snap", d_snap, "f64", 3 * n), ("d_crackle", d_crackle, "f64", 3 * n)])
    rc = load().nbx_set_j_dev(ctx, _stream(stream), n, *args)
    return _check(ctx, rc)


def _force_dev_args(ctx, ni, d_i_addr, d_h2, outs, d_nbr_count, d_nbr_ids):
    """Validated device pointers of the force entry points: sink addresses, radii, the [ni][3] and
    [ni] outputs (outs: (name, tensor, kind, width) in ABI order) and the neighbour-list arrays."""
    info = _CTX_INFO.get(getattr(ctx, "value", None))
    nbr_max = info["nbr_max"] if info is not None else 0
    lists = d_h2 is not None
    specs = [("d_i_addr", d_i_addr, "i32", ni), ("d_h2", d_h2, "f64", ni)]
    specs += [(name, t, kind, width * ni) for name, t, kind, width in outs]
    specs += [("d_nbr_count", d_nbr_count, "i32", ni if lists else 0),
              ("d_nbr_ids", d_nbr_ids, "i64", ni * nbr_max if lists else 0)]
    return _dptrs(ctx, specs)


def nbx_force_dev(ctx, stream, ni, d_i_addr, eps2, d_h2, d_acc, d_jerk, d_snap, d_pot, d_nn_id, d_nn_r2,
                  d_nbr_count=None, d_nbr_ids=None):
    ni = int(ni)
    p = _force_dev_args(ctx, ni, d_i_addr, d_h2,
                        (("d_acc", d_acc, "f64", 3), ("d_jerk", d_jerk, "f64", 3), ("d_snap", d_snap, "f64", 3),
                         ("d_pot", d_pot, "f64", 1), ("d_nn_id", d_nn_id, "i64", 1), ("d_nn_r2", d_nn_r2, "f64", 1)),
                        d_nbr_count, d_nbr_ids)
    rc = load().nbx_force_dev(ctx, _stream(stream), ni, p[0], float(eps2), *p[1:])
    return _check(ctx, rc)


def nbx_force_dev_noalloc(ctx, stream, ni, d_i_addr, eps2, d_h2, d_acc, d_jerk, d_snap, d_pot, d_nn_id, d_nn_r2,
                          d_nbr_count=None, d_nbr_ids=None):
    ni = int(ni)
    p = _force_dev_args(ctx, ni, d_i_addr, d_h2,
                        (("d_acc", d_acc, "f64", 3), ("d_jerk", d_jerk, "f64", 3), ("d_snap", d_snap, "f64", 3),
                         ("d_pot", d_pot, "f64", 1), ("d_nn_id", d_nn_id, "i64", 1), ("d_nn_r2", d_nn_r2, "f64", 1)),
                        d_nbr_count, d_nbr_ids)
    rc = load().nbx_force_dev_noalloc(ctx, _stream(stream), ni, p[0], float(eps2), *p[1:])
    return _check(ctx, rc)


def nbx_force8_dev(ctx, stream, ni, d_i_addr, eps2, d_h2, d_acc, d_jerk, d_snap, d_crackle, d_pot, d_nn_id,
                   d_nn_r2, d_nbr_count=None, d_nbr_ids=None):
    ni = int(ni)
    p = _force_dev_args(ctx, ni, d_i_addr, d_h2,
                        (("d_acc", d_acc, "f64", 3), ("d_jerk", d_jerk, "f64", 3), ("d_snap", d_snap, "f64", 3),
                         ("d_crackle", d_crackle, "f64", 3), ("d_pot", d_pot, "f64", 1),
                         ("d_nn_id", d_nn_id, "i64", 1), ("d_nn_r2", d_nn_r2, "f64", 1)),
                        d_nbr_count, d_nbr_ids)
    rc = load().nbx_force8_dev(ctx, _stream(stream), ni, p[0], float(eps2), *p[1:])
    return _check(ctx, rc)


def nbx_clock_sample(ctx, stream, n_groups, d_out):
    """Enqueue a clock sample: d_out (int64 device tensor, >= 3 n_groups) receives per workgroup
    (XCD, shader-clock cycles, constant-rate ticks)."""
    p = _dptrs(ctx, [("d_out", d_out, "i64", 3 * int(n_groups))])
    return _check(ctx, load().nbx_clock_sample(ctx, _stream(stream), int(n_groups), p[0]))


def nbx_clock_rates(ctx):
    """(constant counter rate, nominal maximum shader clock), in kHz."""
    w, s = ctypes.c_int(0), ctypes.c_int(0)
    _check(ctx, load().nbx_clock_rates(ctx, ctypes.byref(w), ctypes.byref(s)))
    return w.value, s.value


def nbx_sync(ctx, stream=0):
    return _check(ctx, load().nbx_sync(ctx, _stream(stream) if stream != 0 else None))


def nbx_launch_shape(ctx, ni):
    vals = [ctypes.c_int(0) for _ in range(4)]
    rc = load().nbx_launch_shape(ctx, int(ni), *[ctypes.byref(v) for v in vals])
    if rc < 0:
        raise NbxError(rc, "bad arguments")
    return {"lanes_per_sink": vals[0].value, "sinks_per_lane": vals[1].value, "splits": vals[2].value,
            "workgroups": vals[3].value}


def nbx_tune(ctx, ni_max):
    """Tune the launch shape per N_i class; returns an (n_classes, 3) array of (L, P, S)."""
    k = 0
    while (1 << k) < ni_max:
        k += 1
    out = np.zeros((k + 1, 3), dtype=np.int32)
    _check(ctx, load().nbx_tune(ctx, int(ni_max), _ptr(out), int(k + 1)))
    return out


def nbx_batch_setup(ctx, offsets):
    offsets = np.ascontiguousarray(offsets, dtype=np.int32)
    rc = _check(ctx, load().nbx_batch_setup(ctx, int(offsets.shape[0] - 1), _ptr(offsets)))
    info = _CTX_INFO.get(getattr(ctx, "value", None))
    if info is not None:
        info["batch_n"] = int(offsets[-1])
    return rc


def _batch_args(ctx, d_m, d_x, d_v, d_acc, d_jerk, d_pot):
    info = _CTX_INFO.get(getattr(ctx, "value", None))
    n = info["batch_n"] if info is not None else 0
    return _dptrs(ctx, [("d_m", d_m, "f64", n), ("d_x", d_x, "f64", 3 * n), ("d_v", d_v, "f64", 3 * n),
                        ("d_acc", d_acc, "f64", 3 * n), ("d_jerk", d_jerk, "f64", 3 * n),
                        ("d_pot", d_pot, "f64", n)])


def nbx_batch_tune(ctx, stream, d_m, d_x, d_v, eps2, d_acc, d_jerk, d_pot):
    """Returns the lanes-per-sink chosen for each of the 8 size classes (0: class absent)."""
    p = _batch_args(ctx, d_m, d_x, d_v, d_acc, d_jerk, d_pot)
    lanes = np.zeros(8, dtype=np.int32)
    rc = load().nbx_batch_tune(ctx, _stream(stream), p[0], p[1], p[2], float(eps2), p[3], p[4], p[5], _ptr(lanes))
    _check(ctx, rc)
    return lanes


def nbx_batch_force_dev(ctx, stream, d_m, d_x, d_v, eps2, d_acc, d_jerk, d_pot):
    p = _batch_args(ctx, d_m, d_x, d_v, d_acc, d_jerk, d_pot)
    rc = load().nbx_batch_force_dev(ctx, _stream(stream), p[0], p[1], p[2], float(eps2), p[3], p[4], p[5])
    return _check(ctx, rc)


def nbx_force_vjp_dev(ctx, stream, n, d_m, d_x, d_v, eps2, d_g_acc, d_g_jerk, d_g_pot, d_grad_x, d_grad_v, d_grad_m):
    n = int(n)
    p = _dptrs(ctx, [("d_m", d_m, "f64", n), ("d_x", d_x, "f64", 3 * n), ("d_v", d_v, "f64", 3 * n),
                     ("d_g_acc", d_g_acc, "f64", 3 * n), ("d_g_jerk", d_g_jerk, "f64", 3 * n),
                     ("d_g_pot", d_g_pot, "f64", n), ("d_grad_x", d_grad_x, "f64", 3 * n),
                     ("d_grad_v", d_grad_v, "f64", 3 * n), ("d_grad_m", d_grad_m, "f64", n)])
    rc = load().nbx_force_vjp_dev(ctx, _stream(stream), n, p[0], p[1], p[2], float(eps2), *p[3:])
    return _check(ctx, rc)


def nbx_bs_init(ctx, id, m, x, v, eps2, eta4=0.01, eta6=0.1, eta_start=0.01, dt_max=0.125, dt_min=2.0**-30):
    x = _f64(x)
    n = x.shape[0]
    id = np.ascontiguousarray(id, dtype=np.int64)
    m, v = _f64(m, n, 0), _f64(v, n)
    if id.shape != (n,):
        raise ValueError("id must have shape (n,)")
    p = nbx_bs_params(float(eps2), float(eta4), float(eta6), float(eta_start), float(dt_max), float(dt_min))
    return _check(ctx, load().nbx_bs_init(ctx, n, _ptr(id), _ptr(m), _ptr(x), _ptr(v), ctypes.byref(p)))


def nbx_bs_step(ctx, t_end):
    """One block step if due by t_end; returns (N_active, status): N_active 0 when no step was
    taken, status NBX_WARN_DT_MIN once a step has collapsed to dt_min."""
    ni = ctypes.c_int(0)
    rc = _check(ctx, load().nbx_bs_step(ctx, float(t_end), ctypes.byref(ni)))
    return ni.value, rc


def _stats(st):
    return {"t": st.t, "block_steps": st.block_steps, "particle_steps": st.particle_steps}


def nbx_bs_run(ctx, t_end):
    st = nbx_bs_stats()
    rc = _check(ctx, load().nbx_bs_run(ctx, float(t_end), ctypes.byref(st)))
    out = _stats(st)
    out["status"] = rc
    return out


def nbx_bs_get_state(ctx, n):
    t = ctypes.c_double(0.0)
    x, v, dt, ti = np.empty((n, 3)), np.empty((n, 3)), np.empty(n), np.empty(n)
    st = nbx_bs_stats()
    rc = _check(ctx, load().nbx_bs_get_state(ctx, ctypes.byref(t), _ptr(x), _ptr(v), _ptr(dt), _ptr(ti),
                                             ctypes.byref(st)))
    out = {"t": t.value, "x": x, "v": v, "dt": dt, "t_i": ti, "status": rc}
    out.update({k: val for k, val in _stats(st).items() if k != "t"})
    return out


def nbx_bs_energy(ctx):
    ek, ep = ctypes.c_double(0.0), ctypes.c_double(0.0)
    _check(ctx, load().nbx_bs_energy(ctx, ctypes.byref(ek), ctypes.byref(ep)))
    return ek.value, ep.value


class Context:
    """Owns one nbx context; thin convenience wrapper over the entry points above."""

    def __init__(self, order=4, precision=NBX_FP64, nj_max=1, ni_max=1, nbr_max=0, device=0, want_nn=True):
        self.order = order
        self.nbr_max = nbr_max
        self.ctx = nbx_open(device, order, precision, nj_max, ni_max, nbr_max, want_nn)
        self._ni = None

    def close(self):
        if self.ctx is not None:
            nbx_close(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_precision(self, p):
        return nbx_set_precision(self.ctx, p)

    def set_nj(self, nj):
        return nbx_set_nj(self.ctx, nj)

    def set_sources(self, src, addr=None):
        """Load a nbody_ics.SourceSet-like object (fields ids, m, t, x, v, a, jerk[, snap, crackle])."""
        addr = np.arange(src.n, dtype=np.int32) if addr is None else addr
        return nbx_set_j(self.ctx, addr, src.ids, src.m, src.t, src.x, src.v, src.a,
                         src.jerk if self.order != 2 else None,
                         src.snap if self.order >= 6 else None, src.crackle if self.order >= 6 else None)

    def predict(self, t):
        return nbx_predict(self.ctx, t)

    def force(self, i_addr, eps2, h2=None):
        self._ni = len(i_addr)
        return nbx_force(self.ctx, i_addr, eps2, h2)

    def force_ext(self, ids, x, v, a, eps2, h2=None, jerk=None):
        """Explicit sinks; order 8 also takes the sink jerks."""
        self._ni = len(ids)
        if self.order == 8:
            return nbx_force_ext8(self.ctx, ids, x, v, a, jerk, eps2, h2)
        return nbx_force_ext(self.ctx, ids, x, v, a, eps2, h2)

    def get_force(self):
        return nbx_get_force(self.ctx, self._ni, self.order)

    def get_nbr(self):
        """(count[ni], ids[ni][nbr_max], status) of the last force call."""
        return nbx_get_nbr(self.ctx, self._ni, self.nbr_max)

    def get_predicted(self, addr):
        return nbx_get_predicted(self.ctx, addr, self.order)

    def get_j(self, addr):
        return nbx_get_j(self.ctx, addr, self.order)

    def tune(self, ni_max):
        return nbx_tune(self.ctx, ni_max)

    def launch_shape(self, ni):
        return nbx_launch_shape(self.ctx, ni)
