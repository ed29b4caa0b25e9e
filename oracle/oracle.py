"""ctypes front end of the C oracle (see ``oracle.c`` for the definitions).

TEST INFRASTRUCTURE ONLY -- nothing on the product path may import this.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "_build", "liboracle.so")

# -O2, no fast-math, no FMA contraction: each per-pair term is the plain IEEE
# double expression; sums are long double.
CFLAGS = ["-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math", "-std=c11"]

_lib = None


def lib_path() -> str:
    return _LIB


def build(force_rebuild: bool = True) -> str:
    """Compile oracle.c into oracle/_build/liboracle.so with gcc."""
    global _lib
    os.makedirs(os.path.dirname(_LIB), exist_ok=True)
    if force_rebuild or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force_rebuild=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int32)
        lib.oracle_predict.restype = ctypes.c_int
        lib.oracle_predict.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double] + [dp] * 10
        lib.oracle_force.restype = ctypes.c_int
        lib.oracle_force.argtypes = (
            [ctypes.c_int, ctypes.c_double, ctypes.c_int, lp, dp, dp, dp, dp, ctypes.c_int, lp, dp, dp, dp, dp,
             ctypes.c_int, dp, dp, dp, dp, lp, dp, ip, lp, dp, ctypes.c_int]
        )
        lib.oracle_force8.restype = ctypes.c_int
        lib.oracle_force8.argtypes = (
            [ctypes.c_double, ctypes.c_int, lp, dp, dp, dp, dp, dp, ctypes.c_int, lp, dp, dp, dp, dp, dp,
             ctypes.c_int, dp, dp, dp, dp, dp, lp, dp, ip, lp, dp, ctypes.c_int]
        )
        lib.oracle_predict_jerk.restype = ctypes.c_int
        lib.oracle_predict_jerk.argtypes = [ctypes.c_int, ctypes.c_double] + [dp] * 5
        lib.oracle_force_vjp.restype = ctypes.c_int
        lib.oracle_force_vjp.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp, dp, dp, dp, dp, ctypes.c_int, ip, dp,
                                         dp, dp, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def _ptr(a, ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        raise ValueError("expected shape %s, got %s" % (shape, a.shape))
    return a


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def predict(order, t, tj, x, v, a, jerk, snap=None, crackle=None):
    """Taylor-predict every particle from its own time tj to t.

    Returns (xp, vp, ap); ap is the predicted acceleration (6th and 8th
    order), for order 4 it is a + jerk*dt and for order 2 it is a (returned
    for convenience, unused by 2nd- and 4th-order forces).  jerk may be None
    for order 2.  Order 8 predicts x, v, a as order 6 (see predict_jerk).
    """
    lib = _load()
    x = _f64(x)
    n = x.shape[0]
    tj = _f64(tj, (n,))
    v, a = _f64(v, (n, 3)), _f64(a, (n, 3))
    jerk = _f64(jerk, (n, 3)) if order != 2 else None
    snap = _f64(snap, (n, 3)) if order >= 6 else None
    crackle = _f64(crackle, (n, 3)) if order >= 6 else None
    xp, vp, ap = np.empty((n, 3)), np.empty((n, 3)), np.empty((n, 3))
    d = ctypes.c_double
    rc = lib.oracle_predict(n, order, float(t), _ptr(tj, d), _ptr(x, d), _ptr(v, d), _ptr(a, d), _ptr(jerk, d),
                            _ptr(snap, d), _ptr(crackle, d), _ptr(xp, d), _ptr(vp, d), _ptr(ap, d))
    if rc != 0:
        raise ValueError("oracle_predict rejected its arguments")
    return xp, vp, ap


def predict_jerk(t, tj, jerk, snap, crackle):
    """8th-order mode: the predicted jerk, jerk + snap dt + crackle dt^2/2."""
    lib = _load()
    jerk = _f64(jerk)
    n = jerk.shape[0]
    tj, snap, crackle = _f64(tj, (n,)), _f64(snap, (n, 3)), _f64(crackle, (n, 3))
    jp = np.empty((n, 3))
    d = ctypes.c_double
    rc = lib.oracle_predict_jerk(n, float(t), _ptr(tj, d), _ptr(jerk, d), _ptr(snap, d), _ptr(crackle, d),
                                 _ptr(jp, d))
    if rc != 0:
        raise ValueError("oracle_predict_jerk rejected its arguments")
    return jp


def force8(eps2, idj, mj, xj, vj, aj, jj, idi, xi, vi, ai, ji, h2=None, nbr_max=0, nthreads=0):
    """8th-order mode: acc, jerk, snap, crackle, pot, nn_id, nn_r2, cond [ni][4] (and the neighbour
    lists when h2 is given) of the sources (with their accelerations aj and jerks jj) on the sinks."""
    lib = _load()
    xj = _f64(xj)
    nj = xj.shape[0]
    xi = _f64(xi)
    ni = xi.shape[0]
    idj = np.ascontiguousarray(idj, dtype=np.int64)
    idi = np.ascontiguousarray(idi, dtype=np.int64)
    mj = _f64(mj, (nj,))
    vj, aj, jj = _f64(vj, (nj, 3)), _f64(aj, (nj, 3)), _f64(jj, (nj, 3))
    vi, ai, ji = _f64(vi, (ni, 3)), _f64(ai, (ni, 3)), _f64(ji, (ni, 3))
    if idj.shape != (nj,) or idi.shape != (ni,):
        raise ValueError("id arrays have the wrong length")
    if h2 is not None:
        h2 = _f64(np.broadcast_to(np.asarray(h2, dtype=np.float64), (ni,)).copy(), (ni,))
    out = {
        "acc": np.zeros((ni, 3)), "jerk": np.zeros((ni, 3)), "snap": np.zeros((ni, 3)),
        "crackle": np.zeros((ni, 3)), "pot": np.zeros(ni), "nn_id": np.zeros(ni, dtype=np.int64),
        "nn_r2": np.zeros(ni), "cond": np.zeros((ni, 4)),
        "nbr_count": np.zeros(ni, dtype=np.int32) if h2 is not None else None,
        "nbr_ids": np.full((ni, max(nbr_max, 0)), -1, dtype=np.int64) if h2 is not None else None,
    }
    d, L, I = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    rc = lib.oracle_force8(
        float(eps2), nj, _ptr(idj, L), _ptr(mj, d), _ptr(xj, d), _ptr(vj, d), _ptr(aj, d), _ptr(jj, d), ni,
        _ptr(idi, L), _ptr(xi, d), _ptr(vi, d), _ptr(ai, d), _ptr(ji, d), _ptr(h2, d), int(nbr_max),
        _ptr(out["acc"], d), _ptr(out["jerk"], d), _ptr(out["snap"], d), _ptr(out["crackle"], d),
        _ptr(out["pot"], d), _ptr(out["nn_id"], L), _ptr(out["nn_r2"], d), _ptr(out["nbr_count"], I),
        _ptr(out["nbr_ids"], L), _ptr(out["cond"], d), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_force8 rejected its arguments")
    return out


def force(order, eps2, idj, mj, xj, vj, idi, xi, vi, aj=None, ai=None, h2=None, nbr_max=0, nthreads=0):
    """Direct-summation forces of the sources (j) on the sinks (i).

    Returns a dict with acc, jerk (orders 4, 6), snap (6th order), pot, nn_id,
    nn_r2, cond (sum of |term| per sink for acc/jerk/snap) and, when h2 is
    given, nbr_count and nbr_ids (first nbr_max ids in source order, -1
    padded).  Order 2 (GRAPE-5 mode) needs no velocities (vj, vi may be None).
    """
    lib = _load()
    xj = _f64(xj)
    nj = xj.shape[0]
    xi = _f64(xi)
    ni = xi.shape[0]
    idj = np.ascontiguousarray(idj, dtype=np.int64)
    idi = np.ascontiguousarray(idi, dtype=np.int64)
    mj = _f64(mj, (nj,))
    vj = _f64(vj, (nj, 3)) if order != 2 else None
    vi = _f64(vi, (ni, 3)) if order != 2 else None
    if idj.shape != (nj,) or idi.shape != (ni,):
        raise ValueError("id arrays have the wrong length")
    aj = _f64(aj, (nj, 3)) if order == 6 else None
    ai = _f64(ai, (ni, 3)) if order == 6 else None
    if h2 is not None:
        h2 = _f64(np.broadcast_to(np.asarray(h2, dtype=np.float64), (ni,)).copy(), (ni,))
    out = {
        "acc": np.zeros((ni, 3)),
        "jerk": np.zeros((ni, 3)) if order != 2 else None,
        "snap": np.zeros((ni, 3)) if order == 6 else None,
        "pot": np.zeros(ni),
        "nn_id": np.zeros(ni, dtype=np.int64),
        "nn_r2": np.zeros(ni),
        "cond": np.zeros((ni, 3)),
        "nbr_count": np.zeros(ni, dtype=np.int32) if h2 is not None else None,
        "nbr_ids": np.full((ni, max(nbr_max, 0)), -1, dtype=np.int64) if h2 is not None else None,
    }
    d, L, I = ctypes.c_double, ctypes.c_int64, ctypes.c_int32
    rc = lib.oracle_force(
        order, float(eps2), nj, _ptr(idj, L), _ptr(mj, d), _ptr(xj, d), _ptr(vj, d), _ptr(aj, d), ni, _ptr(idi, L),
        _ptr(xi, d), _ptr(vi, d), _ptr(ai, d), _ptr(h2, d), int(nbr_max), _ptr(out["acc"], d), _ptr(out["jerk"], d),
        _ptr(out["snap"], d), _ptr(out["pot"], d), _ptr(out["nn_id"], L), _ptr(out["nn_r2"], d),
        _ptr(out["nbr_count"], I), _ptr(out["nbr_ids"], L), _ptr(out["cond"], d), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_force rejected its arguments")
    return out


def hermite4_correct(dt, xp, vp, a0, j0, a1, j1):
    """4th-order Hermite corrector (Makino & Aarseth 1992).

    From acc/jerk at the start of the step (a0, j0) and at the predicted end
    point (a1, j1), the 2nd and 3rd acceleration derivatives at the start are
    fixed by the cubic Hermite interpolant of the acceleration:
        a2 = (-6 (a0 - a1) - dt (4 j0 + 2 j1)) / dt^2
        a3 = (12 (a0 - a1) + 6 dt (j0 + j1)) / dt^3
    and the predicted position/velocity receive the matching higher terms:
        x = xp + a2 dt^4/24 + a3 dt^5/120,   v = vp + a2 dt^3/6 + a3 dt^4/24
    """
    a2 = (-6.0 * (a0 - a1) - dt * (4.0 * j0 + 2.0 * j1)) / dt**2
    a3 = (12.0 * (a0 - a1) + 6.0 * dt * (j0 + j1)) / dt**3
    x = xp + a2 * dt**4 / 24.0 + a3 * dt**5 / 120.0
    v = vp + a2 * dt**3 / 6.0 + a3 * dt**4 / 24.0
    return x, v


def total_energy(m, v, pot):
    """Kinetic plus potential energy: sum m v^2 / 2 + sum m pot / 2 (each pair once)."""
    m = np.asarray(m, dtype=np.float64)
    return float(0.5 * np.sum(m * np.sum(np.asarray(v) ** 2, axis=1)) + 0.5 * np.sum(m * np.asarray(pot)))


def force_vjp(eps2, m, x, v, g_acc, g_jerk, g_pot, sel=None, nthreads=0):
    """Gradients (grad_x, grad_v, grad_m) of sum(g_acc.acc + g_jerk.jerk + g_pot.pot) for a closed
    4th-order system (every particle a sink and a source), for the particles sel (all if None)."""
    lib = _load()
    x = _f64(x)
    n = x.shape[0]
    m, v = _f64(m, (n,)), _f64(v, (n, 3))
    g_acc, g_jerk, g_pot = _f64(g_acc, (n, 3)), _f64(g_jerk, (n, 3)), _f64(g_pot, (n,))
    if sel is None:
        nsel, selp = n, None
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int32)
        nsel, selp = sel.shape[0], sel
    gx, gv, gm = np.zeros((nsel, 3)), np.zeros((nsel, 3)), np.zeros(nsel)
    d, I = ctypes.c_double, ctypes.c_int32
    rc = lib.oracle_force_vjp(float(eps2), n, _ptr(m, d), _ptr(x, d), _ptr(v, d), _ptr(g_acc, d), _ptr(g_jerk, d),
                              _ptr(g_pot, d), nsel, _ptr(selp, I), _ptr(gx, d), _ptr(gv, d), _ptr(gm, d), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_force_vjp rejected its arguments")
    return gx, gv, gm
