"""Pin of the oracle's vector-Jacobian product (gradients of acc/jerk/pot with respect to x, v, m)
against central finite differences of the oracle's forward forces."""

import numpy as np
import pytest

import nbody_ics
import oracle

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _loss(src_m, x, v, g_acc, g_jerk, g_pot, eps2):
    ids = np.arange(len(src_m), dtype=np.int64)
    out = oracle.force(4, eps2, ids, src_m, x, v, ids, x, v)
    return float(np.sum(g_acc * out["acc"]) + np.sum(g_jerk * out["jerk"]) + np.sum(g_pot * out["pot"]))


@pytest.mark.parametrize("eps2", [1e-3, 0.05])
def test_vjp_matches_finite_differences(eps2):
    n = 12
    src = nbody_ics.make_sources(n, seed=60, masses="salpeter")
    rng = np.random.default_rng(61)
    g_acc, g_jerk, g_pot = rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.normal(size=n)
    gx, gv, gm = oracle.force_vjp(eps2, src.m, src.x, src.v, g_acc, g_jerk, g_pot)
    h = 1e-6
    fx, fv, fm = np.zeros_like(gx), np.zeros_like(gv), np.zeros_like(gm)
    for p in range(n):
        for k in range(3):
            for arr, out in ((src.x, fx), (src.v, fv)):
                a0 = arr[p, k]
                arr[p, k] = a0 + h
                lp = _loss(src.m, src.x, src.v, g_acc, g_jerk, g_pot, eps2)
                arr[p, k] = a0 - h
                lm = _loss(src.m, src.x, src.v, g_acc, g_jerk, g_pot, eps2)
                arr[p, k] = a0
                out[p, k] = (lp - lm) / (2 * h)
        m0 = src.m[p]
        src.m[p] = m0 + h * m0
        lp = _loss(src.m, src.x, src.v, g_acc, g_jerk, g_pot, eps2)
        src.m[p] = m0 - h * m0
        lm = _loss(src.m, src.x, src.v, g_acc, g_jerk, g_pot, eps2)
        src.m[p] = m0
        fm[p] = (lp - lm) / (2 * h * m0)
    for a, f in ((gx, fx), (gv, fv), (gm, fm)):
        np.testing.assert_allclose(a, f, rtol=0, atol=2e-6 * np.abs(f).max())
    # a subset gives the same rows
    sel = np.array([3, 0, 11], dtype=np.int32)
    sx, sv, sm = oracle.force_vjp(eps2, src.m, src.x, src.v, g_acc, g_jerk, g_pot, sel=sel)
    np.testing.assert_array_equal(sx, gx[sel])
    np.testing.assert_array_equal(sm, gm[sel])
