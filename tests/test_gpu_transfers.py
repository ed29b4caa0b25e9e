"""Host-pointer transfers: small ones go through the context's pinned staging buffers, large ones
(over 1 MiB) straight from and to the caller's arrays.  Both forms must give bit-identical
results: the sources loaded in one large nbx_set_j or in small chunks, sinks given explicitly in
one large call or in small batches, results read back large or small.  The launch shape is fixed
(one lane per sink, four source splits) so that a sink's sum order does not depend on N_i."""

import numpy as np
import pytest

import nbody_ics
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, say

pytestmark = pytest.mark.gpu


def _forces(ctx, sel, eps2):
    ctx.force(sel, eps2)
    return ctx.get_force()


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_staged_and_direct_transfers_agree(prec, monkeypatch):
    monkeypatch.setenv("NBX_SHAPE", "1,1,4")
    n, eps2 = 20000, 1e-4  # one nbx_set_j of all sources moves 2.5 MB; results of all sinks 1.8 MB
    say("transfers prec=%s n=%d seed=95" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=95)
    sel_all = np.arange(n, dtype=np.int32)
    sel_small = nbody_ics.active_set(n, 3000, seed=96)
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as big, \
            nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as small:
        big.set_sources(src)  # one large copy
        for k0 in range(0, n, 1500):  # small copies through the staging buffer
            k1 = min(n, k0 + 1500)
            addr = np.arange(k0, k1, dtype=np.int32)
            nbx.nbx_set_j(small.ctx, addr, src.ids[k0:k1], src.m[k0:k1], src.t[k0:k1], src.x[k0:k1],
                          src.v[k0:k1], src.a[k0:k1], src.jerk[k0:k1])
        for ctx in (big, small):
            ctx.predict(0.0)
        # all sinks (large read-back) and a subset (small read-back), on both contexts
        a_big, a_small = _forces(big, sel_all, eps2), _forces(small, sel_all, eps2)
        s_big, s_small = _forces(big, sel_small, eps2), _forces(small, sel_small, eps2)
        for key in ("acc", "jerk", "pot", "nn_id", "nn_r2"):
            np.testing.assert_array_equal(a_big[key], a_small[key])
            np.testing.assert_array_equal(s_big[key], s_small[key])
            np.testing.assert_array_equal(s_big[key], a_big[key][sel_small])
        # explicit sinks: 20000 in one call (1.1 MB of sink state) against batches of 2500
        rng = np.random.default_rng(97)
        m_ext = 20000
        ids = np.arange(10**7, 10**7 + m_ext, dtype=np.int64)
        x = rng.normal(0, 0.5, (m_ext, 3))
        v = rng.normal(0, 0.5, (m_ext, 3))
        big.force_ext(ids, x, v, None, eps2)
        one = big.get_force()
        for k0 in range(0, m_ext, 2500):
            k1 = k0 + 2500
            big.force_ext(ids[k0:k1], x[k0:k1], v[k0:k1], None, eps2)
            part = big.get_force()
            for key in ("acc", "jerk", "pot", "nn_id", "nn_r2"):
                np.testing.assert_array_equal(part[key], one[key][k0:k1])
    say("  staged and direct transfers agree bit for bit")
