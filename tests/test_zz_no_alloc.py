"""The allocation-free entry point nbx_force_dev_noalloc against nbx_force_dev, through the C ABI:
two calls in a row, the second with a smaller input.  Where the launch shape's split partials fit
the static area the two entry points run the same launches and must agree bit for bit; where they
do not (N_i = N = 131072, eight source splits) the no-alloc call uses fewer splits and agrees to
the FP64 bound, 1e-13 relative, with identical nearest neighbours."""

import numpy as np
import pytest

import nbody_ics
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, say

pytestmark = pytest.mark.gpu


def _outs(torch, ni, order, dev, fill):
    f64 = torch.float64
    o = {k: torch.full((ni, 3), fill, dtype=f64, device=dev) for k in ("acc", "jerk", "snap")}
    o["pot"] = torch.full((ni,), fill, dtype=f64, device=dev)
    o["nn_id"] = torch.full((ni,), -7, dtype=torch.int64, device=dev)
    o["nn_r2"] = torch.full((ni,), fill, dtype=f64, device=dev)
    if order == 4:
        o["snap"] = None
    return o


def _max_splits(ni, k_vals):
    """Source splits whose partials fit the static area: per split the values, key and index of
    every sink, each array rounded up to 16 bytes, after the sinks' predicted positions."""
    a16 = lambda b: (b + 15) // 16 * 16
    per_split = a16(ni * k_vals * 8) + a16(ni * 8) + a16(ni * 4)
    return (nbx.NBX_NOALLOC_SCRATCH_BYTES - a16(ni * 24)) // per_split


def _call(fn, ctx, ni, sel, eps2, o):
    fn(ctx.ctx, None, ni, sel, eps2, None, o["acc"], o["jerk"], o["snap"], o["pot"], o["nn_id"], o["nn_r2"])
    nbx.nbx_sync(ctx.ctx, None)
    return {k: v.cpu().numpy() for k, v in o.items() if v is not None}


@pytest.mark.parametrize("prec,order,ni_pair", [
    (nbx.NBX_FP64, 4, (131072, 1000)),   # first call: splits lowered to fit; second: same shape
    (nbx.NBX_MIXED, 4, (2000, 300)),     # both shapes fit: bit-identical
    (nbx.NBX_MIXED, 6, (2000, 7)),
])
def test_noalloc_matches_force_dev(prec, order, ni_pair):
    torch = pytest.importorskip("torch")
    n, eps2 = 131072, 1e-6
    say("noalloc prec=%s order=%d ni=%s" % (PREC_NAME[prec], order, ni_pair))
    src = nbody_ics.make_sources(n, seed=2, order=order)
    dev = torch.device("cuda:0")
    with nbx.Context(order=order, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        k_vals = {4: 7, 6: 10}[order]
        for ni in ni_pair:
            sh = ctx.launch_shape(ni)
            fits = sh["splits"] <= 1 or sh["splits"] <= _max_splits(ni, k_vals)
            sel = torch.as_tensor(nbody_ics.active_set(n, ni, seed=1002), dtype=torch.int32, device=dev)
            say("  ni=%d shape=%s fits=%s" % (ni, sh, fits))
            ref = _call(nbx.nbx_force_dev, ctx, ni, sel, eps2, _outs(torch, ni, order, dev, 3.0))
            got = _call(nbx.nbx_force_dev_noalloc, ctx, ni, sel, eps2, _outs(torch, ni, order, dev, 5.0))
            np.testing.assert_array_equal(got["nn_id"], ref["nn_id"])
            if fits:
                for k in ref:
                    np.testing.assert_array_equal(got[k], ref[k], err_msg=k)
            else:
                assert prec == nbx.NBX_FP64
                for k in ("acc", "jerk"):
                    e = np.linalg.norm(got[k] - ref[k], axis=1) / np.linalg.norm(ref[k], axis=1)
                    say("  %s max rel difference %.2e" % (k, e.max()))
                    assert e.max() <= 1e-13, k
                e = np.abs(got["pot"] - ref["pot"]) / np.abs(ref["pot"])
                assert e.max() <= 1e-13
                np.testing.assert_array_equal(got["nn_r2"], ref["nn_r2"])


def test_noalloc_rejects_what_force_dev_rejects():
    torch = pytest.importorskip("torch")
    n = 1024
    src = nbody_ics.make_sources(n, seed=9)
    dev = torch.device("cuda:0")
    with nbx.Context(order=4, precision=nbx.NBX_FP64, nj_max=n, ni_max=512) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        sel = torch.arange(n, dtype=torch.int32, device=dev)
        o = _outs(torch, n, 4, dev, 0.0)
        with pytest.raises(nbx.NbxError) as e:
            nbx.nbx_force_dev_noalloc(ctx.ctx, None, n, sel, 1e-4, None, o["acc"], o["jerk"], None, o["pot"],
                                      o["nn_id"], o["nn_r2"])
        assert e.value.code == nbx.NBX_ERR_CAPACITY
    with nbx.Context(order=8, precision=nbx.NBX_FP64, nj_max=n, ni_max=n) as ctx:
        with pytest.raises(nbx.NbxError) as e:
            nbx.nbx_force_dev_noalloc(ctx.ctx, None, 4, sel, 1e-4, None, o["acc"], o["jerk"], o["snap"],
                                      o["pot"], o["nn_id"], o["nn_r2"])
        assert e.value.code == nbx.NBX_ERR_ARG
