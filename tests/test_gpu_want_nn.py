"""Contexts opened with want_nn = 0 run the gravity kernels without the nearest-neighbour search
(the paper makes it a compile-time option of its kernel, Results).  Their acc, jerk, snap, crackle,
pot and neighbour lists must be bit-identical to those of the kernels with the search (the pair
arithmetic and every summation order are the same), and the nearest-neighbour outputs must be
left untouched, on the host path and on the device path, for every launch-shape class."""

import numpy as np
import pytest

import nbody_ics
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, say

pytestmark = pytest.mark.gpu

NI_CASES = [1, 3, 64, 257, 1000, 3000]  # several lanes per sink, one lane, splits and none


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_nn_free_outputs_bit_identical(order, prec):
    n, t, eps2 = 3000, 0.0, 1e-5
    say("want_nn order=%d prec=%s n=%d seed=31" % (order, PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=31, order=order, masses="salpeter")
    ctxs = [nbx.Context(order=order, precision=prec, nj_max=n, ni_max=n, want_nn=w) for w in (True, False)]
    try:
        for c in ctxs:
            c.set_sources(src)
            c.predict(t)
        for ni in NI_CASES:
            sel = nbody_ics.active_set(n, ni, seed=2000 + ni)
            say("  ni=%d shape=%s" % (ni, ctxs[0].launch_shape(ni)))
            outs = []
            for c in ctxs:
                c.force(sel, eps2)
                outs.append(c.get_force())
            with_nn, without = outs
            assert without["nn_id"] is None and without["nn_r2"] is None
            for k in ("acc", "jerk", "snap", "crackle", "pot"):
                if with_nn.get(k) is not None:
                    np.testing.assert_array_equal(with_nn[k], without[k], err_msg="%s ni=%d" % (k, ni))
    finally:
        for c in ctxs:
            c.close()


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_nn_free_device_path_leaves_nn_untouched(prec):
    """Device path, order 6 with neighbour lists: NULL nearest-neighbour pointers are accepted, given
    ones are never written, and the lists and sums equal the search kernels' bit for bit."""
    import torch

    n, eps2, h2, nbr_max = 3000, 1e-6, 4e-3, 64
    say("want_nn device prec=%s n=%d seed=32" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=32, order=6, masses="salpeter")
    dev = torch.device("cuda:0")
    T = lambda a, dt: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    f64, i64, i32 = torch.float64, torch.int64, torch.int32
    res = []
    for want in (True, False):
        with nbx.Context(order=6, precision=prec, nj_max=n, ni_max=n, nbr_max=nbr_max, want_nn=want) as c:
            c.set_sources(src)
            c.predict(0.0)
            for ni in (5, 700, n):
                sel = T(nbody_ics.active_set(n, ni, seed=3000 + ni), i32)
                o = [torch.full((ni, 3), 7.0, dtype=f64, device=dev) for _ in range(3)]
                pot = torch.full((ni,), 7.0, dtype=f64, device=dev)
                nnid = torch.full((ni,), 12345, dtype=i64, device=dev)
                nnr2 = torch.full((ni,), 7.0, dtype=f64, device=dev)
                cnt = torch.zeros(ni, dtype=i32, device=dev)
                ids = torch.full((ni, nbr_max), -1, dtype=i64, device=dev)
                d_h2 = torch.full((ni,), h2, dtype=f64, device=dev)
                nbx.nbx_force_dev(c.ctx, None, ni, sel, eps2, d_h2, o[0], o[1], o[2], pot, nnid, nnr2, cnt, ids)
                if not want:  # NULL nearest-neighbour outputs are accepted without the search
                    nbx.nbx_force_dev(c.ctx, None, ni, sel, eps2, d_h2, o[0], o[1], o[2], pot, None, None, cnt,
                                      ids)
                nbx.nbx_sync(c.ctx)
                idh = ids.cpu().numpy()
                idh.sort(axis=1)
                res.append(dict(ni=ni, acc=o[0].cpu().numpy(), jerk=o[1].cpu().numpy(), snap=o[2].cpu().numpy(),
                                pot=pot.cpu().numpy(), nnid=nnid.cpu().numpy(), nnr2=nnr2.cpu().numpy(),
                                cnt=cnt.cpu().numpy(), ids=idh))
    half = len(res) // 2
    for a, b in zip(res[:half], res[half:]):
        say("  ni=%d" % a["ni"])
        for k in ("acc", "jerk", "snap", "pot", "cnt", "ids"):
            np.testing.assert_array_equal(a[k], b[k], err_msg="%s ni=%d" % (k, a["ni"]))
        assert np.all(b["nnid"] == 12345) and np.all(b["nnr2"] == 7.0)
        assert np.all(a["nnid"] != 12345)
