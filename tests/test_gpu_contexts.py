"""Two contexts on one device, driven through the device path on two different torch streams with
their calls interleaved: each produces exactly (bitwise) what it produces alone, so contexts share
no state and the enqueue-only entry points honour the caller's stream."""

import numpy as np
import pytest

import nbody_ics
import paper_1510_04068_amd as nbx
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _load(ctx, src, T, torch, stream):
    n = src.n
    nbx.nbx_set_j_dev(ctx.ctx, stream, n, T(np.arange(n), torch.int32), T(src.ids, torch.int64), T(src.m), T(src.t),
                      T(src.x), T(src.v), T(src.a), T(src.jerk))
    nbx.nbx_set_nj(ctx.ctx, n)
    nbx.nbx_predict(ctx.ctx, 0.0)


def _force(ctx, stream, sel, eps2, out):
    nbx.nbx_force_dev(ctx.ctx, stream, len(sel), sel, eps2, None, out["acc"], out["jerk"], None, out["pot"],
                      out["nn_id"], out["nn_r2"])


def test_two_contexts_two_streams():
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    say("two contexts")
    srcs = [nbody_ics.make_sources(4000, seed=90), nbody_ics.make_sources(2500, seed=91)]
    sels = [T(nbody_ics.active_set(4000, 1500, seed=92), torch.int32), T(nbody_ics.active_set(2500, 700, seed=93),
                                                                         torch.int32)]
    precs = [nbx.NBX_MIXED, nbx.NBX_FP64]

    def outputs(ni):
        return {"acc": torch.empty((ni, 3), dtype=torch.float64, device=dev),
                "jerk": torch.empty((ni, 3), dtype=torch.float64, device=dev),
                "pot": torch.empty(ni, dtype=torch.float64, device=dev),
                "nn_id": torch.empty(ni, dtype=torch.int64, device=dev),
                "nn_r2": torch.empty(ni, dtype=torch.float64, device=dev)}

    # each context alone, on the current stream
    alone = []
    for src, sel, prec in zip(srcs, sels, precs):
        with nbx.Context(order=4, precision=prec, nj_max=src.n, ni_max=src.n) as ctx:
            cur = torch.cuda.current_stream()
            _load(ctx, src, T, torch, cur)
            out = outputs(len(sel))
            _force(ctx, cur, sel, 1e-4, out)
            nbx.nbx_sync(ctx.ctx, cur)
            alone.append({k: v.cpu().numpy() for k, v in out.items()})
    # both contexts at once, interleaved on two streams
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    ctxs = [nbx.Context(order=4, precision=p, nj_max=s.n, ni_max=s.n) for s, p in zip(srcs, precs)]
    try:
        for ctx, src, st in zip(ctxs, srcs, streams):
            _load(ctx, src, T, torch, st)
        outs = [outputs(len(s)) for s in sels]
        for rep in range(3):
            for ctx, sel, st, out in zip(ctxs, sels, streams, outs):
                _force(ctx, st, sel, 1e-4, out)
        for ctx, st in zip(ctxs, streams):
            nbx.nbx_sync(ctx.ctx, st)
        torch.cuda.synchronize()
        for a, out in zip(alone, outs):
            for k in a:
                np.testing.assert_array_equal(out[k].cpu().numpy(), a[k])
    finally:
        for ctx in ctxs:
            ctx.close()
