"""Every launch shape computes the same forces: lanes per sink L, sinks per lane P and source
splits S forced through NBX_SHAPE (one workgroup per sink block with no split, two sinks per lane
in FP64, splits that do not divide the tile count, one split per tile), each against the oracle
with the parity bounds, and the FP64 shapes against each other (summation order only)."""

import os

import numpy as np
import pytest

import nbody_ics
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, check_nn, cond_err_vec, oracle_all, rel_err_vec, run_gpu, say, subset

pytestmark = pytest.mark.gpu

TOL = {nbx.NBX_FP64: 1e-13, nbx.NBX_MIXED: 1e-6}
CRACKLE_TOL = {nbx.NBX_FP64: 2e-12, nbx.NBX_MIXED: 2e-5}  # condition-normalised, as in test_gpu_order8
SHAPES = [(1, 1, 1), (1, 2, 1), (1, 2, 5), (2, 1, 3), (4, 1, 12), (16, 1, 7), (64, 1, 13), (256, 1, 12)]


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
@pytest.mark.parametrize("order", [4, 6, 8])
def test_forced_shapes_agree(order, prec, monkeypatch):
    n, ni, eps2 = 3000, 700, 1e-4  # 12 tiles, the last one ragged
    say("shapes order=%d prec=%s n=%d ni=%d seed=80" % (order, PREC_NAME[prec], n, ni))
    src = nbody_ics.make_sources(n, seed=80, order=order)
    sel = nbody_ics.active_set(n, ni, seed=81)
    ref = subset(oracle_all(src, order, eps2, 0.0), sel)
    outs = []
    with nbx.Context(order=order, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        for L, P, S in SHAPES:
            monkeypatch.setenv("NBX_SHAPE", "%d,%d,%d" % (L, P, S))
            sh = ctx.launch_shape(ni)
            assert (sh["lanes_per_sink"], sh["sinks_per_lane"], sh["splits"]) == (L, P, min(S, 12))
            out = run_gpu(ctx, sel, eps2)
            e_acc = rel_err_vec(out["acc"], ref["acc"]).max()
            e_pot = (np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])).max()
            mism = check_nn(out, ref, ref["xp"], sel, prec, src.ids)
            say("  L=%d P=%d S=%d: max rel acc %.2e pot %.2e nn-mismatch %d" % (L, P, S, e_acc, e_pot, mism))
            assert e_acc <= TOL[prec] and e_pot <= TOL[prec]
            if order == 8:
                e_c = cond_err_vec(out["crackle"], ref["crackle"], ref["cond"][:, 3]).max()
                say("    crackle/cond %.2e" % e_c)
                assert e_c <= CRACKLE_TOL[prec]
            if prec == nbx.NBX_FP64:
                assert mism == 0
            outs.append(out)
        monkeypatch.delenv("NBX_SHAPE")
    if prec == nbx.NBX_FP64:
        base = outs[0]
        for out in outs[1:]:
            assert rel_err_vec(out["acc"], base["acc"]).max() <= 2e-14
            assert rel_err_vec(out["jerk"], base["jerk"]).max() <= 1e-12
            np.testing.assert_array_equal(out["nn_id"], base["nn_id"])
            np.testing.assert_array_equal(out["nn_r2"], base["nn_r2"])
    assert "NBX_SHAPE" not in os.environ
