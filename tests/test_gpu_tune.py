"""Launch-shape tuner: the shapes it picks are valid, are the ones later force calls use, and keep
parity with the oracle (same bounds as the untuned path) and run-to-run bit reproducibility."""

import numpy as np
import pytest

import nbody_ics
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, check_nn, oracle_all, rel_err_vec, run_gpu, say, subset

pytestmark = pytest.mark.gpu

TOL = {nbx.NBX_FP64: 1e-13, nbx.NBX_MIXED: 1e-6}


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_tuned_shapes_keep_parity(prec):
    n, eps2 = 3000, 1e-4
    say("tune prec=%s n=%d seed=70" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=70)
    ref_all = oracle_all(src, 4, eps2, 0.0)
    ntiles = (n + 255) // 256
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        tab = ctx.tune(n)
        say("  table (L, P, S) per class: %s" % tab.tolist())
        assert tab.shape == (int(np.ceil(np.log2(n))) + 1, 3)  # classes 2^0 .. 2^12 >= n
        for L, P, S in tab:
            assert L >= 1 and L <= 256 and (L & (L - 1)) == 0
            assert P in (1, 2) and (P == 1 or L == 1)
            assert 1 <= S <= ntiles
        for ni in (1, 5, 64, 300, 1000, 3000):
            k = int(np.ceil(np.log2(ni))) if ni > 1 else 0
            sh = ctx.launch_shape(ni)
            assert (sh["lanes_per_sink"], sh["sinks_per_lane"]) == (tab[k][0], tab[k][1])
            assert sh["splits"] == min(tab[k][2], ntiles, (1 << 21) // ni)
            sel = nbody_ics.active_set(n, ni, seed=1200 + ni)
            out = run_gpu(ctx, sel, eps2)
            ref = subset(ref_all, sel)
            e_acc = rel_err_vec(out["acc"], ref["acc"])
            e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
            mism = check_nn(out, ref, ref["xp"], sel, prec, src.ids)
            say("  ni=%d shape=%s max rel acc %.2e pot %.2e nn-mismatch %d" % (ni, sh, e_acc.max(), e_pot.max(), mism))
            assert e_acc.max() <= TOL[prec] and e_pot.max() <= TOL[prec]
            if prec == nbx.NBX_FP64:
                assert mism == 0
            again = run_gpu(ctx, sel, eps2)
            for key in ("acc", "jerk", "pot", "nn_id", "nn_r2"):
                np.testing.assert_array_equal(out[key], again[key])


def test_tune_needs_predict_and_reports_errors():
    say("tune error paths")
    src = nbody_ics.make_sources(300, seed=71)
    with nbx.Context(order=4, nj_max=300, ni_max=300) as ctx:
        ctx.set_sources(src)
        with pytest.raises(nbx.NbxError) as e:
            ctx.tune(300)
        assert e.value.code == nbx.NBX_ERR_STATE
        ctx.predict(0.0)
        assert nbx.load().nbx_tune(ctx.ctx, 0, None, 0) == nbx.NBX_ERR_ARG
