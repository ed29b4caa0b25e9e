"""2nd-order (GRAPE-5 / leapfrog) mode on the GPU against the FP64 oracle.

Acceleration and potential only, from positions and masses (Background: the library supports the
2nd-order leapfrog besides 4th- and 6th-order Hermite).  Bounds as for the 4th-order path: FP64
acc and pot relative error <= 1e-13, mixed <= 1e-6; the nearest neighbour as there.
"""

import numpy as np
import pytest

import nbody_ics
import oracle
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, check_nn, oracle_all, rel_err_vec, run_gpu, say, subset

pytestmark = pytest.mark.gpu

TOL = {nbx.NBX_FP64: 1e-13, nbx.NBX_MIXED: 1e-6}


def _compare2(out, ref, prec, sel_addr, ids, label):
    assert out["jerk"] is None
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
    mism = check_nn(out, ref, ref["xp"], sel_addr, prec, ids)
    msg = "%s: max rel acc %.2e pot %.2e nn-mismatch %d" % (label, e_acc.max(), e_pot.max(), mism)
    say(msg)
    assert e_acc.max() <= TOL[prec], msg
    assert e_pot.max() <= TOL[prec], msg
    if prec == nbx.NBX_FP64:
        assert mism == 0, msg


def test_order2_predictor_matches_oracle():
    n, t = 3000, 0.01
    say("order2 predictor n=%d seed=50" % n)
    src = nbody_ics.make_sources(n, seed=50)
    xp, vp, ap = oracle.predict(2, t, src.t, src.x, src.v, src.a, None)
    with nbx.Context(order=2, nj_max=n, ni_max=16) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        gx, gv, ga = ctx.get_predicted(np.arange(n, dtype=np.int32))
        back = ctx.get_j(np.arange(n, dtype=np.int32))
    np.testing.assert_allclose(gx, xp, rtol=2e-15, atol=1e-15)
    np.testing.assert_allclose(gv, vp, rtol=2e-15, atol=1e-14)
    np.testing.assert_array_equal(ga, src.a)
    np.testing.assert_array_equal(back["jerk"], 0.0)  # the 2nd-order mode stores no jerk


NI_CASES = [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 3000]


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order2_parity_active_sets(prec):
    """Active sets of every size class against a ragged source count, per-source times."""
    n, t, eps2 = 3000, 0.0, 1e-4
    say("order2 parity prec=%s n=%d eps2=%g seed=51" % (PREC_NAME[prec], n, eps2))
    src = nbody_ics.make_sources(n, seed=51, masses="salpeter")
    ref_all = oracle_all(src, 2, eps2, t)
    with nbx.Context(order=2, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        for ni in NI_CASES:
            sel = nbody_ics.active_set(n, ni, seed=1100 + ni)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            out = run_gpu(ctx, sel, eps2)
            _compare2(out, subset(ref_all, sel), prec, sel, src.ids, "  ni=%d" % ni)


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order2_positions_and_masses_only(prec):
    """GRAPE-5 style input: sources without velocities or accelerations (NULL, taken as zero, so
    prediction leaves them in place), eps2 = 0, explicit sinks without velocities (foreign ids and
    ids of sources), neighbour lists."""
    n, eps2, nbr_max = 1500, 0.0, 64
    say("order2 positions+masses prec=%s n=%d" % (PREC_NAME[prec], n))
    m, x, _ = nbody_ics.plummer(n, seed=52)
    ids = np.arange(n, dtype=np.int64) * 3 + 1
    rng = np.random.default_rng(53)
    ni = 400
    own = rng.choice(n, size=ni // 2, replace=False)
    sid = np.concatenate([ids[own], np.arange(10**7, 10**7 + ni - ni // 2)]).astype(np.int64)
    sx = np.concatenate([x[own] + rng.normal(0, 1e-3, (ni // 2, 3)), rng.normal(0, 0.5, (ni - ni // 2, 3))])
    h2 = np.full(ni, 5e-3)
    ref = oracle.force(2, eps2, ids, m, x, None, sid, sx, None, h2=h2, nbr_max=n)
    with nbx.Context(order=2, precision=prec, nj_max=n, ni_max=n, nbr_max=nbr_max) as ctx:
        nbx.nbx_set_j(ctx.ctx, np.arange(n, dtype=np.int32), ids, m, np.zeros(n), x, None, None, None)
        ctx.predict(0.25)  # no velocity, no acceleration: the sources stay put
        gx, gv, _ = ctx.get_predicted(np.arange(n, dtype=np.int32))
        np.testing.assert_array_equal(gx, x)
        np.testing.assert_array_equal(gv, 0.0)
        ctx.force_ext(sid, sx, None, None, eps2, h2)
        out = ctx.get_force()
        cnt, nb, _ = ctx.get_nbr()
        # every source as a by-address sink
        allx = run_gpu(ctx, np.arange(n, dtype=np.int32), eps2)
    assert out["jerk"] is None
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
    say("  ext: max rel acc %.2e pot %.2e" % (e_acc.max(), e_pot.max()))
    assert e_acc.max() <= TOL[prec] and e_pot.max() <= TOL[prec]
    assert not np.any(out["nn_id"] == sid)
    d = x[(out["nn_id"] - 1) // 3] - sx
    np.testing.assert_allclose(out["nn_r2"], np.sum(d * d, axis=1), rtol=1e-13)
    if prec == nbx.NBX_FP64:
        np.testing.assert_array_equal(out["nn_id"], ref["nn_id"])
        np.testing.assert_array_equal(cnt, ref["nbr_count"])
        for i in range(ni):
            assert set(nb[i, : min(cnt[i], nbr_max)]) <= set(ref["nbr_ids"][i, : ref["nbr_count"][i]])
    ref_all = oracle.force(2, eps2, ids, m, x, None, ids, x, None)
    ref_all["xp"] = x
    _compare2(allx, ref_all, prec, np.arange(n), ids, "  all by address")


def test_order2_leapfrog_sixteen_steps():
    """Sixteen kick-drift-kick leapfrog steps (dt = 1/256) of the 1024-body Plummer sphere driven
    by the GPU's 2nd-order forces (FP64) and by the oracle's agree to 1e-12."""
    n, eps2, dt = 1024, 1e-4, 1.0 / 256
    say("order2 leapfrog 16 steps")
    src = nbody_ics.make_sources(n, seed=1, time_offsets=False)
    ids, addr = src.ids, np.arange(n, dtype=np.int32)

    def run(force):
        x, v = src.x.copy(), src.v.copy()
        a = force(x)
        for _ in range(16):
            v = v + 0.5 * dt * a
            x = x + dt * v
            a = force(x)
            v = v + 0.5 * dt * a
        return x, v

    with nbx.Context(order=2, nj_max=n, ni_max=n) as ctx:
        def gpu_force(x):
            nbx.nbx_set_j(ctx.ctx, addr, ids, src.m, np.zeros(n), x, None, None, None)
            ctx.predict(0.0)
            return run_gpu(ctx, addr, eps2)["acc"]
        xg, vg = run(gpu_force)
    xo, vo = run(lambda x: oracle.force(2, eps2, ids, src.m, x, None, ids, x, None)["acc"])
    ex = np.abs(xg - xo).max() / np.abs(xo).max()
    ev = np.abs(vg - vo).max() / np.abs(vo).max()
    say("leapfrog: max rel dx %.2e dv %.2e" % (ex, ev))
    assert ex <= 1e-12 and ev <= 1e-12


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order2_full_size_sampled(prec):
    """N = 131072 Plummer, eps2 = 1e-6, per-source times, in the launch shapes of N_i = 1, 4096
    and N; 256 sampled sinks per case against the oracle."""
    n, eps2, t = 131072, 1e-6, 0.0
    say("order2 full size prec=%s n=%d" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=2)
    rng = np.random.default_rng(79)
    with nbx.Context(order=2, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        for ni in (1, 4096, n):
            sel = nbody_ics.active_set(n, ni, seed=1002)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            out = run_gpu(ctx, sel, eps2)
            pick = np.sort(rng.choice(ni, size=min(ni, 256), replace=False))
            ref = oracle_all(src, 2, eps2, t, addr=sel[pick])
            got = {k: (v[pick] if v is not None else None) for k, v in out.items() if k != "status"}
            _compare2(got, ref, prec, sel[pick], src.ids, "  ni=%d" % ni)
