"""Parity of the HIP force path with the FP64 oracle, element by element, on seeded inputs.

Bounds (per sink, max over sinks): FP64 acc and pot relative error <= 1e-13; mixed acc and pot
<= 1e-6.  Jerk and snap have no stated bound; they are checked against looser, condition-
normalised bounds derived from the arithmetic (FP32 velocities in mixed mode).
"""

import numpy as np
import pytest

import nbody_ics
import oracle
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, check_nn, cond_err_vec, oracle_all, rel_err_vec, run_gpu, say, subset

pytestmark = pytest.mark.gpu

TOL = {
    nbx.NBX_FP64: dict(acc=1e-13, pot=1e-13, jerk_cond=1e-13, snap_cond=1e-12),
    nbx.NBX_MIXED: dict(acc=1e-6, pot=1e-6, jerk_cond=2e-6, snap_cond=1e-5),
}


def _compare(out, ref, prec, order, sel_addr, ids, label):
    tol = TOL[prec]
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
    e_jc = cond_err_vec(out["jerk"], ref["jerk"], ref["cond"][:, 1])
    msg = "%s: max rel acc %.2e pot %.2e jerk/cond %.2e" % (label, e_acc.max(), e_pot.max(), e_jc.max())
    if order == 6:
        e_sc = cond_err_vec(out["snap"], ref["snap"], ref["cond"][:, 2])
        msg += " snap/cond %.2e" % e_sc.max()
        assert e_sc.max() <= tol["snap_cond"], msg
    mism = check_nn(out, ref, ref["xp"], sel_addr, prec, ids)
    say(msg + " nn-mismatch %d" % mism)
    assert e_acc.max() <= tol["acc"], msg
    assert e_pot.max() <= tol["pot"], msg
    assert e_jc.max() <= tol["jerk_cond"], msg
    if prec == nbx.NBX_FP64:
        assert mism == 0


@pytest.mark.parametrize("order", [4, 6])
def test_predictor_matches_oracle(order):
    n, t = 3000, 0.01
    say("predictor order=%d n=%d seed=21" % (order, n))
    src = nbody_ics.make_sources(n, seed=21, order=order)
    xp, vp, ap = oracle.predict(order, t, src.t, src.x, src.v, src.a, src.jerk, src.snap, src.crackle)
    with nbx.Context(order=order, nj_max=n, ni_max=16) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        gx, gv, ga = ctx.get_predicted(np.arange(n, dtype=np.int32))
    np.testing.assert_allclose(gx, xp, rtol=2e-15, atol=1e-15)
    np.testing.assert_allclose(gv, vp, rtol=2e-15, atol=1e-14)
    if order == 6:
        np.testing.assert_allclose(ga, ap, rtol=2e-15, atol=1e-13)


NI_CASES = [1, 2, 3, 63, 64, 65, 255, 256, 257, 1000, 3000]


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
@pytest.mark.parametrize("order", [4, 6])
def test_force_parity_active_sets(order, prec):
    """Active sets of every size class (lanes/wave/split edges) against a ragged source count."""
    n, t = 3000, 0.0
    eps2 = 1e-4 if order == 4 else 1e-6
    masses = "equal" if order == 4 else "salpeter"
    say("parity order=%d prec=%s n=%d eps2=%g seed=22" % (order, PREC_NAME[prec], n, eps2))
    src = nbody_ics.make_sources(n, seed=22, order=order, masses=masses)
    ref_all = oracle_all(src, order, eps2, t)
    with nbx.Context(order=order, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        for ni in NI_CASES:
            sel = nbody_ics.active_set(n, ni, seed=1000 + ni)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            out = run_gpu(ctx, sel, eps2)
            _compare(out, subset(ref_all, sel), prec, order, sel, src.ids, "  ni=%d" % ni)


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_config1_shared_step(prec):
    """1024-body equal-mass Plummer sphere, eps2 = 1e-4, t_j = 0, every sink active."""
    n, eps2 = 1024, 1e-4
    say("config1 prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=1, time_offsets=False)
    ref = oracle_all(src, 4, eps2, 0.0)
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        sel = np.arange(n, dtype=np.int32)
        out = run_gpu(ctx, sel, eps2)
        _compare(out, ref, prec, 4, sel, src.ids, "config1")
        again = run_gpu(ctx, sel, eps2)
        for k in ("acc", "jerk", "pot", "nn_id", "nn_r2"):
            np.testing.assert_array_equal(out[k], again[k])  # run-to-run determinism


def test_config1_hermite_eight_steps():
    """Eight shared 4th-order Hermite steps (dt = 1/256) driven through the GPU (FP64) and through
    the oracle agree to 1e-12 in positions and velocities."""
    n, eps2, dt = 1024, 1e-4, 1.0 / 256
    say("config1 hermite 8 steps")
    src = nbody_ics.make_sources(n, seed=1, time_offsets=False)
    ids = src.ids
    zeros = np.zeros((n, 3))
    addr = np.arange(n, dtype=np.int32)

    def corrector(dt, xp, vp, a0, j0, a1, j1):  # the GPU side's own copy of the Hermite corrector
        d2 = (-6.0 * (a0 - a1) - dt * (4.0 * j0 + 2.0 * j1)) / (dt * dt)
        d3 = (12.0 * (a0 - a1) + 6.0 * dt * (j0 + j1)) / (dt * dt * dt)
        return (xp + d2 * dt**4 / 24.0 + d3 * dt**5 / 120.0, vp + d2 * dt**3 / 6.0 + d3 * dt**4 / 24.0)

    # GPU-driven
    with nbx.Context(order=4, nj_max=n, ni_max=n) as ctx:
        x, v = src.x.copy(), src.v.copy()
        nbx.nbx_set_j(ctx.ctx, addr, ids, src.m, np.zeros(n), x, v, zeros, zeros)
        ctx.predict(0.0)
        f = run_gpu(ctx, addr, eps2)
        a0, j0 = f["acc"], f["jerk"]
        t = 0.0
        for _ in range(8):
            nbx.nbx_set_j(ctx.ctx, addr, ids, src.m, np.full(n, t), x, v, a0, j0)
            ctx.predict(t + dt)
            xp, vp, _ = ctx.get_predicted(addr)
            f = run_gpu(ctx, addr, eps2)
            x, v = corrector(dt, xp, vp, a0, j0, f["acc"], f["jerk"])
            t += dt
            nbx.nbx_set_j(ctx.ctx, addr, ids, src.m, np.full(n, t), x, v, zeros, zeros)
            ctx.predict(t)
            f = run_gpu(ctx, addr, eps2)
            a0, j0 = f["acc"], f["jerk"]
        xg, vg = x, v
    # oracle-driven
    x, v = src.x.copy(), src.v.copy()
    f = oracle.force(4, eps2, ids, src.m, x, v, ids, x, v)
    a0, j0 = f["acc"], f["jerk"]
    t = 0.0
    for _ in range(8):
        xp, vp, _ = oracle.predict(4, t + dt, np.full(n, t), x, v, a0, j0)
        f = oracle.force(4, eps2, ids, src.m, xp, vp, ids, xp, vp)
        x, v = oracle.hermite4_correct(dt, xp, vp, a0, j0, f["acc"], f["jerk"])
        t += dt
        f = oracle.force(4, eps2, ids, src.m, x, v, ids, x, v)
        a0, j0 = f["acc"], f["jerk"]
    ex = np.abs(xg - x).max() / np.abs(x).max()
    ev = np.abs(vg - v).max() / np.abs(v).max()
    say("hermite: max rel dx %.2e dv %.2e" % (ex, ev))
    assert ex <= 1e-12 and ev <= 1e-12


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_edge_cases(prec):
    say("edge cases prec=%s" % PREC_NAME[prec])
    # one source, the sink is itself: no force, no potential, no neighbour
    one = nbody_ics.make_sources(1, seed=30)
    with nbx.Context(order=4, precision=prec, nj_max=4, ni_max=4) as ctx:
        ctx.set_sources(one)
        ctx.predict(0.0)
        out = run_gpu(ctx, [0], 1e-4)
        assert np.all(out["acc"] == 0) and np.all(out["jerk"] == 0) and out["pot"][0] == 0
        assert out["nn_id"][0] == -1 and np.isinf(out["nn_r2"][0])
        # zero sinks is a no-op
        out0 = run_gpu(ctx, np.zeros(0, dtype=np.int32), 1e-4)
        assert out0["acc"].shape == (0, 3)
    # eps2 = 0 (guarded self term), ragged n
    n = 500
    src = nbody_ics.make_sources(n, seed=31)
    ref = oracle_all(src, 4, 0.0, 0.0)
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        sel = np.arange(n, dtype=np.int32)
        out = run_gpu(ctx, sel, 0.0)
        _compare(out, ref, prec, 4, sel, src.ids, "eps2=0")


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_coincident_distinct_sources(prec):
    """Two distinct sources at the same position: each is the other's nearest neighbour with
    r2 = 0 (only the sink's own source is excluded), as in the oracle; eps2 > 0 keeps the forces
    finite.  Placed in different tiles and in the same tile."""
    n, eps2 = 700, 1e-4
    say("coincident sources prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=35)
    for k in (18, 600):  # 18: same tile as 17; 600: another tile.  Same orbit, so same predicted position
        src.x[k], src.v[k], src.a[k], src.jerk[k], src.t[k] = src.x[17], src.v[17], src.a[17], src.jerk[17], src.t[17]
    sel = np.array([17, 18, 600, 5], dtype=np.int32)
    ref = oracle_all(src, 4, eps2, 0.0, addr=sel)
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        out = run_gpu(ctx, sel, eps2)
    for k in range(3):
        assert out["nn_r2"][k] == 0.0 and ref["nn_r2"][k] == 0.0
        assert out["nn_id"][k] in (17, 18, 600) and out["nn_id"][k] != sel[k]
    if prec == nbx.NBX_FP64:
        np.testing.assert_array_equal(out["nn_id"], ref["nn_id"])
    e = rel_err_vec(out["acc"], ref["acc"])
    assert e.max() <= (1e-13 if prec == nbx.NBX_FP64 else 1e-6), e


def test_error_paths():
    say("error paths")
    n = 300
    src = nbody_ics.make_sources(n, seed=32)
    with nbx.Context(order=4, nj_max=n, ni_max=100) as ctx:
        ctx.set_sources(src)
        with pytest.raises(nbx.NbxError) as e:
            ctx.force(np.arange(10, dtype=np.int32), 1e-4)
        assert e.value.code == nbx.NBX_ERR_STATE  # force before predict
        ctx.predict(0.0)
        with pytest.raises(nbx.NbxError) as e:
            ctx.force(np.array([0, n], dtype=np.int32), 1e-4)
        assert e.value.code == nbx.NBX_ERR_ARG
        with pytest.raises(nbx.NbxError) as e:
            ctx.force(np.arange(101, dtype=np.int32), 1e-4)
        assert e.value.code == nbx.NBX_ERR_CAPACITY
        with pytest.raises(nbx.NbxError) as e:
            ctx.force(np.arange(10, dtype=np.int32), -1.0)
        assert e.value.code == nbx.NBX_ERR_ARG
        with pytest.raises(nbx.NbxError) as e:
            nbx.nbx_set_j(ctx.ctx, [n], [0], [1.0], [0.0], np.zeros((1, 3)), np.zeros((1, 3)), np.zeros((1, 3)),
                          np.zeros((1, 3)))
        assert e.value.code == nbx.NBX_ERR_ARG
        # stored state reads back exactly (checkpoint)
        back = ctx.get_j(np.arange(n, dtype=np.int32))
        np.testing.assert_array_equal(back["x"], src.x)
        np.testing.assert_array_equal(back["jerk"], src.jerk)
        np.testing.assert_array_equal(back["id"], src.ids)
        # the number of sources in use: [0, nj_max], else a capacity error
        for bad in (-1, n + 1):
            with pytest.raises(nbx.NbxError) as e:
                ctx.set_nj(bad)
            assert e.value.code == nbx.NBX_ERR_CAPACITY
    # no sources in use: every force form refuses sinks with a state error, zero sinks stay a no-op
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    with nbx.Context(order=4, nj_max=n, ni_max=100) as ctx:
        ctx.predict(0.0)
        sinks = nbody_ics.make_sources(4, seed=33)
        with pytest.raises(nbx.NbxError) as e:
            ctx.force(np.arange(4, dtype=np.int32), 1e-4)
        assert e.value.code == nbx.NBX_ERR_STATE
        with pytest.raises(nbx.NbxError) as e:
            ctx.force_ext(sinks.ids, sinks.x, sinks.v, None, 1e-4)
        assert e.value.code == nbx.NBX_ERR_STATE
        f64 = dict(dtype=torch.float64, device=dev)
        outs = (torch.empty((4, 3), **f64), torch.empty((4, 3), **f64), None, torch.empty(4, **f64),
                torch.empty(4, dtype=torch.int64, device=dev), torch.empty(4, **f64))
        d_addr = torch.zeros(4, dtype=torch.int32, device=dev)
        with pytest.raises(nbx.NbxError) as e:
            nbx.nbx_force_dev(ctx.ctx, None, 4, d_addr, 1e-4, None, *outs)
        assert e.value.code == nbx.NBX_ERR_STATE
        ctx.force(np.zeros(0, dtype=np.int32), 1e-4)
        ctx.force_ext(sinks.ids[:0], sinks.x[:0], sinks.v[:0], None, 1e-4)
        # sources loaded afterwards: the same context computes again
        ctx.set_sources(src)
        ctx.predict(0.0)
        sel = np.arange(0, n, 7, dtype=np.int32)[:100]
        out = run_gpu(ctx, sel, 1e-4)
        ref = oracle_all(src, 4, 1e-4, 0.0, addr=sel)
        assert rel_err_vec(out["acc"], ref["acc"]).max() <= 1e-13


def test_device_path_matches_host_path():
    torch = pytest.importorskip("torch")
    n, eps2 = 2000, 1e-4
    say("device path n=%d" % n)
    src = nbody_ics.make_sources(n, seed=33)
    sel = nbody_ics.active_set(n, 700, seed=34)
    dev = torch.device("cuda:0")
    with nbx.Context(order=4, precision=nbx.NBX_MIXED, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        host = run_gpu(ctx, sel, eps2)
        # reload the sources through the device path and compute into torch tensors
        T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
        d_addr = T(np.arange(n), torch.int32)
        nbx.nbx_set_j_dev(ctx.ctx, None, n, d_addr, T(src.ids, torch.int64), T(src.m), T(src.t), T(src.x), T(src.v),
                          T(src.a), T(src.jerk))
        nbx.nbx_set_nj(ctx.ctx, n)
        ni = len(sel)
        acc = torch.empty((ni, 3), dtype=torch.float64, device=dev)
        jrk = torch.empty_like(acc)
        pot = torch.empty(ni, dtype=torch.float64, device=dev)
        nnid = torch.empty(ni, dtype=torch.int64, device=dev)
        nnr2 = torch.empty(ni, dtype=torch.float64, device=dev)
        nbx.nbx_force_dev(ctx.ctx, None, ni, T(sel, torch.int32), eps2, None, acc, jrk, None, pot, nnid, nnr2)
        nbx.nbx_sync(ctx.ctx, None)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(acc.cpu().numpy(), host["acc"])
        np.testing.assert_array_equal(jrk.cpu().numpy(), host["jerk"])
        np.testing.assert_array_equal(pot.cpu().numpy(), host["pot"])
        np.testing.assert_array_equal(nnid.cpu().numpy(), host["nn_id"])


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_full_size_sampled(prec):
    """The headline workload at full size (N = 131072 Plummer, eps2 = 1e-6, per-source times) in the
    launch shapes the benchmark times: every sink active (16384 seeded sinks checked) and small
    active sets (checked in full).

    End to end, each side predicts the sources with its own FP64 predictor (pinned to each other at
    2e-15 relative); a close pair (|x| / |r| ~ 1e3) amplifies their last-bit differences in the
    pair's acceleration, so the FP64 bound here is 1e-12 (a +-1 ulp perturbation of the oracle's own
    predicted positions moves its acc by up to 1e-13 on this workload); test_full_size_same_state
    holds the force arithmetic to 1e-13 on identical inputs.  Mixed: FP32 pair terms carry ~u =
    6e-8 from each rounding and up to 3.6e-7 from R^-3 (v_rsq_f32 is good to 1 ulp, cubed), so
    where the acceleration cancels (kappa = sum_j |a_ij| / |a| large) the plain relative error
    grows with kappa: 1e-6 where kappa <= 5, and the condition-normalised error
    |da| / sum_j |a_ij| <= 5e-7 everywhere."""
    n, eps2, t = 131072, 1e-6, 0.0
    say("full size prec=%s n=%d" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=2)
    rng = np.random.default_rng(77)
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        for ni in (1, 64, 4096, n):
            sel = nbody_ics.active_set(n, ni, seed=1002)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            out = run_gpu(ctx, sel, eps2)
            pick = np.sort(rng.choice(ni, size=min(ni, 16384), replace=False))
            ref = oracle_all(src, 4, eps2, t, addr=sel[pick])
            got = {k: (v[pick] if v is not None else None) for k, v in out.items() if k != "status"}
            e_acc = rel_err_vec(got["acc"], ref["acc"])
            kappa = ref["cond"][:, 0] / np.linalg.norm(ref["acc"], axis=1)
            e_pot = np.abs(got["pot"] - ref["pot"]) / np.abs(ref["pot"])
            e_jc = cond_err_vec(got["jerk"], ref["jerk"], ref["cond"][:, 1])
            w = int(np.argmax(e_acc))
            say("  ni=%d sinks=%d max rel acc %.2e (kappa %.1f there) acc/cond %.2e pot %.2e jerk/cond %.2e" % (
                ni, len(pick), e_acc.max(), kappa[w], (e_acc / kappa).max(), e_pot.max(), e_jc.max()))
            mism = check_nn(got, ref, ref["xp"], sel[pick], prec, src.ids)
            if prec == nbx.NBX_FP64:
                assert e_acc.max() <= 1e-12 and e_pot.max() <= 1e-13 and e_jc.max() <= 1e-12
                assert mism == 0
            else:
                assert (e_acc / kappa).max() <= 5e-7
                assert e_acc[kappa <= 5].max() <= 1e-6 and e_pot.max() <= 1e-6 and e_jc.max() <= 2e-6


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_full_size_same_state(prec):
    """The headline sources with every t_j = 0, predicted to t = 0: the predictor is the identity on
    both sides, so GPU and oracle see bit-identical inputs and the force arithmetic alone is held to
    the bounds, 1e-13 (FP64) and 1e-6 (mixed, where kappa <= 5; condition-normalised 5e-7
    everywhere, as in test_full_size_sampled), on 16384 seeded sinks of the N_i = N launch."""
    n, eps2 = 131072, 1e-6
    say("full size same state prec=%s n=%d" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=2, time_offsets=False)
    assert np.all(src.t == 0.0)
    sel = np.arange(n, dtype=np.int32)
    pick = np.sort(np.random.default_rng(78).choice(n, size=16384, replace=False))
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        say("  ni=%d shape=%s" % (n, ctx.launch_shape(n)))
        out = run_gpu(ctx, sel, eps2)
    ref = oracle.force(4, eps2, src.ids, src.m, src.x, src.v, src.ids[pick], src.x[pick], src.v[pick])
    e_acc = rel_err_vec(out["acc"][pick], ref["acc"])
    kappa = ref["cond"][:, 0] / np.linalg.norm(ref["acc"], axis=1)
    e_pot = np.abs(out["pot"][pick] - ref["pot"]) / np.abs(ref["pot"])
    e_jc = cond_err_vec(out["jerk"][pick], ref["jerk"], ref["cond"][:, 1])
    w = int(np.argmax(e_acc))
    say("  max rel acc %.2e (kappa %.1f there) acc/cond %.2e pot %.2e jerk/cond %.2e" % (
        e_acc.max(), kappa[w], (e_acc / kappa).max(), e_pot.max(), e_jc.max()))
    if prec == nbx.NBX_FP64:
        assert e_acc.max() <= 1e-13 and e_pot.max() <= 1e-13 and e_jc.max() <= 1e-13
        np.testing.assert_array_equal(out["nn_id"][pick], ref["nn_id"])
    else:
        assert (e_acc / kappa).max() <= 5e-7
        assert e_acc[kappa <= 5].max() <= 1e-6 and e_pot.max() <= 1e-6 and e_jc.max() <= 2e-6


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_large_n_same_state(prec):
    """Past the headline sizes: N = 2^22 + 77 Plummer sources (a ragged last tile), every t_j = 0
    and predicted to t = 0 (identical inputs on both sides), eps2 = 1e-6; 3000 sinks (split sources)
    and 2^21 + 5 sinks, above the 2^21 cap on sinks x splits of partials, so one split takes every
    source and writes the outputs itself.  128 seeded sinks of each launch against the oracle.
    FP64: each pair term carries a few ulps and a 64-term chunk adds at most 63 u in plain FP64 before
    its compensated fold, so |da| / sum_j |a_ij| <= ~70 u = 7.8e-15 (bound 1e-14), and the plain
    relative bound 1e-13 holds where kappa <= 10; mixed: the bounds of test_full_size_sampled."""
    n, eps2, big = (1 << 22) + 77, 1e-6, (1 << 21) + 5
    say("large n same state prec=%s n=%d" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=3, time_offsets=False)
    assert np.all(src.t == 0.0)
    rng = np.random.default_rng(79)
    with nbx.Context(order=4, precision=prec, nj_max=n, ni_max=big) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        for ni in (3000, big):
            sel = nbody_ics.active_set(n, ni, seed=1003)
            shape = ctx.launch_shape(ni)
            say("  ni=%d shape=%s" % (ni, shape))
            assert (shape["splits"] == 1) == (ni == big)
            out = run_gpu(ctx, sel, eps2)
            pick = np.sort(rng.choice(ni, size=128, replace=False))
            a = sel[pick]
            ref = oracle.force(4, eps2, src.ids, src.m, src.x, src.v, src.ids[a], src.x[a], src.v[a])
            e_acc = rel_err_vec(out["acc"][pick], ref["acc"])
            kappa = ref["cond"][:, 0] / np.linalg.norm(ref["acc"], axis=1)
            e_pot = np.abs(out["pot"][pick] - ref["pot"]) / np.abs(ref["pot"])
            e_jc = cond_err_vec(out["jerk"][pick], ref["jerk"], ref["cond"][:, 1])
            w = int(np.argmax(e_acc))
            say("  ni=%d max rel acc %.2e (kappa %.1f there) acc/cond %.2e pot %.2e jerk/cond %.2e" % (
                ni, e_acc.max(), kappa[w], (e_acc / kappa).max(), e_pot.max(), e_jc.max()))
            got = {k: (v[pick] if v is not None else None) for k, v in out.items() if k != "status"}
            mism = check_nn(got, ref, src.x, a, prec, src.ids, eps2=eps2)
            say("  ni=%d nn-mismatch %d" % (ni, mism))
            if prec == nbx.NBX_FP64:
                assert (e_acc / kappa).max() <= 1e-14 and e_acc[kappa <= 10].max() <= 1e-13
                assert e_pot.max() <= 1e-13 and e_jc.max() <= 1e-13
                assert mism == 0
            else:
                assert (e_acc / kappa).max() <= 5e-7
                assert e_acc[kappa <= 5].max() <= 1e-6 and e_pot.max() <= 1e-6 and e_jc.max() <= 2e-6


def _pair_r2(xp, sink_x):
    d = xp[None, :, :] - sink_x[:, None, :]
    return np.sum(d * d, axis=2)


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
@pytest.mark.parametrize("order", [4, 6])
def test_neighbour_lists(order, prec):
    """Neighbour sets equal the oracle's; in mixed precision pairs within 2e-6 relative of the
    radius may fall either way."""
    n, t, nbr_max = 3000, 0.0, 64
    eps2 = 1e-4 if order == 4 else 1e-6
    say("neighbour lists order=%d prec=%s" % (order, PREC_NAME[prec]))
    src = nbody_ics.make_sources(n, seed=40, order=order, masses="salpeter" if order == 6 else "equal")
    sel = nbody_ics.active_set(n, 1500, seed=41)
    rng = np.random.default_rng(42)
    h2 = rng.uniform(0.002, 0.01, size=len(sel))
    ref = oracle_all(src, order, eps2, t, addr=sel, h2=h2, nbr_max=n)
    with nbx.Context(order=order, precision=prec, nj_max=n, ni_max=n, nbr_max=nbr_max) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        ctx.force(sel, eps2, h2)
        out = ctx.get_force()
        cnt, ids, status = ctx.get_nbr()
    _compare(out, ref, prec, order, sel, src.ids, "  with lists")
    r2 = _pair_r2(ref["xp"], ref["xp"][sel])
    total = 0
    for i in range(len(sel)):
        want = set(ref["nbr_ids"][i, : ref["nbr_count"][i]])
        got = set(ids[i, : min(cnt[i], nbr_max)])
        if prec == nbx.NBX_FP64:
            assert cnt[i] == ref["nbr_count"][i], i
        else:
            border = set(src.ids[np.nonzero(np.abs(r2[i] - h2[i]) <= 2e-6 * h2[i])[0]])
            assert want - border <= got | border and got - border <= want | border, i
            assert abs(int(cnt[i]) - int(ref["nbr_count"][i])) <= len(border), i
        if cnt[i] <= nbr_max:
            assert got <= want | (set() if prec == nbx.NBX_FP64 else border)
        total += cnt[i]
    assert status in (nbx.NBX_OK, nbx.NBX_WARN_NBR_OVERFLOW)
    assert (status == nbx.NBX_WARN_NBR_OVERFLOW) == bool(np.any(cnt > nbr_max))
    say("  mean neighbours %.1f, max %d" % (total / len(sel), cnt.max()))


def test_neighbour_overflow():
    """A dense clump: counts stay exact, stored ids are a subset, the call warns."""
    n, nbr_max = 600, 16
    say("neighbour overflow")
    src = nbody_ics.make_sources(n, seed=43)
    src.x[:300] = src.x[:300] * 1e-3  # 300 sources within ~1e-3 of the centre
    sel = np.arange(0, 300, 7, dtype=np.int32)
    h2 = np.full(len(sel), 1e-2)
    ref = oracle_all(src, 4, 1e-6, 0.0, addr=sel, h2=h2, nbr_max=n)
    with nbx.Context(order=4, precision=nbx.NBX_FP64, nj_max=n, ni_max=n, nbr_max=nbr_max) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        ctx.force(sel, 1e-6, h2)
        out = ctx.get_force()
        cnt, ids, status = ctx.get_nbr()
    assert out["status"] == nbx.NBX_WARN_NBR_OVERFLOW
    assert status == nbx.NBX_WARN_NBR_OVERFLOW
    np.testing.assert_array_equal(cnt, ref["nbr_count"])
    for i in range(len(sel)):
        want = set(ref["nbr_ids"][i, : ref["nbr_count"][i]])
        got = list(ids[i, : min(cnt[i], nbr_max)])
        assert len(set(got)) == len(got) and set(got) <= want


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
@pytest.mark.parametrize("order", [4, 6])
def test_explicit_sinks(order, prec):
    """Sinks given explicitly: foreign ids feel every source; sinks carrying a source's id (at a
    shifted position) exclude exactly that source."""
    n, t = 2500, 0.0
    eps2 = 1e-4
    say("explicit sinks order=%d prec=%s" % (order, PREC_NAME[prec]))
    src = nbody_ics.make_sources(n, seed=44, order=order)
    xp, vp, ap = oracle.predict(order, t, src.t, src.x, src.v, src.a, src.jerk, src.snap, src.crackle)
    rng = np.random.default_rng(45)
    ni = 700
    own = rng.choice(n, size=ni // 2, replace=False)
    ids = np.concatenate([src.ids[own], np.arange(10**6, 10**6 + ni - ni // 2)]).astype(np.int64)
    x = np.concatenate([xp[own] + rng.normal(0, 1e-3, (ni // 2, 3)), rng.normal(0, 0.5, (ni - ni // 2, 3))])
    v = rng.normal(0, 0.5, (ni, 3))
    a = rng.normal(0, 0.5, (ni, 3)) if order == 6 else None
    h2 = np.full(ni, 4e-3)
    ref = oracle.force(order, eps2, src.ids, src.m, xp, vp, ids, x, v, aj=ap if order == 6 else None, ai=a,
                       h2=h2, nbr_max=n)
    ref["xp"] = xp
    with nbx.Context(order=order, precision=prec, nj_max=n, ni_max=ni, nbr_max=32) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        ctx.force_ext(ids, x, v, a, eps2, h2)
        out = ctx.get_force()
        cnt, nb, _ = ctx.get_nbr()
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
    say("  ext: max rel acc %.2e pot %.2e" % (e_acc.max(), e_pot.max()))
    assert e_acc.max() <= TOL[prec]["acc"] and e_pot.max() <= TOL[prec]["pot"]
    assert not np.any(out["nn_id"] == ids)  # never the sink's own source
    d = xp[out["nn_id"]] - x
    np.testing.assert_allclose(out["nn_r2"], np.sum(d * d, axis=1), rtol=1e-13)
    slack = 1e-14 if prec == nbx.NBX_FP64 else 4e-7
    assert np.all(out["nn_r2"] <= ref["nn_r2"] * (1 + slack))
    if prec == nbx.NBX_FP64:
        np.testing.assert_array_equal(cnt, ref["nbr_count"])


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order6_million_sampled(prec):
    """1048576-body Plummer cluster with Salpeter masses, eps2 = 1e-8, 6th order with neighbour
    lists (h2 = 1e-4, at most 256): the launch shapes of N_i = 1024, 65536 and N, checked on
    sampled sinks against the oracle (forces, nearest neighbour and neighbour sets)."""
    n, eps2, h2v, nbr_max = 1 << 20, 1e-8, 1e-4, 256
    say("order6 1M prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=3, order=6, masses="salpeter")
    rng = np.random.default_rng(78)
    with nbx.Context(order=6, precision=prec, nj_max=n, ni_max=n, nbr_max=nbr_max) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        for ni in (1024, 65536, n):
            sel = nbody_ics.active_set(n, ni, seed=1003)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            ctx.force(sel, eps2, np.full(ni, h2v))
            out = ctx.get_force()
            cnt, ids, status = ctx.get_nbr()
            pick = np.sort(rng.choice(ni, size=96, replace=False))
            ref = oracle_all(src, 6, eps2, 0.0, addr=sel[pick], h2=np.full(96, h2v), nbr_max=n)
            got = {k: (v[pick] if v is not None else None) for k, v in out.items() if k != "status"}
            _compare(got, ref, prec, 6, sel[pick], src.ids, "  ni=%d" % ni)
            r2 = _pair_r2(ref["xp"], ref["xp"][sel[pick]])
            for a, i in enumerate(pick):
                want = set(ref["nbr_ids"][a, : ref["nbr_count"][a]])
                have = set(ids[i, : min(cnt[i], nbr_max)])
                if prec == nbx.NBX_FP64:
                    assert cnt[i] == ref["nbr_count"][a]
                    assert have == want or cnt[i] > nbr_max
                else:
                    border = set(src.ids[np.nonzero(np.abs(r2[a] - h2v) <= 2e-6 * h2v)[0]])
                    assert want - border <= have | border
            say("  ni=%d mean neighbours %.2f max %d status %d" % (ni, cnt.mean(), cnt.max(), status))
