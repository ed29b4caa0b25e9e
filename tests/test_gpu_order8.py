"""Order 8 (acc, jerk, snap, crackle; Conclusion: the next expansion of the double-precision
storage) against the FP64 oracle, element by element, on seeded inputs.

Bounds per sink (max over sinks): acc and pot relative error as at the other orders (FP64 1e-13,
mixed 1e-6; the mixed acc bound is plain on sinks whose pair terms cancel little and
condition-normalised on every sink); jerk, snap and crackle condition-normalised (error over
sum_j |pair term|), as the jerk and snap of the other orders.  The crackle pair term is the snap's
products plus one more product per component and the gamma factor, each rounded once more, so its
bound is twice the snap's: FP64 2e-12, mixed 2e-5 (the mixed path carries the jerks in FP32).

The 1048576-body case (eps2 = 1e-8) has pairs with |x| / |r| near 1e3: there a difference of one
or two units of rounding between two FP64 predictors of the same source is amplified a thousand
times.  Perturbing the oracle's own predicted positions and velocities by up to two units changes
its acc by up to 1.2e-13 and its jerk, snap and crackle by up to 2.8e-13, 3.5e-13 and 4.4e-13
(condition-normalised, on the sampled sinks).  That is the floor of any comparison there, so the
FP64 derivative bounds of that case are 1e-12; acc keeps its 1e-13.
"""

import numpy as np
import pytest

import nbody_ics
import oracle
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, check_nn, cond_err_vec, rel_err_vec, run_gpu, say

pytestmark = pytest.mark.gpu

TOL = {
    nbx.NBX_FP64: dict(acc=1e-13, pot=1e-13, jerk_cond=1e-13, snap_cond=1e-12, crackle_cond=2e-12),
    nbx.NBX_MIXED: dict(acc=1e-6, pot=1e-6, jerk_cond=2e-6, snap_cond=1e-5, crackle_cond=2e-5),
}
TOL_1M = {
    nbx.NBX_FP64: dict(TOL[nbx.NBX_FP64], jerk_cond=1e-12, snap_cond=1e-12, crackle_cond=1e-12),
    nbx.NBX_MIXED: TOL[nbx.NBX_MIXED],
}


def oracle8(src, eps2, t, addr, h2=None, nbr_max=0):
    """Oracle order-8 forces on sinks taken by address from the predicted sources."""
    xp, vp, ap = oracle.predict(8, t, src.t, src.x, src.v, src.a, src.jerk, src.snap, src.crackle)
    jp = oracle.predict_jerk(t, src.t, src.jerk, src.snap, src.crackle)
    sel = np.asarray(addr)
    ref = oracle.force8(eps2, src.ids, src.m, xp, vp, ap, jp, src.ids[sel], xp[sel], vp[sel], ap[sel], jp[sel],
                        h2=h2, nbr_max=nbr_max)
    ref["xp"] = xp
    ref["eps2"] = eps2
    return ref


def _sub(ref, pick):
    return {k: (v if k in ("xp", "eps2") or v is None else v[pick]) for k, v in ref.items()}


KAPPA_MAX = 10.0  # mixed: plain relative acc bound on sinks with kappa = sum_j |a_ij| / |a| up to this


def _compare(out, ref, prec, sel_addr, ids, label, tols=TOL):
    """FP64: every bound on every sink.  Mixed: the acc bound holds as a plain relative error on
    sinks whose acceleration is a sum of terms that do not cancel much (kappa <= KAPPA_MAX) and
    condition-normalised on every sink (FP32 pair terms carry their own rounding, which a
    cancelling sum cannot remove); the plain maximum and its kappa are reported."""
    tol = tols[prec]
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    kappa = ref["cond"][:, 0] / np.linalg.norm(ref["acc"], axis=1)
    worst = int(np.argmax(e_acc))
    say("%s: plain max rel acc %.2e at kappa %.1f" % (label, e_acc[worst], kappa[worst]))
    if prec == nbx.NBX_MIXED:
        assert e_acc[kappa <= KAPPA_MAX].max(initial=0.0) <= tol["acc"]
        e_acc = e_acc / kappa
    e = {
        "acc": e_acc.max(),
        "pot": (np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])).max(),
        "jerk_cond": cond_err_vec(out["jerk"], ref["jerk"], ref["cond"][:, 1]).max(),
        "snap_cond": cond_err_vec(out["snap"], ref["snap"], ref["cond"][:, 2]).max(),
        "crackle_cond": cond_err_vec(out["crackle"], ref["crackle"], ref["cond"][:, 3]).max(),
    }
    mism = check_nn(out, ref, ref["xp"], sel_addr, prec, ids)
    msg = "%s: %s nn-mismatch %d" % (label, " ".join("%s %.2e" % kv for kv in e.items()), mism)
    say(msg)
    for k, v in e.items():
        assert v <= tol[k], msg
    if prec == nbx.NBX_FP64:
        assert mism == 0, msg
    return e


def test_order8_predictor():
    """Positions, velocities and accelerations predicted at order 8 are those of the oracle (the
    same polynomial as order 6)."""
    n, t = 3000, 0.01
    say("order8 predictor n=%d seed=121" % n)
    src = nbody_ics.make_sources(n, seed=121, order=8)
    xp, vp, ap = oracle.predict(8, t, src.t, src.x, src.v, src.a, src.jerk, src.snap, src.crackle)
    with nbx.Context(order=8, nj_max=n, ni_max=16) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        gx, gv, ga = ctx.get_predicted(np.arange(n, dtype=np.int32))
    np.testing.assert_allclose(gx, xp, rtol=2e-15, atol=1e-15)
    np.testing.assert_allclose(gv, vp, rtol=2e-15, atol=1e-14)
    np.testing.assert_allclose(ga, ap, rtol=2e-15, atol=1e-13)


NI_CASES = [1, 3, 63, 64, 65, 257, 1000, 3000]


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order8_parity_active_sets(prec):
    """Active sets of several size classes (lanes/wave/split edges) against a ragged source count
    (3000 = 11 full tiles and a partial one), sources at their own times t_j < t (predicted jerk)."""
    n, t, eps2 = 3000, 0.0, 1e-6
    say("order8 parity prec=%s n=%d eps2=%g seed=122" % (PREC_NAME[prec], n, eps2))
    src = nbody_ics.make_sources(n, seed=122, order=8, masses="salpeter")
    ref_all = oracle8(src, eps2, t, np.arange(n))
    with nbx.Context(order=8, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        for ni in NI_CASES:
            sel = nbody_ics.active_set(n, ni, seed=1100 + ni)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            ctx.force(sel, eps2)
            out = ctx.get_force()
            _compare(out, _sub(ref_all, sel), prec, sel, src.ids, "  ni=%d" % ni)
            again = ctx.get_force()
            np.testing.assert_array_equal(again["crackle"], out["crackle"])


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order8_neighbour_lists(prec):
    """Order 8 with neighbour lists: forces, and neighbour sets equal to the oracle's (in mixed,
    pairs within 2e-6 relative of the radius may fall either way)."""
    n, t, eps2, nbr_max = 3000, 0.0, 1e-6, 64
    say("order8 neighbour lists prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=123, order=8, masses="salpeter")
    sel = nbody_ics.active_set(n, 1500, seed=124)
    h2 = np.random.default_rng(125).uniform(0.002, 0.01, size=len(sel))
    ref = oracle8(src, eps2, t, sel, h2=h2, nbr_max=n)
    with nbx.Context(order=8, precision=prec, nj_max=n, ni_max=n, nbr_max=nbr_max) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        ctx.force(sel, eps2, h2)
        out = ctx.get_force()
        cnt, ids, status = ctx.get_nbr()
    _compare(out, ref, prec, sel, src.ids, "  with lists")
    xs = ref["xp"][sel]
    for i in range(len(sel)):
        want = set(ref["nbr_ids"][i, : ref["nbr_count"][i]])
        got = set(ids[i, : min(cnt[i], nbr_max)])
        if prec == nbx.NBX_FP64:
            assert cnt[i] == ref["nbr_count"][i], i
            if cnt[i] <= nbr_max:
                assert got == want, i
        else:
            d = ref["xp"] - xs[i]
            r2 = np.sum(d * d, axis=1)
            border = set(src.ids[np.nonzero(np.abs(r2 - h2[i]) <= 2e-6 * h2[i])[0]])
            assert want - border <= got | border or cnt[i] > nbr_max, i
            assert abs(int(cnt[i]) - int(ref["nbr_count"][i])) <= len(border), i
    assert status in (nbx.NBX_OK, nbx.NBX_WARN_NBR_OVERFLOW)


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order8_million_sampled(prec):
    """1048576-body Plummer cluster with Salpeter masses, eps2 = 1e-8, order 8 with neighbour lists
    (h2 = 1e-4, at most 256), through the device entry point: the launch shapes of N_i = 1024 and
    N, checked on sampled sinks against the oracle."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    n, eps2, h2v, nbr_max = 1 << 20, 1e-8, 1e-4, 256
    say("order8 1M prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=3, order=8, masses="salpeter")
    rng = np.random.default_rng(126)
    T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    with nbx.Context(order=8, precision=prec, nj_max=n, ni_max=n, nbr_max=nbr_max) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        stream = torch.cuda.current_stream()
        for ni in (1024, n):
            sel = nbody_ics.active_set(n, ni, seed=1003)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            outs = {k: torch.empty((ni, 3), dtype=torch.float64, device=dev) for k in ("acc", "jerk", "snap",
                                                                                       "crackle")}
            outs["pot"] = torch.empty(ni, dtype=torch.float64, device=dev)
            outs["nn_id"] = torch.empty(ni, dtype=torch.int64, device=dev)
            outs["nn_r2"] = torch.empty(ni, dtype=torch.float64, device=dev)
            cnt = torch.empty(ni, dtype=torch.int32, device=dev)
            ids = torch.empty((ni, nbr_max), dtype=torch.int64, device=dev)
            nbx.nbx_force8_dev(ctx.ctx, stream, ni, T(sel, torch.int32), eps2, T(np.full(ni, h2v)), outs["acc"],
                               outs["jerk"], outs["snap"], outs["crackle"], outs["pot"], outs["nn_id"],
                               outs["nn_r2"], cnt, ids)
            status = nbx.nbx_sync(ctx.ctx, stream)
            pick = np.sort(rng.choice(ni, size=64, replace=False))
            got = {k: v.cpu().numpy()[pick] for k, v in outs.items()}
            cnt_h, ids_h = cnt.cpu().numpy(), ids.cpu().numpy()
            ref = oracle8(src, eps2, 0.0, sel[pick], h2=np.full(64, h2v), nbr_max=n)
            _compare(got, ref, prec, sel[pick], src.ids, "  ni=%d" % ni, TOL_1M)
            if prec == nbx.NBX_FP64:
                for a, i in enumerate(pick):
                    assert cnt_h[i] == ref["nbr_count"][a]
                    want = set(ref["nbr_ids"][a, : ref["nbr_count"][a]])
                    assert set(ids_h[i, : min(cnt_h[i], nbr_max)]) == want or cnt_h[i] > nbr_max
            say("  ni=%d mean neighbours %.2f max %d status %d" % (ni, cnt_h.mean(), cnt_h.max(), status))


def test_order8_device_path_and_errors():
    """The device entry point gives the host path's bits; order-8 contexts refuse the entry points
    of other orders (explicit sinks, nbx_force_dev, the integrator) and the others refuse the
    order-8 ones."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda:0")
    n, ni, eps2 = 2000, 700, 1e-6
    say("order8 device path n=%d ni=%d" % (n, ni))
    src = nbody_ics.make_sources(n, seed=127, order=8)
    sel = nbody_ics.active_set(n, ni, seed=128)
    T = lambda a, dt=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=dt, device=dev)
    lib = nbx.load()
    with nbx.Context(order=8, precision=nbx.NBX_MIXED, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        ctx.force(sel, eps2)
        host = ctx.get_force()
        stream = torch.cuda.current_stream()
        d = {k: torch.empty((ni, 3), dtype=torch.float64, device=dev) for k in ("acc", "jerk", "snap", "crackle")}
        d["pot"] = torch.empty(ni, dtype=torch.float64, device=dev)
        d["nn_id"] = torch.empty(ni, dtype=torch.int64, device=dev)
        d["nn_r2"] = torch.empty(ni, dtype=torch.float64, device=dev)
        d_sel = T(sel, torch.int32)
        nbx.nbx_force8_dev(ctx.ctx, stream, ni, d_sel, eps2, None, d["acc"], d["jerk"], d["snap"], d["crackle"],
                           d["pot"], d["nn_id"], d["nn_r2"])
        nbx.nbx_sync(ctx.ctx, stream)
        for k, v in d.items():
            np.testing.assert_array_equal(v.cpu().numpy(), host[k])
        # refused at order 8, before any work is enqueued
        assert lib.nbx_force_dev(ctx.ctx, None, ni, d_sel.data_ptr(), eps2, None, d["acc"].data_ptr(),
                                 d["jerk"].data_ptr(), d["snap"].data_ptr(), d["pot"].data_ptr(),
                                 d["nn_id"].data_ptr(), d["nn_r2"].data_ptr(), None, None) == nbx.NBX_ERR_ARG
        assert lib.nbx_force8_dev(ctx.ctx, None, ni, d_sel.data_ptr(), eps2, None, d["acc"].data_ptr(),
                                  d["jerk"].data_ptr(), d["snap"].data_ptr(), None, d["pot"].data_ptr(),
                                  d["nn_id"].data_ptr(), d["nn_r2"].data_ptr(), None, None) == nbx.NBX_ERR_ARG
        with pytest.raises(nbx.NbxError) as e:  # order 8 explicit sinks go through nbx_force_ext8
            nbx.nbx_force_ext(ctx.ctx, np.arange(10**6, 10**6 + 4), np.zeros((4, 3)), np.zeros((4, 3)),
                              np.zeros((4, 3)), eps2)
        assert e.value.code == nbx.NBX_ERR_ARG
        with pytest.raises(nbx.NbxError) as e:  # which needs the sink jerks
            ctx.force_ext(np.arange(10**6, 10**6 + 4), np.zeros((4, 3)), np.zeros((4, 3)), np.zeros((4, 3)), eps2)
        assert e.value.code == nbx.NBX_ERR_ARG
        with pytest.raises(nbx.NbxError) as e:
            nbx.nbx_bs_init(ctx.ctx, src.ids[:100], src.m[:100], src.x[:100], src.v[:100], 1e-4)
        assert e.value.code == nbx.NBX_ERR_ARG
    with nbx.Context(order=6, precision=nbx.NBX_MIXED, nj_max=n, ni_max=n) as ctx6:
        ctx6.set_sources(src)
        ctx6.predict(0.0)
        ctx6.force(sel, eps2)
        crackle = np.empty((ni, 3))
        assert lib.nbx_get_crackle(ctx6.ctx, crackle.ctypes.data) == nbx.NBX_ERR_ARG
        with pytest.raises(nbx.NbxError) as e:
            nbx.nbx_force_ext8(ctx6.ctx, np.arange(10**6, 10**6 + 4), np.zeros((4, 3)), np.zeros((4, 3)),
                               np.zeros((4, 3)), np.zeros((4, 3)), eps2)
        assert e.value.code == nbx.NBX_ERR_ARG
        assert lib.nbx_force8_dev(ctx6.ctx, None, ni, d_sel.data_ptr(), eps2, None, d["acc"].data_ptr(),
                                  d["jerk"].data_ptr(), d["snap"].data_ptr(), d["crackle"].data_ptr(),
                                  d["pot"].data_ptr(), d["nn_id"].data_ptr(), d["nn_r2"].data_ptr(), None,
                                  None) == nbx.NBX_ERR_ARG
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order8_tuned_shapes(prec):
    """The launch-shape tuner on an order-8 context: the shapes it keeps (which may put two sinks
    on a lane) keep parity with the oracle."""
    n, t, eps2 = 3000, 0.0, 1e-6
    say("order8 tuned prec=%s n=%d seed=129" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=129, order=8, masses="salpeter")
    ref_all = oracle8(src, eps2, t, np.arange(n))
    with nbx.Context(order=8, precision=prec, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        tab = ctx.tune(n)
        say("  table (L, P, S) per class: %s" % tab.tolist())
        ctx.predict(t)
        for ni in (1, 300, 3000):
            sel = nbody_ics.active_set(n, ni, seed=1300 + ni)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            ctx.force(sel, eps2)
            _compare(ctx.get_force(), _sub(ref_all, sel), prec, sel, src.ids, "  ni=%d" % ni)


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_order8_explicit_sinks(prec):
    """Explicit order-8 sinks (x, v, a, jerk used as given): foreign ids feel every source; sinks
    carrying a source's id, at a shifted position, exclude exactly that source."""
    n, t, eps2, ni = 2500, 0.0, 1e-4, 700
    say("order8 explicit sinks prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=130, order=8)
    xp, vp, ap = oracle.predict(8, t, src.t, src.x, src.v, src.a, src.jerk, src.snap, src.crackle)
    jp = oracle.predict_jerk(t, src.t, src.jerk, src.snap, src.crackle)
    rng = np.random.default_rng(131)
    own = rng.choice(n, size=ni // 2, replace=False)
    ids = np.concatenate([src.ids[own], np.arange(10**6, 10**6 + ni - ni // 2)]).astype(np.int64)
    x = np.concatenate([xp[own] + rng.normal(0, 1e-3, (ni // 2, 3)), rng.normal(0, 0.5, (ni - ni // 2, 3))])
    v, a, jerk = rng.normal(0, 0.5, (ni, 3)), rng.normal(0, 0.5, (ni, 3)), rng.normal(0, 2.0, (ni, 3))
    h2 = np.full(ni, 4e-3)
    ref = oracle.force8(eps2, src.ids, src.m, xp, vp, ap, jp, ids, x, v, a, jerk, h2=h2, nbr_max=n)
    with nbx.Context(order=8, precision=prec, nj_max=n, ni_max=ni, nbr_max=32) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        ctx.force_ext(ids, x, v, a, eps2, h2, jerk=jerk)
        out = ctx.get_force()
        cnt, _, _ = ctx.get_nbr()
    tol = TOL[prec]
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    kappa = ref["cond"][:, 0] / np.linalg.norm(ref["acc"], axis=1)
    e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
    e_snap = cond_err_vec(out["snap"], ref["snap"], ref["cond"][:, 2])
    e_crk = cond_err_vec(out["crackle"], ref["crackle"], ref["cond"][:, 3])
    say("  ext: max rel acc %.2e (kappa %.1f) pot %.2e snap/cond %.2e crackle/cond %.2e" % (
        e_acc.max(), kappa[np.argmax(e_acc)], e_pot.max(), e_snap.max(), e_crk.max()))
    if prec == nbx.NBX_FP64:
        assert e_acc.max() <= tol["acc"]
    else:
        assert e_acc[kappa <= KAPPA_MAX].max(initial=0.0) <= tol["acc"] and (e_acc / kappa).max() <= tol["acc"]
    assert e_pot.max() <= tol["pot"] and e_snap.max() <= tol["snap_cond"] and e_crk.max() <= tol["crackle_cond"]
    assert not np.any(out["nn_id"] == ids)  # never the sink's own source
    d = xp[out["nn_id"]] - x
    r2 = np.sum(d * d, axis=1)  # two FP64 predictors agree to rounding in x; x_j - x_i cancels
    scale = np.maximum(np.linalg.norm(x, axis=1), np.linalg.norm(xp[out["nn_id"]], axis=1)) * np.sqrt(r2)
    assert np.all(np.abs(out["nn_r2"] - r2) <= 1e-13 * r2 + 16 * np.finfo(np.float64).eps * scale)
    slack = 1e-14 if prec == nbx.NBX_FP64 else 4e-7
    assert np.all(out["nn_r2"] <= ref["nn_r2"] * (1 + slack))
    if prec == nbx.NBX_FP64:
        np.testing.assert_array_equal(cnt, ref["nbr_count"])


def test_order8_hermite_steps_match_oracle():
    """Eight shared 8th-order Hermite steps (dt = 1/256, two evaluate-correct passes per step) on a
    256-body Plummer sphere, driven through the GPU (FP64) and through the oracle, agree to 1e-12 in
    positions and velocities.  The GPU side corrects with the closed-form two-point Hermite
    quadrature (weights 1/2, 3/28, 1/84, 1/1680), the oracle with its interpolating polynomials."""
    from oracle import blockstep as bs

    n, eps2, dt, nsteps = 256, 1e-4, 1.0 / 256, 8
    say("order8 hermite %d steps n=%d" % (nsteps, n))
    src = nbody_ics.make_sources(n, seed=132, order=8, time_offsets=False)
    ids, m, addr = src.ids, src.m, np.arange(n, dtype=np.int32)
    zeros = np.zeros((n, 3))

    def corrector8(h, x0, v0, a0, j0, s0, c0, a1, j1, s1, c1):  # the GPU side's own corrector
        v1 = v0 + h / 2 * (a0 + a1) + 3 * h**2 / 28 * (j0 - j1) + h**3 / 84 * (s0 + s1) + h**4 / 1680 * (c0 - c1)
        x1 = x0 + h / 2 * (v0 + v1) + 3 * h**2 / 28 * (a0 - a1) + h**3 / 84 * (j0 + j1) + h**4 / 1680 * (s0 - s1)
        return x1, v1

    with nbx.Context(order=8, nj_max=n, ni_max=n) as ctx:
        def gpu_forces(t, x, v, a, j, s, c, t_eval):
            nbx.nbx_set_j(ctx.ctx, addr, ids, m, np.full(n, t), x, v, a, j, s, c)
            ctx.predict(t_eval)
            f = run_gpu(ctx, addr, eps2)
            return f["acc"], f["jerk"], f["snap"], f["crackle"]

        x, v = src.x.copy(), src.v.copy()
        a, j, _, _ = gpu_forces(0.0, x, v, zeros, zeros, zeros, zeros, 0.0)
        a, j, s, c = gpu_forces(0.0, x, v, a, j, zeros, zeros, 0.0)
        t = 0.0
        for _ in range(nsteps):
            d1 = gpu_forces(t, x, v, a, j, s, c, t + dt)
            for _ in range(2):
                x1, v1 = corrector8(dt, x, v, a, j, s, c, *d1)
                d1 = gpu_forces(t + dt, x1, v1, d1[0], d1[1], d1[2], d1[3], t + dt)
            x, v, (a, j, s, c) = x1, v1, d1
            t += dt
        xg, vg = x, v

    def oracle_forces(x, v, a, j):
        f = oracle.force8(eps2, ids, m, x, v, a, j, ids, x, v, a, j)
        return f["acc"], f["jerk"], f["snap"], f["crackle"]

    x, v = src.x.copy(), src.v.copy()
    a, j, _, _ = oracle_forces(x, v, zeros, zeros)
    a, j, s, c = oracle_forces(x, v, a, j)
    t = 0.0
    for _ in range(nsteps):
        xp, vp, ap = oracle.predict(8, t + dt, np.full(n, t), x, v, a, j, s, c)
        jp = oracle.predict_jerk(t + dt, np.full(n, t), j, s, c)
        d1 = oracle_forces(xp, vp, ap, jp)
        for _ in range(2):
            x1, v1 = bs.hermite8_correct(np.full(n, dt), x, v, a, j, s, c, *d1)
            d1 = oracle_forces(x1, v1, d1[0], d1[1])
        x, v, (a, j, s, c) = x1, v1, d1
        t += dt
    ex = np.abs(xg - x).max() / np.abs(x).max()
    ev = np.abs(vg - v).max() / np.abs(v).max()
    say("  max rel dx %.2e dv %.2e" % (ex, ev))
    assert ex <= 1e-12 and ev <= 1e-12


def test_order8_state_and_capacity_errors():
    """Order-8 entry points report call-order and capacity errors without touching the device
    state: crackle before any force call, too many sinks, and an empty sink set."""
    torch = pytest.importorskip("torch")
    n = 500
    say("order8 state and capacity errors")
    src = nbody_ics.make_sources(n, seed=133, order=8)
    lib = nbx.load()
    with nbx.Context(order=8, nj_max=n, ni_max=100) as ctx:
        crackle = np.empty((100, 3))
        assert lib.nbx_get_crackle(ctx.ctx, crackle.ctypes.data) == nbx.NBX_ERR_STATE
        ctx.set_sources(src)
        ctx.predict(0.0)
        d = {k: torch.empty((200, 3), dtype=torch.float64, device="cuda:0") for k in ("a", "j", "s", "c")}
        o = torch.empty(200, dtype=torch.float64, device="cuda:0")
        i64 = torch.empty(200, dtype=torch.int64, device="cuda:0")
        addr = torch.arange(200, dtype=torch.int32, device="cuda:0")
        assert lib.nbx_force8_dev(ctx.ctx, None, 200, addr.data_ptr(), 1e-4, None, d["a"].data_ptr(),
                                  d["j"].data_ptr(), d["s"].data_ptr(), d["c"].data_ptr(), o.data_ptr(),
                                  i64.data_ptr(), o.data_ptr(), None, None) == nbx.NBX_ERR_CAPACITY
        assert lib.nbx_force8_dev(ctx.ctx, None, 0, None, 1e-4, None, None, None, None, None, None, None, None,
                                  None, None) == nbx.NBX_OK
        ctx.force(np.arange(0, dtype=np.int32), 1e-4)  # an empty sink set is a valid call
        out = ctx.get_force()
        assert out["crackle"].shape == (0, 3)
        torch.cuda.synchronize()
