"""Double-single precision (NBX_DS, orders 4 and 6): the paper's DS force computation, every pair
quantity in double-single arithmetic from the FP64 predicted state.

Bounds, from the arithmetic: a double-single value carries 48 significant bits (unit roundoff
u = 2^-48 ~ 3.6e-15), each pair term passes through ~40 such roundings, and the FP64 positions are
cut to 48 bits before the differences, which a close pair amplifies by |x| / |r| (~1e2 on these
clusters).  Hence acc and pot within 1e-12 relative and the jerk and snap within 1e-11
condition-normalised, against the FP64 oracle; the nearest neighbour is chosen on the leading
FP32 part of the DS |r|^2 and is checked as in mixed precision.  The 6th-order block time-step
integrator driven by DS forces completes without the step collapse of the mixed path and stays
close to the FP64-driven run (Results > Block time-step simulations)."""

import numpy as np
import pytest

import nbody_ics
import oracle
import paper_1510_04068_amd as nbx
from gpu_helpers import check_nn, cond_err_vec, oracle_all, rel_err_vec, run_gpu, say, subset

pytestmark = pytest.mark.gpu

NI_CASES = [1, 3, 64, 257, 1000, 3000]


def _check(out, ref, order, sel, ids, label):
    e_acc = rel_err_vec(out["acc"], ref["acc"])
    e_pot = np.abs(out["pot"] - ref["pot"]) / np.abs(ref["pot"])
    e_jc = cond_err_vec(out["jerk"], ref["jerk"], ref["cond"][:, 1])
    msg = "%s: max rel acc %.2e pot %.2e jerk/cond %.2e" % (label, e_acc.max(), e_pot.max(), e_jc.max())
    if order == 6:
        e_sc = cond_err_vec(out["snap"], ref["snap"], ref["cond"][:, 2])
        msg += " snap/cond %.2e" % e_sc.max()
        assert e_sc.max() <= 1e-11, msg
    check_nn(out, ref, ref["xp"], sel, nbx.NBX_MIXED, ids)
    say(msg)
    assert e_acc.max() <= 1e-12 and e_pot.max() <= 1e-12 and e_jc.max() <= 1e-11, msg


@pytest.mark.parametrize("order", [4, 6])
def test_ds_parity_active_sets(order):
    n, t, eps2 = 3000, 0.0, 1e-6
    say("ds parity order=%d n=%d seed=22" % (order, n))
    src = nbody_ics.make_sources(n, seed=22, order=order, masses="salpeter")
    ref_all = oracle_all(src, order, eps2, t)
    with nbx.Context(order=order, precision=nbx.NBX_DS, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(t)
        for ni in NI_CASES:
            sel = nbody_ics.active_set(n, ni, seed=1000 + ni)
            say("  ni=%d shape=%s" % (ni, ctx.launch_shape(ni)))
            out = run_gpu(ctx, sel, eps2)
            _check(out, subset(ref_all, sel), order, sel, src.ids, "  ni=%d" % ni)


def test_ds_full_size_sampled():
    """The headline workload (N = 131072, per-source times) with every sink active, 2048 sampled
    sinks, 4th order; and eps2 = 0 with the guarded self term on a ragged source count."""
    n, eps2 = 131072, 1e-6
    say("ds full size n=%d" % n)
    src = nbody_ics.make_sources(n, seed=2)
    sel = np.arange(n, dtype=np.int32)
    pick = np.sort(np.random.default_rng(79).choice(n, size=2048, replace=False))
    with nbx.Context(order=4, precision=nbx.NBX_DS, nj_max=n, ni_max=n) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        say("  shape=%s" % ctx.launch_shape(n))
        out = run_gpu(ctx, sel, eps2)
    ref = oracle_all(src, 4, eps2, 0.0, addr=pick)
    got = {k: (v[pick] if v is not None else None) for k, v in out.items() if k != "status"}
    _check(got, ref, 4, pick, src.ids, "  n=131072")
    m = 1001
    src = nbody_ics.make_sources(m, seed=23)
    ref = oracle_all(src, 4, 0.0, 0.0)
    with nbx.Context(order=4, precision=nbx.NBX_DS, nj_max=m, ni_max=m) as ctx:
        ctx.set_sources(src)
        ctx.predict(0.0)
        out = run_gpu(ctx, np.arange(m, dtype=np.int32), 0.0)
    _check(out, ref, 4, np.arange(m), src.ids, "  eps2=0 n=1001")


def test_ds_only_where_built():
    for order in (2, 8):
        with pytest.raises(nbx.NbxError) as e:
            nbx.Context(order=order, precision=nbx.NBX_DS, nj_max=8, ni_max=8)
        assert e.value.code == nbx.NBX_ERR_ARG
        with nbx.Context(order=order, nj_max=8, ni_max=8) as ctx:
            with pytest.raises(nbx.NbxError) as e:
                ctx.set_precision(nbx.NBX_DS)
            assert e.value.code == nbx.NBX_ERR_ARG


def _bs_run(prec, m, x, v, eps2, t_end):
    n = len(m)
    with nbx.Context(order=6, precision=prec, nj_max=n, ni_max=n) as ctx:
        nbx.nbx_bs_init(ctx.ctx, np.arange(n), m, x, v, eps2, eta4=0.01, eta6=0.1, eta_start=0.01)
        e0 = sum(nbx.nbx_bs_energy(ctx.ctx))
        st = nbx.nbx_bs_run(ctx.ctx, t_end)
        full = nbx.nbx_bs_get_state(ctx.ctx, n)
        e1 = sum(nbx.nbx_bs_energy(ctx.ctx))
    return st, full, abs((e1 - e0) / e0)


def test_ds_blockstep_order6_completes():
    """6th-order block steps (averaged criterion, eta4 = 0.01, eta6 = 0.1) with DS forces on a
    1024-body Plummer sphere to t = 1/8: no step clamped at dt_min, the final state within 1e-8 of
    the FP64-driven run and the energy error below 1e-9, where the mixed path's criterion
    collapses (see test_blockstep_mixed_order6_collapse_known)."""
    n, eps2, t_end = 1024, 1e-6, 1.0 / 8
    say("ds blockstep order 6 n=%d t_end=%g" % (n, t_end))
    m, x, v = nbody_ics.plummer(n, seed=7)
    st_d, full_d, de_d = _bs_run(nbx.NBX_DS, m, x, v, eps2, t_end)
    st_f, full_f, de_f = _bs_run(nbx.NBX_FP64, m, x, v, eps2, t_end)
    ex = np.abs(full_d["x"] - full_f["x"]).max() / np.abs(full_f["x"]).max()
    say("  DS: status %d t %g blocks %d <N_active> %.1f dE/E %.2e | FP64: blocks %d dE/E %.2e | max rel dx %.2e"
        % (st_d["status"], st_d["t"], st_d["block_steps"], st_d["particle_steps"] / max(st_d["block_steps"], 1),
           de_d, st_f["block_steps"], de_f, ex))
    assert st_d["status"] == nbx.NBX_OK and st_d["t"] == t_end
    assert ex <= 1e-8
    assert de_d <= 1e-9
