"""Adjoint of the 4th-order force evaluation: the HIP vector-Jacobian product against the oracle's
(itself pinned to finite differences), the torch autograd wrapper against finite differences, and
gradients through 16 checkpointed Hermite steps.

Bounds, as the norm of the gradient error per particle over the largest gradient norm: FP64
1e-12 (each pair term passes ~20 roundings of 1.1e-16, summed over up to 65536 pairs with
compensation); mixed 2e-6 (the same in FP32 arithmetic, u = 6e-8)."""

import numpy as np
import pytest

import nbody_ics
import oracle
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, say

pytestmark = pytest.mark.gpu

TOL = {nbx.NBX_FP64: 1e-12, nbx.NBX_MIXED: 2e-6}


def _err(g, r):
    return np.linalg.norm(g - r, axis=-1) / np.abs(r).max() if g.ndim == 2 else np.abs(g - r) / np.abs(r).max()


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_vjp_matches_oracle(prec):
    torch = pytest.importorskip("torch")
    n, eps2 = 2000, 1e-4
    say("vjp prec=%s n=%d" % (PREC_NAME[prec], n))
    src = nbody_ics.make_sources(n, seed=70, masses="salpeter")
    rng = np.random.default_rng(71)
    ga, gj, gp = rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.normal(size=n)
    rx, rv, rm = oracle.force_vjp(eps2, src.m, src.x, src.v, ga, gj, gp)
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    gx, gv, gm = torch.empty((n, 3), dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64,
                                                                                 device=dev), torch.empty(n, dtype=torch.float64, device=dev)
    with nbx.Context(order=4, precision=prec, nj_max=1, ni_max=1) as ctx:
        nbx.nbx_force_vjp_dev(ctx.ctx, None, n, T(src.m), T(src.x), T(src.v), eps2, T(ga), T(gj), T(gp), gx, gv, gm)
        nbx.nbx_sync(ctx.ctx, None)
    torch.cuda.synchronize()
    ex, ev, em = _err(gx.cpu().numpy(), rx), _err(gv.cpu().numpy(), rv), _err(gm.cpu().numpy(), rm)
    say("  max err x %.2e v %.2e m %.2e" % (ex.max(), ev.max(), em.max()))
    assert max(ex.max(), ev.max(), em.max()) <= TOL[prec]


def _fc(torch, n, prec):
    from paper_1510_04068_amd.autograd import ForceContext

    return ForceContext(n, precision=prec)


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_config5_loss_gradient_sampled(prec):
    """65536-body Plummer sphere, eps2 = 1e-6, loss = seeded weights . (acc, jerk) + total potential
    energy; gradients w.r.t. x, v, m from autograd against the oracle on 128 sampled particles."""
    torch = pytest.importorskip("torch")
    from paper_1510_04068_amd.autograd import forces

    n, eps2 = 65536, 1e-6
    say("config5 prec=%s" % PREC_NAME[prec])
    src = nbody_ics.make_sources(n, seed=5)
    rng = np.random.default_rng(5005)
    wa, wj = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    x, v, m = T(src.x).requires_grad_(), T(src.v).requires_grad_(), T(src.m).requires_grad_()
    fc = _fc(torch, n, prec)
    acc, jerk, pot = forces(x, v, m, eps2, fc)
    loss = (T(wa) * acc).sum() + (T(wj) * jerk).sum() + 0.5 * (m * pot).sum()
    loss.backward()
    torch.cuda.synchronize()
    gx, gv, gm = x.grad.cpu().numpy(), v.grad.cpu().numpy(), m.grad.cpu().numpy()
    pot_h = pot.detach().cpu().numpy()
    fc.close()
    sel = np.sort(rng.choice(n, 128, replace=False)).astype(np.int32)
    rx, rv, rm = oracle.force_vjp(eps2, src.m, src.x, src.v, wa, wj, 0.5 * src.m, sel=sel)
    ref_pot = oracle.force(4, eps2, src.ids, src.m, src.x, src.v, src.ids[sel], src.x[sel], src.v[sel])["pot"]
    rm = rm + 0.5 * ref_pot  # the loss also depends on m directly through 0.5 m pot
    ex, ev, em = _err(gx[sel], rx), _err(gv[sel], rv), _err(gm[sel], rm)
    say("  max err x %.2e v %.2e m %.2e (pot %.2e)" % (ex.max(), ev.max(), em.max(),
                                                       np.abs(pot_h[sel] - ref_pot).max() / np.abs(ref_pot).max()))
    assert max(ex.max(), ev.max(), em.max()) <= TOL[prec]


def test_autograd_matches_finite_differences():
    torch = pytest.importorskip("torch")
    from paper_1510_04068_amd.autograd import forces

    n, eps2 = 48, 1e-3
    say("autograd vs finite differences")
    src = nbody_ics.make_sources(n, seed=72, masses="salpeter")
    rng = np.random.default_rng(73)
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    wa, wj, wp = T(rng.normal(size=(n, 3))), T(rng.normal(size=(n, 3))), T(rng.normal(size=n))
    fc = _fc(torch, n, nbx.NBX_FP64)

    def loss(x, v, m):
        a, j, p = forces(x, v, m, eps2, fc)
        return (wa * a).sum() + (wj * j).sum() + (wp * p).sum()

    x, v, m = T(src.x).requires_grad_(), T(src.v).requires_grad_(), T(src.m).requires_grad_()
    loss(x, v, m).backward()
    for k in range(4):
        dx, dv, dm = T(rng.normal(size=(n, 3))), T(rng.normal(size=(n, 3))), T(rng.normal(size=n) * src.m)
        h = 1e-6
        with torch.no_grad():
            lp = loss(x + h * dx, v + h * dv, m + h * dm).item()
            lm = loss(x - h * dx, v - h * dv, m - h * dm).item()
        fd = (lp - lm) / (2 * h)
        ad = float((x.grad * dx).sum() + (v.grad * dv).sum() + (m.grad * dm).sum())
        say("  direction %d: autograd %.10e fd %.10e" % (k, ad, fd))
        assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-9
    fc.close()


def test_hermite_trajectory_gradient():
    """Gradient of a loss on the state after 16 checkpointed Hermite steps (dt = 1/512) equals the
    non-checkpointed gradient bit for bit and matches finite differences of the whole trajectory."""
    torch = pytest.importorskip("torch")
    from paper_1510_04068_amd.autograd import hermite4

    n, eps2, dt, steps = 256, 1e-6, 1.0 / 512, 16
    say("hermite trajectory gradient n=%d" % n)
    src = nbody_ics.make_sources(n, seed=74, time_offsets=False)
    rng = np.random.default_rng(75)
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    wx, wv = T(rng.normal(size=(n, 3))), T(rng.normal(size=(n, 3)))
    fc = _fc(torch, n, nbx.NBX_FP64)

    def loss(x, v, m, ck):
        x1, v1 = hermite4(x, v, m, eps2, dt, steps, fc, checkpoint=ck)
        return (wx * x1).sum() + (wv * v1).sum()

    grads = []
    for ck in (True, False):
        x, v, m = T(src.x).requires_grad_(), T(src.v).requires_grad_(), T(src.m).requires_grad_()
        loss(x, v, m, ck).backward()
        grads.append((x.grad.clone(), v.grad.clone(), m.grad.clone()))
    for a, b in zip(*grads):
        assert torch.equal(a, b)
    gx, gv, gm = grads[0]
    for k in range(3):
        dx, dv, dm = T(rng.normal(size=(n, 3))), T(rng.normal(size=(n, 3))), T(rng.normal(size=n) * src.m)
        h = 1e-6
        with torch.no_grad():
            lp = loss(T(src.x) + h * dx, T(src.v) + h * dv, T(src.m) + h * dm, False).item()
            lm = loss(T(src.x) - h * dx, T(src.v) - h * dv, T(src.m) - h * dm, False).item()
        fd = (lp - lm) / (2 * h)
        ad = float((gx * dx).sum() + (gv * dv).sum() + (gm * dm).sum())
        say("  direction %d: autograd %.10e fd %.10e" % (k, ad, fd))
        assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-9
    fc.close()


def _oracle_hermite16(x, v, m, eps2, dt, steps):
    """The same 16 shared 4th-order Hermite steps driven entirely by the oracle: its forces, its
    predictor (from t = 0 to dt) and its corrector."""
    n = len(m)
    ids = np.arange(n, dtype=np.int64)
    f = oracle.force(4, eps2, ids, m, x, v, ids, x, v)
    a0, j0 = f["acc"], f["jerk"]
    zeros_t = np.zeros(n)
    for _ in range(steps):
        xp, vp, _ = oracle.predict(4, dt, zeros_t, x, v, a0, j0)
        f = oracle.force(4, eps2, ids, m, xp, vp, ids, xp, vp)
        x, v = oracle.hermite4_correct(dt, xp, vp, a0, j0, f["acc"], f["jerk"])
        a0, j0 = f["acc"], f["jerk"]
    return x, v


def test_hermite_trajectory_gradient_vs_oracle():
    """The checkpointed gradient through 16 Hermite steps (dt = 1/512, N = 256, FP64) against central
    finite differences of the oracle-driven trajectory (oracle forces, predictor and corrector), so
    the gradient is checked against a trajectory the library never computed."""
    torch = pytest.importorskip("torch")
    from paper_1510_04068_amd.autograd import hermite4

    n, eps2, dt, steps = 256, 1e-6, 1.0 / 512, 16
    say("hermite trajectory gradient vs oracle n=%d" % n)
    src = nbody_ics.make_sources(n, seed=76, time_offsets=False)
    rng = np.random.default_rng(77)
    wx_h, wv_h = rng.normal(size=(n, 3)), rng.normal(size=(n, 3))
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    fc = _fc(torch, n, nbx.NBX_FP64)
    x, v, m = T(src.x).requires_grad_(), T(src.v).requires_grad_(), T(src.m).requires_grad_()
    x1, v1 = hermite4(x, v, m, eps2, dt, steps, fc, checkpoint=True)
    ((T(wx_h) * x1).sum() + (T(wv_h) * v1).sum()).backward()
    gx, gv, gm = x.grad.cpu().numpy(), v.grad.cpu().numpy(), m.grad.cpu().numpy()
    fc.close()
    ox, ov = _oracle_hermite16(src.x, src.v, src.m, eps2, dt, steps)
    np.testing.assert_allclose(x1.detach().cpu().numpy(), ox, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v1.detach().cpu().numpy(), ov, rtol=0, atol=1e-11)

    def loss(xx, vv, mm):
        a, b = _oracle_hermite16(xx, vv, mm, eps2, dt, steps)
        return float(np.sum(wx_h * a) + np.sum(wv_h * b))

    for k in range(3):
        dx, dv, dm = rng.normal(size=(n, 3)), rng.normal(size=(n, 3)), rng.normal(size=n) * src.m
        h = 1e-6
        fd = (loss(src.x + h * dx, src.v + h * dv, src.m + h * dm) -
              loss(src.x - h * dx, src.v - h * dv, src.m - h * dm)) / (2 * h)
        ad = float(np.sum(gx * dx) + np.sum(gv * dv) + np.sum(gm * dm))
        say("  direction %d: library gradient %.10e oracle finite difference %.10e" % (k, ad, fd))
        assert abs(ad - fd) <= 1e-6 * abs(fd) + 1e-9
