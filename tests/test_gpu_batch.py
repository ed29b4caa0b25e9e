"""Batched few-body systems: 4096 independent Plummer systems of 3..96 particles, eps2 = 0,
4th order (acc, jerk, pot), one persistent launch, FP64 and mixed, default and autotuned lane
mappings, each system checked against the oracle.

FP64: max relative error of acc and pot <= 1e-13.  Mixed: the per-pair terms carry FP32 rounding
(~2e-7 relative), so a particle whose pair terms nearly cancel (kappa = sum_j |a_ij| / |a| large,
common with eps2 = 0 in small systems) can exceed 1e-6 relative; the bound is applied to the
condition-normalised error |da| / sum_j |a_ij| <= 1e-6 for every particle (about ten FP32 roundings
of u = 6e-8 per pair term) and to the plain relative
error for particles with kappa <= 2.  The plain maximum is printed."""

import numpy as np
import pytest

import nbody_ics
import oracle
import paper_1510_04068_amd as nbx
from gpu_helpers import PREC_NAME, rel_err_vec, say

pytestmark = pytest.mark.gpu


def make_batch(n_sys=4096, seed=4):
    sizes = nbody_ics.few_body_sizes(n_sys, seed)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    m, x, v = [], [], []
    for s, n in enumerate(sizes):
        mm, xx, vv = nbody_ics.plummer(int(n), seed=10000 + s)
        m.append(mm), x.append(xx), v.append(vv)
    return off, np.concatenate(m), np.concatenate(x), np.concatenate(v)


def oracle_batch(off, m, x, v, eps2):
    n = off[-1]
    acc, jrk, pot, cond = np.empty((n, 3)), np.empty((n, 3)), np.empty(n), np.empty(n)
    for s in range(len(off) - 1):
        a, b = off[s], off[s + 1]
        ids = np.arange(b - a, dtype=np.int64)
        r = oracle.force(4, eps2, ids, m[a:b], x[a:b], v[a:b], ids, x[a:b], v[a:b])
        acc[a:b], jrk[a:b], pot[a:b], cond[a:b] = r["acc"], r["jerk"], r["pot"], r["cond"][:, 0]
    return acc, jrk, pot, cond


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_batch_few_body(prec):
    torch = pytest.importorskip("torch")
    say("batch prec=%s" % PREC_NAME[prec])
    off, m, x, v = make_batch()
    eps2 = 0.0
    acc_r, jrk_r, pot_r, cond = oracle_batch(off, m, x, v, eps2)
    kappa = cond / np.linalg.norm(acc_r, axis=1)
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    n = int(off[-1])
    dm, dx, dv = T(m), T(x), T(v)
    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    jrk, pot = torch.empty_like(acc), torch.empty(n, dtype=torch.float64, device=dev)
    tol = 1e-13 if prec == nbx.NBX_FP64 else 1e-6
    with nbx.Context(order=4, precision=prec, nj_max=1, ni_max=1) as ctx:
        nbx.nbx_batch_setup(ctx.ctx, off)
        for tuned in (False, True):
            if tuned:
                lanes = nbx.nbx_batch_tune(ctx.ctx, None, dm, dx, dv, eps2, acc, jrk, pot)
                say("  tuned lanes per class %s" % list(lanes))
                assert all(l in (0, 1, 2, 4, 8, 16, 32, 64) for l in lanes)
            acc.zero_(), jrk.zero_(), pot.zero_()
            nbx.nbx_batch_force_dev(ctx.ctx, None, dm, dx, dv, eps2, acc, jrk, pot)
            nbx.nbx_sync(ctx.ctx, None)
            torch.cuda.synchronize()
            a_gpu = acc.cpu().numpy()
            e_acc = rel_err_vec(a_gpu, acc_r)
            e_cond = np.linalg.norm(a_gpu - acc_r, axis=1) / cond
            e_pot = np.abs(pot.cpu().numpy() - pot_r) / np.abs(pot_r)
            e_jrk = rel_err_vec(jrk.cpu().numpy(), jrk_r)
            worst = int(np.argmax(e_acc))
            say("  tuned=%s max rel acc %.2e (kappa %.1f there; kappa<=2: %.2e) acc/cond %.2e pot %.2e "
                "jerk median %.2e" % (tuned, e_acc.max(), kappa[worst], e_acc[kappa <= 2].max(), e_cond.max(),
                                      e_pot.max(), np.median(e_jrk)))
            if prec == nbx.NBX_FP64:
                assert e_acc.max() <= tol and e_pot.max() <= tol
            else:
                assert e_cond.max() <= 1e-6 and e_acc[kappa <= 2].max() <= tol and e_pot.max() <= tol
            assert np.median(e_jrk) <= 100 * tol


@pytest.mark.parametrize("prec", [nbx.NBX_FP64, nbx.NBX_MIXED])
def test_batch_edge_sizes_and_errors(prec):
    """Systems at the size limits (1, 2, 63, 64, 65, 127, 128 particles) in one batch, eps2 > 0;
    a lone particle feels nothing.  Sizes 0 and 129 and a bad first offset are argument errors."""
    torch = pytest.importorskip("torch")
    say("batch edge sizes prec=%s" % PREC_NAME[prec])
    sizes = [1, 2, 63, 64, 65, 127, 128, 1, 128]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    parts = [nbody_ics.plummer(n, seed=20000 + s) for s, n in enumerate(sizes)]
    m = np.concatenate([p[0] for p in parts])
    x = np.concatenate([p[1] for p in parts])
    v = np.concatenate([p[2] for p in parts])
    eps2 = 1e-4
    acc_r, jrk_r, pot_r, cond = oracle_batch(off, m, x, v, eps2)
    dev = torch.device("cuda:0")
    T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)
    n = int(off[-1])
    acc = torch.empty((n, 3), dtype=torch.float64, device=dev)
    jrk, pot = torch.empty_like(acc), torch.empty(n, dtype=torch.float64, device=dev)
    with nbx.Context(order=4, precision=prec, nj_max=1, ni_max=1) as ctx:
        for bad in ([0, 0, 3], [0, 3, 3 + 129], [1, 4]):
            with pytest.raises(nbx.NbxError) as e:
                nbx.nbx_batch_setup(ctx.ctx, np.array(bad, dtype=np.int32))
            assert e.value.code == nbx.NBX_ERR_ARG
        nbx.nbx_batch_setup(ctx.ctx, off)
        nbx.nbx_batch_force_dev(ctx.ctx, None, T(m), T(x), T(v), eps2, acc, jrk, pot)
        nbx.nbx_sync(ctx.ctx, None)
        torch.cuda.synchronize()
        a, p = acc.cpu().numpy(), pot.cpu().numpy()
    lone = off[:-1][np.array(sizes) == 1]
    assert np.all(a[lone] == 0.0) and np.all(p[lone] == 0.0)
    live = np.setdiff1d(np.arange(n), lone)
    e_cond = np.linalg.norm(a[live] - acc_r[live], axis=1) / cond[live]
    e_pot = np.abs(p[live] - pot_r[live]) / np.abs(pot_r[live])
    tol = 1e-13 if prec == nbx.NBX_FP64 else 1e-6
    say("  acc/cond %.2e pot %.2e" % (e_cond.max(), e_pot.max()))
    assert e_cond.max() <= tol and e_pot.max() <= tol
