"""Reverse-mode differentiation of the 4th-order force evaluation (torch.autograd).

``forces(x, v, m, eps2, ctx)`` returns (acc, jerk, pot) of a closed system (every particle a
sink and a source of all others) computed by the library's force kernels; its backward pass is
the library's adjoint kernel (``nbx_force_vjp_dev``).  ``hermite4`` integrates a system with the
4th-order Hermite predictor-evaluator-corrector scheme (Makino & Aarseth 1992, the integrator the
paper's Results section is built around) in torch operations, so gradients of a loss at the end of
a trajectory flow back to the initial positions, velocities and masses; with ``checkpoint=True``
each step keeps only its inputs and is recomputed during the backward pass.

The arithmetic of forces and gradients runs in the HIP library; torch provides device memory,
streams and the elementwise integrator algebra.
"""

from __future__ import annotations

import torch
import torch.utils.checkpoint

from . import nbx as _nbx


class ForceContext:
    """A library context sized for closed systems of up to n_max particles (4th order), with the
    gravity kernels that skip the nearest-neighbour search (the integrator never uses it)."""

    def __init__(self, n_max, precision=_nbx.NBX_FP64, device=0):
        self.n_max = n_max
        self.ctx = _nbx.Context(order=4, precision=precision, nj_max=n_max, ni_max=n_max, device=device,
                                want_nn=False)
        self._addr = torch.arange(n_max, dtype=torch.int32, device="cuda:%d" % device)
        self._ids = torch.arange(n_max, dtype=torch.int64, device="cuda:%d" % device)

    def close(self):
        self.ctx.close()


class _Forces(torch.autograd.Function):
    @staticmethod
    def forward(fctx, x, v, m, eps2, fc):
        n = x.shape[0]
        if n > fc.n_max:
            raise ValueError("system of %d particles exceeds the context's n_max=%d" % (n, fc.n_max))
        x, v, m = x.detach().contiguous(), v.detach().contiguous(), m.detach().contiguous()
        stream = torch.cuda.current_stream()
        zeros = torch.zeros_like(x)
        t = torch.zeros(n, dtype=torch.float64, device=x.device)
        c = fc.ctx.ctx
        _nbx.nbx_set_j_dev(c, stream, n, fc._addr[:n], fc._ids[:n], m, t, x, v, zeros, zeros)
        _nbx.nbx_set_nj(c, n)
        _nbx.nbx_predict(c, 0.0)
        acc = torch.empty_like(x)
        jerk = torch.empty_like(x)
        pot = torch.empty(n, dtype=torch.float64, device=x.device)
        _nbx.nbx_force_dev(c, stream, n, fc._addr[:n], eps2, None, acc, jerk, None, pot, None, None)
        fctx.save_for_backward(x, v, m)
        fctx.eps2 = eps2
        fctx.fc = fc
        return acc, jerk, pot

    @staticmethod
    def backward(fctx, g_acc, g_jerk, g_pot):
        x, v, m = fctx.saved_tensors
        n = x.shape[0]
        g_acc = torch.zeros_like(x) if g_acc is None else g_acc.contiguous()
        g_jerk = torch.zeros_like(x) if g_jerk is None else g_jerk.contiguous()
        g_pot = torch.zeros_like(m) if g_pot is None else g_pot.contiguous()
        gx, gv, gm = torch.empty_like(x), torch.empty_like(v), torch.empty_like(m)
        _nbx.nbx_force_vjp_dev(fctx.fc.ctx.ctx, torch.cuda.current_stream(), n, m, x, v, fctx.eps2, g_acc, g_jerk,
                               g_pot, gx, gv, gm)
        return gx, gv, gm, None, None


def forces(x, v, m, eps2, fc):
    """(acc, jerk, pot) of the closed system (x, v, m); differentiable in x, v and m."""
    return _Forces.apply(x, v, m, eps2, fc)


def _step(x, v, a0, j0, m, dt, eps2, fc):
    """One 4th-order Hermite step (predict, evaluate, correct); the force at the predicted point
    starts the next step."""
    xp = x + dt * v + (dt * dt / 2.0) * a0 + (dt ** 3 / 6.0) * j0
    vp = v + dt * a0 + (dt * dt / 2.0) * j0
    a1, j1, _ = forces(xp, vp, m, eps2, fc)
    a2 = (-6.0 * (a0 - a1) - dt * (4.0 * j0 + 2.0 * j1)) / (dt * dt)
    a3 = (12.0 * (a0 - a1) + 6.0 * dt * (j0 + j1)) / dt ** 3
    x1 = xp + (dt ** 4 / 24.0) * a2 + (dt ** 5 / 120.0) * a3
    v1 = vp + (dt ** 3 / 6.0) * a2 + (dt ** 4 / 24.0) * a3
    return x1, v1, a1, j1


def hermite4(x, v, m, eps2, dt, nsteps, fc, checkpoint=True):
    """Integrate nsteps shared 4th-order Hermite steps; returns (x, v) at the end.  With
    checkpoint=True only the inputs of each step are kept and the step is recomputed in backward."""
    a0, j0, _ = forces(x, v, m, eps2, fc)
    for _ in range(nsteps):
        if checkpoint:
            x, v, a0, j0 = torch.utils.checkpoint.checkpoint(_step, x, v, a0, j0, m, dt, eps2, fc,
                                                             use_reentrant=False)
        else:
            x, v, a0, j0 = _step(x, v, a0, j0, m, dt, eps2, fc)
    return x, v
