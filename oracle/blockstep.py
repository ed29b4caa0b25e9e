"""Block time-step Hermite integrator (4th and 6th order) on top of the oracle's predictor and forces.

TEST INFRASTRUCTURE ONLY -- nothing on the product path may import this.

The paper runs a 6th-order Hermite integrator with individual block time steps on top of the
library (Results > Block time-step simulations): Aarseth's criterion for 4th order, the average of
the Aarseth criterion and its 6th-order generalisation for 6th order, eta4 = 0.01, eta6 = 0.1.  The
paper prints none of the formulas; this module writes the method out from its definitions:

  * Hermite interpolation: on a step [t0, t0 + dt] the acceleration is the polynomial that matches
    a, a' (and a'' for 6th order) at both ends (degree 3 or 5).  It is found here by solving that
    linear system (numpy.linalg.solve) in the scaled variable u = (t - t0) / dt.
  * Corrector: the new velocity is v0 plus the integral of that interpolant over the step; the new
    position is x0 plus the integral of the interpolant of the velocity through v, v' = a (and
    v'' = jerk) at both ends, using the corrected v1.
  * Derivatives for the step criteria at the end of the step are those of the interpolant (the
    6th-order snap at the end is the computed one).
  * Criteria: Aarseth dt4 = sqrt(eta4 (|a||a2| + |a1|^2) / (|a1||a3| + |a2|^2)); 6th-order
    dt6 = eta6 ((|a||a2| + |a1|^2) / (|a3||a5| + |a4|^2))^(1/6); order 6 uses (dt4 + dt6) / 2.
  * Block steps: powers of two; halve until at most the criterion (not below dt_min), double at
    most once per step (not above dt_max) when the criterion allows twice the step and the new time
    is a multiple of the doubled step.  Start: eta_start |a|/|j| (order 6: at most
    eta_start sqrt(|a|/|s|)) rounded down to a power of two, crackle zero.
  * Each block step advances the particles whose t_i + dt_i is the smallest; every particle is
    predicted to that time (the oracle's Taylor predictor) and the active ones feel all of them.
  * Once a step has been clamped at dt_min the integration stops: the criterion has collapsed,
    which the paper reports for the 6th-order criterion when the forces carry too much rounding
    noise (Results > Block time-step simulations).
"""

from __future__ import annotations

import math

import numpy as np

from . import oracle as _o


def _basis(deg, u, k):
    """Row of d^k/du^k of (1, u, u^2, ..., u^deg) at u."""
    row = np.zeros(deg + 1)
    for m in range(k, deg + 1):
        row[m] = math.factorial(m) / math.factorial(m - k) * u ** (m - k)
    return row


def _interp_matrix(nd):
    """Conditions: derivatives 0..nd-1 at u = 0 and at u = 1 of a polynomial of degree 2 nd - 1."""
    deg = 2 * nd - 1
    rows = [_basis(deg, 0.0, k) for k in range(nd)] + [_basis(deg, 1.0, k) for k in range(nd)]
    return np.array(rows)


def interpolant(dt, left, right):
    """Scaled coefficients b (shape (deg+1, n, 3)) of p(u) = sum b_k u^k with p^(k)(0) = dt^k left[k]
    and p^(k)(1) = dt^k right[k]; the function of time is f(t0 + u dt) = p(u).
    left/right: lists of nd arrays [n, 3] (value, first derivative, ...); dt: [n]."""
    nd = len(left)
    M = _interp_matrix(nd)
    n = left[0].shape[0]
    rhs = np.zeros((2 * nd, n, 3))
    for k in range(nd):
        s = (dt ** k)[:, None]
        rhs[k] = left[k] * s
        rhs[nd + k] = right[k] * s
    b = np.linalg.solve(M, rhs.reshape(2 * nd, -1)).reshape(2 * nd, n, 3)
    return b


def integral(dt, b):
    """Integral over the step of the function whose scaled coefficients are b."""
    deg = b.shape[0] - 1
    return dt[:, None] * sum(b[k] / (k + 1) for k in range(deg + 1))


def derivative_at_end(dt, b, k):
    """k-th time derivative at the end of the step (u = 1)."""
    deg = b.shape[0] - 1
    acc = np.zeros_like(b[0])
    for m in range(k, deg + 1):
        acc = acc + b[m] * (math.factorial(m) / math.factorial(m - k))
    return acc / (dt ** k)[:, None]


def hermite_correct(order, dt, x0, v0, a0, j0, a1, j1, s0=None, s1=None):
    """Corrected (x1, v1) and the derivatives of the acceleration at the end of the step:
    returns x1, v1, d where d[k] is the k-th derivative (k = 2, 3 for order 4; 2..5 for order 6)."""
    dt = np.asarray(dt, dtype=np.float64)
    if order == 4:
        ba = interpolant(dt, [a0, j0], [a1, j1])
    else:
        ba = interpolant(dt, [a0, j0, s0], [a1, j1, s1])
    v1 = v0 + integral(dt, ba)
    if order == 4:
        bv = interpolant(dt, [v0, a0], [v1, a1])
    else:
        bv = interpolant(dt, [v0, a0, j0], [v1, a1, j1])
    x1 = x0 + integral(dt, bv)
    d = {k: derivative_at_end(dt, ba, k) for k in range(2, 4 if order == 4 else 6)}
    if order == 6:
        d[2] = np.array(s1, dtype=np.float64)  # the computed snap at the end of the step
    return x1, v1, d


def hermite8_correct(dt, x0, v0, a0, j0, s0, c0, a1, j1, s1, c1):
    """8th-order Hermite corrector for a shared step (Nitadori & Makino 2008, the integrator the
    paper's double-precision storage is meant to allow, Methods > Numerical Accuracy): the
    acceleration on the step is the degree-7 polynomial that matches a, jerk, snap and crackle at
    both ends; v1 = v0 plus its integral over the step; x1 = x0 plus the integral of the degree-7
    interpolant of the velocity through v, a, jerk and snap at both ends (with the corrected v1).
    dt: [n]; returns (x1, v1)."""
    dt = np.asarray(dt, dtype=np.float64)
    ba = interpolant(dt, [a0, j0, s0, c0], [a1, j1, s1, c1])
    v1 = v0 + integral(dt, ba)
    bv = interpolant(dt, [v0, a0, j0, s0], [v1, a1, j1, s1])
    x1 = x0 + integral(dt, bv)
    return x1, v1


def _norm(a):
    return np.sqrt(np.sum(np.asarray(a) ** 2, axis=1))


def criterion(order, a1, j1, d, eta4, eta6):
    """Time-step criterion at the end of a step from a, jerk and the higher derivatives d."""
    na, nj, n2, n3 = _norm(a1), _norm(j1), _norm(d[2]), _norm(d[3])
    num = na * n2 + nj * nj
    with np.errstate(divide="ignore", invalid="ignore"):
        dt4 = np.sqrt(eta4 * num / (nj * n3 + n2 * n2))
        if order == 4:
            return dt4
        n4, n5 = _norm(d[4]), _norm(d[5])
        dt6 = eta6 * (num / (n3 * n5 + n4 * n4)) ** (1.0 / 6.0)
    return 0.5 * (dt4 + dt6)


def quantise(crit, dt_old, t1, dt_max, dt_min):
    """Next power-of-two step of one particle; returns (dt_new, clamped)."""
    if not crit >= 0.0:
        return dt_old, True
    if crit < dt_old:
        dn = dt_old
        while dn > crit and dn > dt_min:
            dn /= 2.0
        return dn, dn > crit
    if crit >= 2.0 * dt_old and 2.0 * dt_old <= dt_max and math.fmod(t1, 2.0 * dt_old) == 0.0:
        return 2.0 * dt_old, False
    return dt_old, False


def first_step(order, a, j, s, eta_start, dt_max, dt_min):
    na, nj = _norm(a), _norm(j)
    with np.errstate(divide="ignore", invalid="ignore"):
        d0 = np.where(nj > 0, eta_start * na / np.where(nj > 0, nj, 1.0), dt_max)
        if order == 6:
            ns = _norm(s)
            d0 = np.where(ns > 0, np.minimum(d0, eta_start * np.sqrt(na / np.where(ns > 0, ns, 1.0))), d0)
    out = np.empty_like(d0)
    for i, d in enumerate(d0):
        dn = dt_max
        while dn > d and dn > dt_min:
            dn /= 2.0
        out[i] = dn
    return out


class BlockStep:
    """The integrator state: particles at their own times t_i with Taylor data for the predictor."""

    def __init__(self, order, m, x, v, eps2, eta4=0.01, eta6=0.1, eta_start=0.01, dt_max=0.125,
                 dt_min=2.0**-30, ids=None):
        if order not in (4, 6):
            raise ValueError("order must be 4 or 6")
        self.order, self.eps2 = order, float(eps2)
        self.eta4, self.eta6, self.eta_start = eta4, eta6, eta_start
        self.dt_max, self.dt_min = dt_max, dt_min
        n = len(m)
        self.n = n
        self.ids = np.arange(n, dtype=np.int64) if ids is None else np.asarray(ids, dtype=np.int64)
        self.m = np.array(m, dtype=np.float64)
        self.x = np.array(x, dtype=np.float64)
        self.v = np.array(v, dtype=np.float64)
        self.t_i = np.zeros(n)
        self.t = 0.0
        self.clamped = 0
        self.log = []  # (block time, N_active) per block step
        f = _o.force(4, self.eps2, self.ids, self.m, self.x, self.v, self.ids, self.x, self.v)
        self.a, self.j = f["acc"], f["jerk"]
        self.s = np.zeros((n, 3))
        self.c = np.zeros((n, 3))
        if order == 6:
            f6 = _o.force(6, self.eps2, self.ids, self.m, self.x, self.v, self.ids, self.x, self.v,
                          aj=self.a, ai=self.a)
            self.s = f6["snap"]
        self.dt = first_step(order, self.a, self.j, self.s, eta_start, dt_max, dt_min)

    def step(self, t_end):
        """One block step if due by t_end; returns N_active (0: none, or stopped after a clamp)."""
        if self.clamped:
            return 0
        tn_all = self.t_i + self.dt
        tn = tn_all.min()
        if not tn <= t_end:
            return 0
        act = np.nonzero(tn_all == tn)[0]
        o = self.order
        xp, vp, ap = _o.predict(o, tn, self.t_i, self.x, self.v, self.a, self.j,
                                self.s if o == 6 else None, self.c if o == 6 else None)
        f = _o.force(o, self.eps2, self.ids, self.m, xp, vp, self.ids[act], xp[act], vp[act],
                     aj=ap if o == 6 else None, ai=ap[act] if o == 6 else None)
        dt = self.dt[act]
        a1, j1 = f["acc"], f["jerk"]
        s1 = f["snap"] if o == 6 else None
        x1, v1, d = hermite_correct(o, dt, self.x[act], self.v[act], self.a[act], self.j[act], a1, j1,
                                    self.s[act] if o == 6 else None, s1)
        crit = criterion(o, a1, j1, d, self.eta4, self.eta6)
        for k, i in enumerate(act):
            dn, cl = quantise(crit[k], dt[k], tn, self.dt_max, self.dt_min)
            self.dt[i] = dn
            self.clamped += int(cl)
        self.x[act], self.v[act], self.a[act], self.j[act] = x1, v1, a1, j1
        if o == 6:
            self.s[act] = s1
            self.c[act] = d[3]
        self.t_i[act] = tn
        self.t = tn
        self.log.append((tn, len(act)))
        return len(act)

    def run(self, t_end):
        while self.step(t_end):
            pass
        return self

    def state(self):
        """Positions and velocities predicted to the current block time."""
        xp, vp, _ = _o.predict(self.order, self.t, self.t_i, self.x, self.v, self.a, self.j,
                               self.s if self.order == 6 else None, self.c if self.order == 6 else None)
        return xp, vp

    def energy(self):
        xp, vp = self.state()
        f = _o.force(4, self.eps2, self.ids, self.m, xp, vp, self.ids, xp, vp)
        ek = 0.5 * np.sum(self.m * np.sum(vp * vp, axis=1))
        ep = 0.5 * np.sum(self.m * f["pot"])
        return float(ek), float(ep)
