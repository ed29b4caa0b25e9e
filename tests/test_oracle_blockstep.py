"""Pins of the oracle's block time-step Hermite integrator against facts fixed outside its code.

  * exactness: the corrector and the interpolated derivatives reproduce polynomial motion of the
    degree the Hermite interpolation is built for;
  * the time-step criteria on a circular orbit, where every derivative has a closed form;
  * the convergence order of the correctors with every step forced to the same size (dt^4, dt^6);
  * energy conservation, block-step invariants and synchronisation on a Plummer sphere.
"""

import math

import numpy as np
import pytest

import nbody_ics
from oracle import blockstep as bs

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _poly_motion(rng, deg, n):
    """x(t) = sum_k c_k t^k / k!; returns a function giving the q-th derivative at t."""
    c = rng.normal(0, 1, size=(deg + 1, n, 3))

    def deriv(q, t):
        t = np.asarray(t)[:, None]
        return sum(c[k] * t ** (k - q) / math.factorial(k - q) for k in range(q, deg + 1))

    return deriv


@pytest.mark.parametrize("order,deg", [(4, 4), (6, 6)])
def test_corrector_exact_on_polynomial_motion(order, deg):
    # the velocity update integrates an interpolant of degree 2 nd - 1 of the acceleration and the
    # position update one of the velocity: both exact when x(t) has degree <= 2 nd (nd = 2 or 3)
    rng = np.random.default_rng(60)
    n = 20
    D = _poly_motion(rng, deg, n)
    t0 = rng.uniform(-1, 1, n)
    dt = 2.0 ** rng.integers(-3, 0, n)
    t1 = t0 + dt
    args = [D(0, t0), D(1, t0), D(2, t0), D(3, t0), D(2, t1), D(3, t1)]
    kw = dict(s0=D(4, t0), s1=D(4, t1)) if order == 6 else {}
    x1, v1, d = bs.hermite_correct(order, dt, *args, **kw)
    np.testing.assert_allclose(v1, D(1, t1), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(x1, D(0, t1), rtol=1e-12, atol=1e-12)
    scale = np.abs(D(2, t1)).max()
    for k in d:  # rounding of the interpolant grows as dt^-k for the k-th derivative
        want = D(k + 2, t1) + np.zeros((n, 3))
        np.testing.assert_allclose(d[k], want, rtol=1e-9, atol=1e-11 * scale * 8.0**k)


def test_corrector_not_exact_beyond_its_degree():
    # one degree more breaks the 4th-order velocity update (guards against a test that passes
    # trivially, e.g. by returning the exact answer from elsewhere)
    rng = np.random.default_rng(61)
    D = _poly_motion(rng, 6, 10)
    t0, dt = np.zeros(10), np.full(10, 0.25)
    x1, v1, _ = bs.hermite_correct(4, dt, D(0, t0), D(1, t0), D(2, t0), D(3, t0), D(2, dt), D(3, dt))
    assert np.abs(v1 - D(1, dt)).max() > 1e-8


def test_criteria_on_circular_orbit():
    # circular motion with angular frequency w and radius d: |a^(k)| = d w^(k+2), so
    # Aarseth dt4 = sqrt(eta4) / w and the 6th-order dt6 = eta6 / w
    d, w, th = 0.8, 1.7, 0.4

    def der(k):
        c, s = math.cos(th + k * math.pi / 2), math.sin(th + k * math.pi / 2)
        return np.array([[d * w**k * c, d * w**k * s, 0.0]])

    a1, j1 = der(2), der(3)
    dd = {2: der(4), 3: der(5), 4: der(6), 5: der(7)}
    dt4 = bs.criterion(4, a1, j1, dd, 0.01, 0.1)[0]
    assert abs(dt4 - 0.1 / w) <= 1e-15
    dt46 = bs.criterion(6, a1, j1, dd, 0.01, 0.3)[0]
    assert abs(dt46 - 0.5 * (0.1 / w + 0.3 / w)) <= 1e-15


def test_quantise_rules():
    # halving to the criterion, doubling only on commensurate times, caps at dt_max / dt_min
    assert bs.quantise(0.01, 1 / 16, 0.5, 1 / 8, 2.0**-20) == (1 / 128, False)
    assert bs.quantise(1.0, 1 / 16, 0.5, 1 / 8, 2.0**-20) == (1 / 8, False)
    assert bs.quantise(1.0, 1 / 16, 0.5 + 1 / 16, 1 / 8, 2.0**-20) == (1 / 16, False)  # not commensurate
    assert bs.quantise(1.0, 1 / 8, 0.5, 1 / 8, 2.0**-20) == (1 / 8, False)  # at dt_max
    assert bs.quantise(1e-9, 1 / 16, 0.5, 1 / 8, 2.0**-10) == (2.0**-10, True)  # clamped
    dn, cl = bs.quantise(float("nan"), 1 / 16, 0.5, 1 / 8, 2.0**-20)
    assert dn == 1 / 16 and cl


def _binary(e=0.0):
    m = np.array([0.5, 0.5])
    x = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    v = np.array([[0, -0.5, 0], [0, 0.5, 0]])
    return m, x, v


@pytest.mark.parametrize("order,expect", [(4, 16.0), (6, 64.0)])
def test_fixed_step_convergence_order(order, expect):
    # every step forced to dt (dt_min = dt_max = dt): the orbit error falls as dt^order
    m, x, v = _binary()
    errs = []
    for k in (4, 5, 6):
        dt = 2.0**-k
        it = bs.BlockStep(order, m, x, v, 0.0, dt_max=dt, dt_min=dt).run(1.0)
        assert it.t == 1.0 and all(n == 2 for _, n in it.log) and len(it.log) == 2**k
        xe, _ = it.state()
        exact = 0.5 * np.array([math.cos(1.0), math.sin(1.0), 0.0])
        errs.append(np.abs(xe[1] - exact).max())
    for e1, e2 in zip(errs, errs[1:]):
        assert 0.6 * expect < e1 / e2 < 1.5 * expect, errs


@pytest.mark.parametrize("order", [4, 6])
def test_plummer_block_steps_invariants_and_energy(order):
    n, eps2, t_end = 256, 1e-4, 0.125
    src = nbody_ics.make_sources(n, seed=62, time_offsets=False)
    it = bs.BlockStep(order, src.m, src.x, src.v, eps2)
    e0 = sum(it.energy())
    it.run(t_end)
    assert it.t == t_end
    np.testing.assert_array_equal(it.t_i, t_end)  # every particle synchronised at t_end
    lv = np.log2(it.dt)
    assert np.all(lv == np.round(lv)) and np.all(it.dt <= 0.125)
    assert np.all(np.fmod(it.t_i, it.dt) == 0.0)
    assert it.clamped == 0
    ts = [t for t, _ in it.log]
    assert all(a < b for a, b in zip(ts, ts[1:]))
    n_act = np.array([k for _, k in it.log])
    assert n_act.min() >= 1 and n_act.max() <= n and len(set(n_act.tolist())) > 1  # really block steps
    de = abs(sum(it.energy()) - e0) / abs(e0)
    assert de < (1e-7 if order == 4 else 1e-9), de


def test_hermite8_corrector_exact_on_degree8_motion_only():
    # the 8th-order corrector integrates degree-7 interpolants (a, jerk, snap, crackle at both ends
    # for v; v, a, jerk, snap for x): v exact while a(t) has degree <= 7 (x degree <= 9), x exact
    # while v(t) has degree <= 7 (x degree <= 8); one degree more breaks each
    rng = np.random.default_rng(62)
    n = 20
    for deg, v_exact, x_exact in ((8, True, True), (9, True, False), (10, False, False)):
        D = _poly_motion(rng, deg, n)
        t0 = rng.uniform(-1, 1, n)
        dt = 2.0 ** rng.integers(-1, 1, n)
        t1 = t0 + dt
        x1, v1 = bs.hermite8_correct(dt, D(0, t0), D(1, t0), D(2, t0), D(3, t0), D(4, t0), D(5, t0),
                                     D(2, t1), D(3, t1), D(4, t1), D(5, t1))
        ev, ex = np.abs(v1 - D(1, t1)).max(), np.abs(x1 - D(0, t1)).max()
        assert (ev < 1e-12) == v_exact and (ev > 1e-11 or v_exact), (deg, ev)
        assert (ex < 1e-12) == x_exact and (ex > 1e-11 or x_exact), (deg, ex)


def _hermite8_orbit(nsteps, n_ec):
    # shared-step 8th-order Hermite on the circular equal-mass binary (d = 1, omega = 1) for one
    # period, forces from the oracle's order-8 mode, n_ec evaluate-correct passes per step
    import oracle

    m, ids = np.array([0.5, 0.5]), np.arange(2, dtype=np.int64)
    x, v = np.array([[-0.5, 0, 0], [0.5, 0, 0]]), np.array([[0, -0.5, 0], [0, 0.5, 0]])

    def forces(x, v, a, j):
        f = oracle.force8(0.0, ids, m, x, v, a, j, ids, x, v, a, j)
        return f["acc"], f["jerk"], f["snap"], f["crackle"]

    a, j, _, _ = forces(x, v, np.zeros((2, 3)), np.zeros((2, 3)))  # a, j need no a, j
    a, j, s, c = forces(x, v, a, j)  # snap and crackle with the exact a, j
    T, t = 2.0 * math.pi, 0.0
    dt = T / nsteps
    for _ in range(nsteps):
        xp, vp, ap = oracle.predict(8, t + dt, np.full(2, t), x, v, a, j, s, c)
        jp = oracle.predict_jerk(t + dt, np.full(2, t), j, s, c)
        d1 = forces(xp, vp, ap, jp)
        for _ in range(n_ec):
            x1, v1 = bs.hermite8_correct(np.full(2, dt), x, v, a, j, s, c, *d1)
            d1 = forces(x1, v1, d1[0], d1[1])
        x, v, (a, j, s, c) = x1, v1, d1
        t += dt
    return np.abs(x - np.array([[-0.5, 0, 0], [0.5, 0, 0]])).max()  # back at the start after a period


def test_hermite8_circular_orbit_eighth_order():
    # with two evaluate-correct passes per step the predictor's error (crackle-order Taylor terms)
    # is corrected away and the global error falls as dt^8 (2^8 = 256 per halving)
    errs = [_hermite8_orbit(nsteps, 2) for nsteps in (16, 32, 64)]
    assert errs[-1] < 1e-11
    for e1, e2 in zip(errs, errs[1:]):
        assert 180.0 < e1 / e2 < 330.0, errs
