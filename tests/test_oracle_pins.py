"""Pins of the FP64 oracle against facts that do not come from its own formulas.

Each test checks the oracle against something fixed independently of the code
under test: kinematics of an exact orbit, Newton's third law, the potential
whose gradient the acceleration must be, finite differences in time,
polynomial exactness of the Taylor predictor, brute-force nearest neighbours
from scipy, the known energy of the Plummer model and the convergence order of
the Hermite scheme.  A dropped term, a wrong sign, index or power in any output
fails at least one of them.
"""

import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import nbody_ics
import oracle

pytestmark = pytest.mark.usefixtures("oracle_lib")


def _all_pairs(order, eps2, m, x, v, a=None, ids=None, **kw):
    n = len(m)
    ids = np.arange(n, dtype=np.int64) if ids is None else ids
    return oracle.force(order, eps2, ids, m, x, v, ids, x, v, aj=a, ai=a, **kw)


# --------------------------------------------------------------------------------------------
# Two-body circular orbit: an exact solution of the softened two-body problem.  With separation
# d and softening eps2 the separation R = sqrt(d^2 + eps2) stays constant, the relative orbit
# r(t) = d (cos wt, sin wt, 0) has w^2 = M / R^3, and particle 1 sits at -(m2/M) r(t).  Its
# acceleration, jerk and snap are the 2nd, 3rd and 4th time derivatives of that position.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("eps2", [0.0, 1e-2, 0.3])
@pytest.mark.parametrize("m1,m2", [(0.5, 0.5), (0.9, 0.1), (1e-3, 2.0)])
def test_circular_binary_kinematics(eps2, m1, m2):
    d, M = 0.7, m1 + m2
    R = math.sqrt(d * d + eps2)
    w = math.sqrt(M / R**3)
    th = 0.37  # arbitrary phase

    def r_deriv(k):  # k-th time derivative of r(t) = d (cos wt, sin wt, 0) at phase th
        c, s = math.cos(th + k * math.pi / 2), math.sin(th + k * math.pi / 2)
        return d * w**k * np.array([c, s, 0.0])

    x = np.array([-(m2 / M) * r_deriv(0), (m1 / M) * r_deriv(0)])
    v = np.array([-(m2 / M) * r_deriv(1), (m1 / M) * r_deriv(1)])
    acc_true = np.array([-(m2 / M) * r_deriv(2), (m1 / M) * r_deriv(2)])
    jerk_true = np.array([-(m2 / M) * r_deriv(3), (m1 / M) * r_deriv(3)])
    snap_true = np.array([-(m2 / M) * r_deriv(4), (m1 / M) * r_deriv(4)])
    m = np.array([m1, m2])
    out = _all_pairs(6, eps2, m, x, v, a=acc_true)
    scale = np.abs(acc_true).max()
    np.testing.assert_allclose(out["acc"], acc_true, rtol=0, atol=1e-14 * scale)
    np.testing.assert_allclose(out["jerk"], jerk_true, rtol=0, atol=1e-14 * scale * w)
    np.testing.assert_allclose(out["snap"], snap_true, rtol=0, atol=1e-14 * scale * w * w)
    np.testing.assert_allclose(out["pot"], [-m2 / R, -m1 / R], rtol=1e-15)
    assert list(out["nn_id"]) == [1, 0]
    np.testing.assert_allclose(out["nn_r2"], [d * d, d * d], rtol=1e-15)
    out4 = _all_pairs(4, eps2, m, x, v)
    np.testing.assert_array_equal(out4["acc"], out["acc"])
    np.testing.assert_array_equal(out4["jerk"], out["jerk"])


# --------------------------------------------------------------------------------------------
# Newton's third law: the pair terms are antisymmetric, so the mass-weighted sums of acc, jerk
# and snap over a closed system vanish; the potential energy is symmetric.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("order", [4, 6])
def test_newton_third_law(order):
    src = nbody_ics.make_sources(96, seed=11, order=6, masses="salpeter")
    a = src.a
    out = _all_pairs(order, 1e-4, src.m, src.x, src.v, a=a if order == 6 else None)
    for key in ["acc", "jerk"] + (["snap"] if order == 6 else []):
        q = out[key]
        total = np.sum(src.m[:, None] * q, axis=0)
        scale = np.sum(src.m[:, None] * np.abs(q))
        assert np.all(np.abs(total) <= 1e-14 * scale), (key, total, scale)


def test_potential_energy_pair_symmetry():
    src = nbody_ics.make_sources(64, seed=12)
    out = _all_pairs(4, 1e-3, src.m, src.x, src.v)
    # W counted once per pair from row sums must equal the same from column order (reverse ids).
    rev = np.arange(63, -1, -1)
    out_r = _all_pairs(4, 1e-3, src.m[rev], src.x[rev], src.v[rev])
    w1 = 0.5 * np.sum(src.m * out["pot"])
    w2 = 0.5 * np.sum(src.m[rev] * out_r["pot"])
    assert abs(w1 - w2) <= 1e-15 * abs(w1)


# --------------------------------------------------------------------------------------------
# The acceleration is minus the gradient of the potential at the sink position.  A foreign sink
# (id not among the sources) is moved along each axis; central differences with Richardson
# extrapolation give the gradient to ~h^4.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("eps2", [1e-3, 0.05])
def test_acceleration_is_minus_grad_potential(eps2):
    src = nbody_ics.make_sources(40, seed=13, masses="salpeter")
    rng = np.random.default_rng(5)
    y = rng.normal(0, 0.4, size=(5, 3))
    vy = np.zeros_like(y)
    ids = np.arange(1000, 1005, dtype=np.int64)
    base = oracle.force(4, eps2, src.ids, src.m, src.x, src.v, ids, y, vy)
    h = 1e-3
    grad = np.zeros_like(y)
    for k in range(3):
        def pot_at(s):
            yy = y.copy()
            yy[:, k] += s
            return oracle.force(4, eps2, src.ids, src.m, src.x, src.v, ids, yy, vy)["pot"]
        grad[:, k] = (-pot_at(2 * h) + 8 * pot_at(h) - 8 * pot_at(-h) + pot_at(-2 * h)) / (12 * h)
    np.testing.assert_allclose(base["acc"], -grad, rtol=0, atol=2e-8 * np.abs(base["acc"]).max())


# --------------------------------------------------------------------------------------------
# Jerk is the time derivative of the acceleration when every particle moves on x + v t; snap is
# the derivative of the jerk when every particle moves on x + v t + a t^2/2 with velocity v + a t.
# --------------------------------------------------------------------------------------------
def _fd(f, h):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.mark.parametrize("eps2", [1e-2, 1e-1])
def test_jerk_is_time_derivative_of_acc(eps2):
    src = nbody_ics.make_sources(24, seed=14, masses="salpeter")
    out = _all_pairs(4, eps2, src.m, src.x, src.v)
    fd = _fd(lambda s: _all_pairs(4, eps2, src.m, src.x + src.v * s, src.v)["acc"], 4e-4)
    np.testing.assert_allclose(out["jerk"], fd, rtol=0, atol=1e-7 * np.abs(out["jerk"]).max())


@pytest.mark.parametrize("eps2", [1e-2, 1e-1])
def test_snap_is_time_derivative_of_jerk(eps2):
    src = nbody_ics.make_sources(24, seed=15, order=6, masses="salpeter")
    a = src.a
    out = _all_pairs(6, eps2, src.m, src.x, src.v, a=a)

    def jerk_at(s):
        return _all_pairs(6, eps2, src.m, src.x + src.v * s + 0.5 * a * s * s, src.v + a * s, a=a)["jerk"]

    fd = _fd(jerk_at, 4e-4)
    np.testing.assert_allclose(out["snap"], fd, rtol=0, atol=1e-7 * np.abs(out["snap"]).max())


# --------------------------------------------------------------------------------------------
# The Taylor predictor is exact for motion that is a polynomial of the predictor's degree
# (cubic for 4th order, quintic for 6th) and is the identity at dt = 0.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("order,deg", [(4, 3), (6, 5)])
def test_predictor_exact_on_polynomials(order, deg):
    rng = np.random.default_rng(6)
    n = 50
    c = rng.normal(0, 1, size=(deg + 1, n, 3))  # x(t) = sum_k c_k (t - tj)^k
    tj = rng.uniform(-1, 0, size=n)
    t = 0.25
    fact = [math.factorial(k) for k in range(6)]
    derivs = [c[k] * fact[k] if k <= deg else np.zeros((n, 3)) for k in range(6)]
    xp, vp, ap = oracle.predict(order, t, tj, derivs[0], derivs[1], derivs[2], derivs[3], derivs[4], derivs[5])
    dt = (t - tj)[:, None]
    x_true = sum(np.polynomial.polynomial.polyval(0, [0]) + c[k] * dt**k for k in range(deg + 1))
    v_true = sum(k * c[k] * dt ** (k - 1) for k in range(1, deg + 1))
    a_true = sum(k * (k - 1) * c[k] * dt ** (k - 2) for k in range(2, deg + 1))
    np.testing.assert_allclose(xp, x_true, rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(vp, v_true, rtol=1e-13, atol=1e-13)
    if order == 6:
        np.testing.assert_allclose(ap, a_true, rtol=1e-13, atol=1e-13)
    # identity at t = tj
    xp0, vp0, ap0 = oracle.predict(order, 0.0, np.zeros(n), *derivs)
    np.testing.assert_array_equal(xp0, derivs[0])
    np.testing.assert_array_equal(vp0, derivs[1])
    if order == 6:
        np.testing.assert_array_equal(ap0, derivs[2])


# --------------------------------------------------------------------------------------------
# Nearest neighbour and neighbour lists against scipy's brute-force distance matrix.
# --------------------------------------------------------------------------------------------
def test_nn_and_neighbour_lists_brute_force():
    src = nbody_ics.make_sources(300, seed=16)
    ids = src.ids * 7 + 3  # ids are not addresses
    h2 = np.full(300, 0.04)
    out = _all_pairs(4, 1e-4, src.m, src.x, src.v, ids=ids, h2=h2, nbr_max=300)
    d2 = cdist(src.x, src.x, "sqeuclidean")
    np.fill_diagonal(d2, np.inf)
    nn = np.argmin(d2, axis=1)
    np.testing.assert_array_equal(out["nn_id"], ids[nn])
    np.testing.assert_allclose(out["nn_r2"], d2[np.arange(300), nn], rtol=1e-14)
    for i in range(300):
        expect = set(ids[np.nonzero(d2[i] < h2[i])[0]])
        assert out["nbr_count"][i] == len(expect)
        assert set(out["nbr_ids"][i, : out["nbr_count"][i]]) == expect


def test_nn_ties_none_and_overflow():
    # sink at the origin, equidistant sources at +-x: the lower address wins the tie
    x = np.array([[0.0, 0, 0], [0.5, 0, 0], [-0.5, 0, 0], [0, 0, 2.0]])
    v = np.zeros_like(x)
    m = np.full(4, 0.25)
    ids = np.array([10, 20, 30, 40], dtype=np.int64)
    out = oracle.force(4, 0.0, ids, m, x, v, ids[:1], x[:1], v[:1], h2=[1.0], nbr_max=1)
    assert out["nn_id"][0] == 20 and out["nn_r2"][0] == 0.25
    assert out["nbr_count"][0] == 2 and out["nbr_ids"][0, 0] == 20  # exact count, first stored
    # a lone particle has no neighbour
    one = oracle.force(4, 0.0, ids[:1], m[:1], x[:1], v[:1], ids[:1], x[:1], v[:1])
    assert one["nn_id"][0] == -1 and np.isinf(one["nn_r2"][0])
    np.testing.assert_array_equal(one["acc"], 0.0)
    assert one["pot"][0] == 0.0


def test_self_excluded_by_id_not_by_position():
    # a sink whose id matches a source is not attracted by it even at another position;
    # a different id at the same position as a source is attracted (softened).
    xj = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    vj = np.zeros_like(xj)
    mj = np.array([1.0, 2.0])
    idj = np.array([0, 1], dtype=np.int64)
    xi = np.array([[0.5, 0, 0], [0.0, 0, 0]])
    vi = np.zeros_like(xi)
    idi = np.array([0, 99], dtype=np.int64)
    eps2 = 0.01
    out = oracle.force(4, eps2, idj, mj, xj, vj, idi, xi, vi)
    R0 = math.sqrt(0.25 + eps2)
    np.testing.assert_allclose(out["acc"][0], [2.0 * 0.5 / R0**3, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(out["pot"][0], -2.0 / R0, rtol=1e-15)
    R1 = math.sqrt(1.0 + eps2)
    np.testing.assert_allclose(out["acc"][1], [2.0 / R1**3, 0, 0], rtol=1e-15)
    np.testing.assert_allclose(out["pot"][1], -1.0 / math.sqrt(eps2) - 2.0 / R1, rtol=1e-15)


# --------------------------------------------------------------------------------------------
# Plummer model in standard units: total energy -1/4 and virial ratio K/|W| = 1/2 (sampling
# noise ~ N^-1/2).  Pins the normalisation and sign of the potential.
# --------------------------------------------------------------------------------------------
def test_plummer_energy_and_virial_ratio():
    n = 4096
    m, x, v = nbody_ics.plummer(n, seed=1)
    ids = np.arange(n, dtype=np.int64)
    out = oracle.force(4, 0.0, ids, m, x, v, ids, x, v)
    K = 0.5 * np.sum(m * np.sum(v * v, axis=1))
    W = 0.5 * np.sum(m * out["pot"])
    assert abs((K + W) + 0.25) < 0.02
    assert abs(K / abs(W) - 0.5) < 0.03


# --------------------------------------------------------------------------------------------
# Hermite corrector: a circular binary integrated with the oracle's predictor, forces and the
# 4th-order corrector follows the exact rotation, and the error falls as dt^4.
# --------------------------------------------------------------------------------------------
def _oracle_hermite(m, x, v, dt, nsteps, eps2):
    n = len(m)
    ids = np.arange(n, dtype=np.int64)
    f = oracle.force(4, eps2, ids, m, x, v, ids, x, v)
    a0, j0 = f["acc"], f["jerk"]
    t = 0.0
    for _ in range(nsteps):
        xp, vp, _ = oracle.predict(4, t + dt, np.full(n, t), x, v, a0, j0)
        f = oracle.force(4, eps2, ids, m, xp, vp, ids, xp, vp)
        x, v = oracle.hermite4_correct(dt, xp, vp, a0, j0, f["acc"], f["jerk"])
        f = oracle.force(4, eps2, ids, m, x, v, ids, x, v)
        a0, j0 = f["acc"], f["jerk"]
        t += dt
    return x, v


def test_hermite4_circular_orbit_fourth_order():
    m = np.array([0.5, 0.5])
    d = 1.0
    w = 1.0  # M / d^3 = 1
    x = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    v = np.array([[0, -0.5 * w, 0], [0, 0.5 * w, 0]])
    errs = []
    T = 1.0
    for nsteps in (16, 32, 64):
        xe, _ = _oracle_hermite(m, x, v, T / nsteps, nsteps, 0.0)
        exact = 0.5 * d * np.array([math.cos(w * T), math.sin(w * T), 0.0])
        errs.append(np.abs(xe[1] - exact).max())
    assert errs[-1] < 1e-8
    for e1, e2 in zip(errs, errs[1:]):
        assert 12.0 < e1 / e2 < 20.0, errs  # 2^4 = 16


def test_hermite4_config1_energy_drift_small():
    # 1024-body Plummer sphere, eps2 = 1e-4, 8 shared steps of dt = 1/256: energy drift is tiny.
    src = nbody_ics.make_sources(1024, seed=1, time_offsets=False)
    ids = src.ids
    e0_f = oracle.force(4, 1e-4, ids, src.m, src.x, src.v, ids, src.x, src.v)
    e0 = oracle.total_energy(src.m, src.v, e0_f["pot"])
    x, v = _oracle_hermite(src.m, src.x, src.v, 1.0 / 256, 8, 1e-4)
    e1 = oracle.total_energy(src.m, v, oracle.force(4, 1e-4, ids, src.m, x, v, ids, x, v)["pot"])
    assert abs((e1 - e0) / e0) < 1e-6


# --------------------------------------------------------------------------------------------
# Rounding: the long-double sums make the oracle agree with a 40-digit evaluation of the same
# definition to ~1e-15; results do not depend on the OpenMP thread count.
# --------------------------------------------------------------------------------------------
def test_oracle_rounding_against_high_precision():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    src = nbody_ics.make_sources(20, seed=17, order=6, masses="salpeter")
    eps2 = 1e-4
    out = _all_pairs(6, eps2, src.m, src.x, src.v, a=src.a)
    n = 20
    for i in (0, 7, 19):
        acc = [mpmath.mpf(0)] * 3
        pot = mpmath.mpf(0)
        for j in range(n):
            if j == i:
                continue
            r = [mpmath.mpf(src.x[j, k]) - mpmath.mpf(src.x[i, k]) for k in range(3)]
            R2 = sum(c * c for c in r) + mpmath.mpf(eps2)
            acc = [acc[k] + mpmath.mpf(src.m[j]) * r[k] / R2**1.5 for k in range(3)]
            pot -= mpmath.mpf(src.m[j]) / mpmath.sqrt(R2)
        ref = np.array([float(c) for c in acc])
        assert np.abs(out["acc"][i] - ref).max() <= 4e-16 * np.abs(ref).max() * 4
        assert abs(out["pot"][i] - float(pot)) <= 4e-16 * abs(float(pot))


def test_oracle_independent_of_thread_count():
    src = nbody_ics.make_sources(200, seed=18, order=6)
    r1 = _all_pairs(6, 1e-4, src.m, src.x, src.v, a=src.a, nthreads=1)
    r4 = _all_pairs(6, 1e-4, src.m, src.x, src.v, a=src.a, nthreads=4)
    for k in ("acc", "jerk", "snap", "pot", "nn_r2"):
        np.testing.assert_array_equal(r1[k], r4[k])


# --------------------------------------------------------------------------------------------
# 2nd-order (GRAPE-5, leapfrog) mode: acceleration and potential only, positions and masses are
# all the force needs (Background: the library supports the 2nd-order leapfrog).  Pinned by the
# exact circular orbit, Newton's third law, -grad of the potential, the 40-digit evaluation, the
# predictor's exactness on quadratics and the 2nd-order convergence of a leapfrog built on it.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("eps2", [0.0, 1e-2])
def test_order2_circular_binary_without_velocities(eps2):
    d, m1, m2 = 0.7, 0.9, 0.1
    M = m1 + m2
    R = math.sqrt(d * d + eps2)
    w2 = M / R**3
    th = 1.1
    r = d * np.array([math.cos(th), math.sin(th), 0.0])
    x = np.array([-(m2 / M) * r, (m1 / M) * r])
    acc_true = -w2 * x  # centripetal, towards the centre of mass at the origin
    ids = np.arange(2, dtype=np.int64)
    out = oracle.force(2, eps2, ids, np.array([m1, m2]), x, None, ids, x, None)
    assert out["jerk"] is None
    np.testing.assert_allclose(out["acc"], acc_true, rtol=0, atol=1e-14 * np.abs(acc_true).max())
    np.testing.assert_allclose(out["pot"], [-m2 / R, -m1 / R], rtol=1e-15)
    assert list(out["nn_id"]) == [1, 0]


def test_order2_newton_third_law_and_minus_grad_potential():
    src = nbody_ics.make_sources(96, seed=21, masses="salpeter")
    out = oracle.force(2, 1e-4, src.ids, src.m, src.x, None, src.ids, src.x, None)
    total = np.sum(src.m[:, None] * out["acc"], axis=0)
    assert np.all(np.abs(total) <= 1e-14 * np.sum(src.m[:, None] * np.abs(out["acc"])))
    rng = np.random.default_rng(22)
    y = rng.normal(0, 0.4, size=(4, 3))
    ids = np.arange(5000, 5004, dtype=np.int64)
    base = oracle.force(2, 0.02, src.ids, src.m, src.x, None, ids, y, None)
    grad = np.zeros_like(y)
    for k in range(3):
        def pot_at(s):
            yy = y.copy()
            yy[:, k] += s
            return oracle.force(2, 0.02, src.ids, src.m, src.x, None, ids, yy, None)["pot"]
        grad[:, k] = _fd(pot_at, 1e-3)
    np.testing.assert_allclose(base["acc"], -grad, rtol=0, atol=2e-8 * np.abs(base["acc"]).max())


def test_order2_rounding_against_high_precision():
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    src = nbody_ics.make_sources(24, seed=23, masses="salpeter")
    eps2 = 1e-5
    out = oracle.force(2, eps2, src.ids, src.m, src.x, None, src.ids, src.x, None)
    for i in (0, 11, 23):
        acc = [mpmath.mpf(0)] * 3
        pot = mpmath.mpf(0)
        for j in range(24):
            if j == i:
                continue
            r = [mpmath.mpf(src.x[j, k]) - mpmath.mpf(src.x[i, k]) for k in range(3)]
            R2 = sum(c * c for c in r) + mpmath.mpf(eps2)
            acc = [acc[k] + mpmath.mpf(src.m[j]) * r[k] / R2**1.5 for k in range(3)]
            pot -= mpmath.mpf(src.m[j]) / mpmath.sqrt(R2)
        ref = np.array([float(c) for c in acc])
        assert np.abs(out["acc"][i] - ref).max() <= 1.6e-15 * np.abs(ref).max()
        assert abs(out["pot"][i] - float(pot)) <= 4e-16 * abs(float(pot))


def test_order2_predictor_exact_on_quadratics_ignores_jerk():
    rng = np.random.default_rng(24)
    n = 40
    x0, v0, a0 = rng.normal(size=(3, n, 3))
    jerk = rng.normal(size=(n, 3))  # not part of the 2nd-order polynomial
    tj = rng.uniform(-1, 0, size=n)
    t = 0.3
    dt = (t - tj)[:, None]
    xp, vp, ap = oracle.predict(2, t, tj, x0, v0, a0, jerk)
    np.testing.assert_allclose(xp, x0 + v0 * dt + 0.5 * a0 * dt**2, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(vp, v0 + a0 * dt, rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(ap, a0)
    xq, vq, _ = oracle.predict(2, t, tj, x0, v0, a0, None)
    np.testing.assert_array_equal(xq, xp)
    np.testing.assert_array_equal(vq, vp)


def test_order2_leapfrog_circular_orbit_second_order():
    # kick-drift-kick leapfrog driven by the 2nd-order forces: error falls as dt^2
    m = np.array([0.5, 0.5])
    ids = np.arange(2, dtype=np.int64)
    x0 = np.array([[-0.5, 0, 0], [0.5, 0, 0]])
    v0 = np.array([[0, -0.5, 0], [0, 0.5, 0]])
    errs = []
    for nsteps in (32, 64, 128):
        dt = 1.0 / nsteps
        x, v = x0.copy(), v0.copy()
        a = oracle.force(2, 0.0, ids, m, x, None, ids, x, None)["acc"]
        for _ in range(nsteps):
            v = v + 0.5 * dt * a
            x = x + dt * v
            a = oracle.force(2, 0.0, ids, m, x, None, ids, x, None)["acc"]
            v = v + 0.5 * dt * a
        exact = 0.5 * np.array([math.cos(1.0), math.sin(1.0), 0.0])
        errs.append(np.abs(x[1] - exact).max())
    for e1, e2 in zip(errs, errs[1:]):
        assert 3.0 < e1 / e2 < 5.0, errs  # 2^2 = 4


# --------------------------------------------------------------------------------------------
# 8th-order mode (crackle, the third time derivative of the pair acceleration).
# --------------------------------------------------------------------------------------------
def _all_pairs8(eps2, m, x, v, a, j, **kw):
    ids = np.arange(len(m), dtype=np.int64)
    return oracle.force8(eps2, ids, m, x, v, a, j, ids, x, v, a, j, **kw)


@pytest.mark.parametrize("eps2", [0.0, 1e-2, 0.3])
@pytest.mark.parametrize("m1,m2", [(0.5, 0.5), (0.9, 0.1)])
def test_order8_circular_binary_kinematics(eps2, m1, m2):
    # same exact orbit as above: acc .. crackle are the 2nd .. 5th time derivatives of x(t)
    d, M = 0.7, m1 + m2
    R = math.sqrt(d * d + eps2)
    w = math.sqrt(M / R**3)
    th = 1.1

    def r_deriv(k):
        c, s = math.cos(th + k * math.pi / 2), math.sin(th + k * math.pi / 2)
        return d * w**k * np.array([c, s, 0.0])

    def body(k):
        return np.array([-(m2 / M) * r_deriv(k), (m1 / M) * r_deriv(k)])

    out = _all_pairs8(eps2, np.array([m1, m2]), body(0), body(1), body(2), body(3))
    scale = np.abs(body(2)).max()
    for key, k in (("acc", 2), ("jerk", 3), ("snap", 4), ("crackle", 5)):
        np.testing.assert_allclose(out[key], body(k), rtol=0, atol=1e-14 * scale * w ** (k - 2))
    np.testing.assert_allclose(out["pot"], [-m2 / R, -m1 / R], rtol=1e-15)
    assert out["cond"].shape == (2, 4)


@pytest.mark.parametrize("eps2", [1e-2, 1e-1])
def test_crackle_is_time_derivative_of_snap(eps2):
    # every particle moves on x + v t + a t^2/2 + j t^3/6 (velocity, acceleration and jerk
    # following); the snap along that motion has the crackle as its time derivative
    src = nbody_ics.make_sources(24, seed=16, order=6, masses="salpeter")
    rng = np.random.default_rng(17)
    a, j = src.a, rng.normal(0, 1, size=src.a.shape)
    out = _all_pairs8(eps2, src.m, src.x, src.v, a, j)

    def snap_at(s):
        return _all_pairs8(eps2, src.m, src.x + src.v * s + a * s * s / 2 + j * s**3 / 6,
                           src.v + a * s + j * s * s / 2, a + j * s, j)["snap"]

    fd = _fd(snap_at, 4e-4)
    np.testing.assert_allclose(out["crackle"], fd, rtol=0, atol=1e-7 * np.abs(out["crackle"]).max())
    # and the lower derivatives are those of the 6th-order path
    out6 = _all_pairs(6, eps2, src.m, src.x, src.v, a=a)
    for key in ("acc", "jerk", "snap", "pot", "nn_id", "nn_r2"):
        np.testing.assert_array_equal(out[key], out6[key])


def test_order8_newton_third_law():
    src = nbody_ics.make_sources(96, seed=18, order=6, masses="salpeter")
    j = np.random.default_rng(19).normal(0, 1, size=src.a.shape)
    out = _all_pairs8(1e-4, src.m, src.x, src.v, src.a, j)
    q = out["crackle"]
    total = np.sum(src.m[:, None] * q, axis=0)
    assert np.all(np.abs(total) <= 1e-14 * np.sum(src.m[:, None] * np.abs(q)))


def test_order8_predicted_jerk_exact_on_quintics():
    # x(t) quintic: the jerk x''' is quadratic, so jerk + snap dt + crackle dt^2/2 is exact
    rng = np.random.default_rng(20)
    n = 30
    c = rng.normal(0, 1, size=(6, n, 3))  # x(t) = sum_k c_k (t - tj)^k
    tj = rng.uniform(-1, 0, size=n)
    t = 0.3
    dt = (t - tj)[:, None]
    jerk, snap, crackle = 6 * c[3], 24 * c[4], 120 * c[5]
    exact = 6 * c[3] + 24 * c[4] * dt + 60 * c[5] * dt * dt
    np.testing.assert_allclose(oracle.predict_jerk(t, tj, jerk, snap, crackle), exact, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------------------------------------------
# Condition sums cond_k = sum_j |A_k(i, j)|, the denominators of the condition-normalised error
# bounds.  With one source per sink the sum has one term, so cond_k equals the magnitude of the
# exact k-th derivative of the circular orbit; with two sources placed symmetrically it is the
# sum of two known magnitudes while the signed sum partly cancels.
# --------------------------------------------------------------------------------------------
def _binary_derivs(m1, m2, eps2, d=0.7, th=0.37):
    M = m1 + m2
    R = math.sqrt(d * d + eps2)
    w = math.sqrt(M / R**3)

    def body(k):
        c, s = math.cos(th + k * math.pi / 2), math.sin(th + k * math.pi / 2)
        r = d * w**k * np.array([c, s, 0.0])
        return np.array([-(m2 / M) * r, (m1 / M) * r])

    return body, R, w


@pytest.mark.parametrize("eps2", [0.0, 1e-2, 0.3])
@pytest.mark.parametrize("m1,m2", [(0.5, 0.5), (0.9, 0.1), (1e-3, 2.0)])
def test_cond_single_pair_is_the_term_magnitude(eps2, m1, m2):
    body, _, _ = _binary_derivs(m1, m2, eps2)
    m = np.array([m1, m2])
    mag = lambda k: np.linalg.norm(body(k), axis=1)
    out6 = _all_pairs(6, eps2, m, body(0), body(1), a=body(2))
    np.testing.assert_allclose(out6["cond"][:, 0], mag(2), rtol=1e-14)
    np.testing.assert_allclose(out6["cond"][:, 1], mag(3), rtol=1e-14)
    np.testing.assert_allclose(out6["cond"][:, 2], mag(4), rtol=1e-13)
    out4 = _all_pairs(4, eps2, m, body(0), body(1))
    np.testing.assert_array_equal(out4["cond"][:, :2], out6["cond"][:, :2])
    assert np.all(out4["cond"][:, 2] == 0.0)
    out2 = oracle.force(2, eps2, np.arange(2), m, body(0), None, np.arange(2), body(0), None)
    np.testing.assert_array_equal(out2["cond"][:, 0], out6["cond"][:, 0])
    assert np.all(out2["cond"][:, 1:] == 0.0)
    out8 = _all_pairs8(eps2, m, body(0), body(1), body(2), body(3))
    for k in range(4):
        np.testing.assert_allclose(out8["cond"][:, k], mag(2 + k), rtol=1e-13)


@pytest.mark.parametrize("eps2", [0.0, 0.05])
def test_cond_three_body_sums_magnitudes(eps2):
    # a foreign sink at rest at the origin; sources of masses m1, m2 at (+d, 0, 0) and (-d, 0, 0)
    # moving with (0, +u, 0) and (0, -u, 0), no accelerations or jerks.  Then r.v = 0 for both
    # pairs (alpha = 0), beta = u^2/R^2 and gamma = 0, so with R^2 = d^2 + eps2:
    #   A0 = +-m d/R^3 x,  A1 = +-m u/R^3 y,  A2 = -3 (u/R)^2 A0,  A3 = -9 (u/R)^2 A1
    # and the signed sums carry (m1 - m2) where the condition sums carry (m1 + m2).
    d, u, m1, m2 = 0.3, 1.7, 0.8, 0.3
    R = math.sqrt(d * d + eps2)
    xs = np.array([[d, 0, 0], [-d, 0, 0]])
    vs = np.array([[0, u, 0], [0, -u, 0]])
    zs = np.zeros((2, 3))
    m = np.array([m1, m2])
    ids = np.array([0, 1], dtype=np.int64)
    sink = (np.array([7], dtype=np.int64), np.zeros((1, 3)), np.zeros((1, 3)))
    o6 = oracle.force(6, eps2, ids, m, xs, vs, *sink, aj=zs, ai=np.zeros((1, 3)))
    o8 = oracle.force8(eps2, ids, m, xs, vs, zs, zs, sink[0], sink[1], sink[2], np.zeros((1, 3)),
                       np.zeros((1, 3)))
    b = (u / R) ** 2
    signed = {"acc": (m1 - m2) * d / R**3 * np.array([1, 0, 0]),
              "jerk": (m1 - m2) * u / R**3 * np.array([0, 1, 0])}
    signed["snap"] = -3 * b * signed["acc"]
    signed["crackle"] = -9 * b * signed["jerk"]
    cond = [(m1 + m2) * d / R**3, (m1 + m2) * u / R**3, 3 * b * (m1 + m2) * d / R**3,
            9 * b * (m1 + m2) * u / R**3]
    for key in ("acc", "jerk", "snap"):
        np.testing.assert_allclose(o6[key][0], signed[key], rtol=1e-14, atol=1e-15 * np.abs(signed[key]).max())
    np.testing.assert_allclose(o8["crackle"][0], signed["crackle"], rtol=1e-14,
                               atol=1e-15 * np.abs(signed["crackle"]).max())
    np.testing.assert_allclose(o6["cond"][0], cond[:3], rtol=1e-14)
    np.testing.assert_allclose(o8["cond"][0], cond, rtol=1e-14)
    np.testing.assert_allclose(o6["pot"][0], -(m1 + m2) / R, rtol=1e-15)
    # the condition number of the acceleration is the known ratio
    assert abs(o6["cond"][0, 0] / np.linalg.norm(o6["acc"][0]) - (m1 + m2) / (m1 - m2)) < 1e-13


# --------------------------------------------------------------------------------------------
# Energy helpers against the closed-form energy of the circular softened binary,
# E = mu (w d)^2 / 2 - m1 m2 / R with mu = m1 m2 / M, and against an explicit pair sum.
# --------------------------------------------------------------------------------------------
@pytest.mark.parametrize("eps2", [0.0, 1e-2])
@pytest.mark.parametrize("m1,m2", [(0.5, 0.5), (0.9, 0.1)])
def test_total_energy_circular_binary(eps2, m1, m2):
    body, R, w = _binary_derivs(m1, m2, eps2)
    d = 0.7
    m = np.array([m1, m2])
    out = _all_pairs(4, eps2, m, body(0), body(1))
    e_kin = 0.5 * (m1 * m2 / (m1 + m2)) * (w * d) ** 2
    e_pot = -m1 * m2 / R
    assert abs(oracle.total_energy(m, body(1), out["pot"]) - (e_kin + e_pot)) <= 1e-15 * (e_kin - e_pot)
    # a cluster: kinetic sum plus the potential energy counted once per pair, written as a pair loop
    src = nbody_ics.make_sources(40, seed=19, masses="salpeter")
    eps = 1e-3
    o = _all_pairs(4, eps, src.m, src.x, src.v)
    w_pairs = 0.0
    for i in range(40):
        for j in range(i + 1, 40):
            w_pairs -= src.m[i] * src.m[j] / math.sqrt(np.sum((src.x[i] - src.x[j]) ** 2) + eps)
    k_sum = sum(0.5 * src.m[i] * float(np.dot(src.v[i], src.v[i])) for i in range(40))
    assert abs(oracle.total_energy(src.m, src.v, o["pot"]) - (k_sum + w_pairs)) <= 1e-14 * (k_sum - w_pairs)


@pytest.mark.parametrize("order", [4, 6])
def test_blockstep_energy_circular_binary(order):
    from oracle.blockstep import BlockStep

    m1, m2, eps2 = 0.9, 0.1, 1e-2
    body, R, w = _binary_derivs(m1, m2, eps2)
    d = 0.7
    e_kin = 0.5 * (m1 * m2 / (m1 + m2)) * (w * d) ** 2
    e_pot = -m1 * m2 / R
    bs = BlockStep(order, np.array([m1, m2]), body(0), body(1), eps2, dt_max=1.0 / 64)
    ek, ep = bs.energy()
    assert abs(ek - e_kin) <= 1e-15 * e_kin and abs(ep - e_pot) <= 1e-15 * abs(e_pot)
    # the orbit is circular, so the energy stays the closed form along the integrated motion
    bs.run(0.5)
    ek, ep = bs.energy()
    assert abs((ek + ep) - (e_kin + e_pot)) <= 1e-9 * abs(e_kin + e_pot)
    assert abs(ek - e_kin) <= 1e-7 * e_kin
