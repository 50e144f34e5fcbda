"""Pins for the oracle's acceleration and jerk (Eq. 1 with the softening of Eq. 2).

The oracle writes the pair terms out explicitly.  These tests check them against
things that do not restate that formula: the gradient of the softened potential
taken numerically at 40 digits (mpmath), the time derivative of that gradient
along straight-line motion (jerk), Newton's third law and the central character
of the pair force, and linearity of the sum over j.
"""
import math

import mpmath as mp
import numpy as np
import pytest


def _tiny_system(seed, n=5):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, 3))
    x[1] = x[0] + 0.03 * rng.normal(size=3)          # one close pair
    v = rng.normal(size=(n, 3))
    m = rng.uniform(0.2, 2.0, n)
    return x, v, m


def _phi_mp(i, y, xs, ms, eps):
    """Softened potential felt at point y from every body but i (40-digit)."""
    tot = mp.mpf(0)
    for j in range(len(ms)):
        if j == i:
            continue
        d2 = sum((y[c] - xs[j][c]) ** 2 for c in range(3))
        tot -= ms[j] / mp.sqrt(d2 + eps * eps)
    return tot


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_acc_is_minus_gradient_of_potential(orc, seed):
    x, v, m = _tiny_system(seed)
    eps = 0.05
    acc, _ = orc.force(x, v, m, eps)
    mp.mp.dps = 40
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    ms = [mp.mpf(float(q)) for q in m]
    e = mp.mpf(eps)
    for i in range(len(m)):
        for c in range(3):
            def f(u, i=i, c=c):
                y = list(xs[i])
                y[c] = y[c] + u
                return _phi_mp(i, y, xs, ms, e)
            g = -mp.diff(f, 0)
            assert abs(float(g) - acc[i, c]) <= 1e-13 * np.linalg.norm(acc[i]), (i, c)


@pytest.mark.parametrize("seed", [3, 4])
def test_jerk_is_time_derivative_of_acc(orc, seed):
    x, v, m = _tiny_system(seed)
    eps = 0.05
    _, jerk = orc.force(x, v, m, eps)
    mp.mp.dps = 40
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    vs = [[mp.mpf(float(c)) for c in row] for row in v]
    ms = [mp.mpf(float(q)) for q in m]
    e = mp.mpf(eps)
    for i in range(len(m)):
        for c in range(3):
            # F(t, u) = potential at body i's straight-line position shifted by u along c,
            # with every other body also on its straight line; jerk_c = -d2F/dt du.
            def F(t, u, i=i, c=c):
                moved = [[xs[k][d] + vs[k][d] * t for d in range(3)] for k in range(len(ms))]
                y = list(moved[i])
                y[c] = y[c] + u
                return _phi_mp(i, y, moved, ms, e)
            g = -mp.diff(F, (0, 0), (1, 1))
            assert abs(float(g) - jerk[i, c]) <= 1e-12 * np.linalg.norm(jerk[i]), (i, c)


def test_newton_third_law_and_central_forces(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(256, 11, masses=inputs.salpeter_masses(256, 12))
    acc, jerk = orc.force(s.x, s.v, s.m, 1e-3)
    ma = s.m[:, None] * acc
    mj = s.m[:, None] * jerk
    assert np.all(np.abs(ma.sum(0)) <= 1e-14 * np.abs(ma).sum())
    assert np.all(np.abs(mj.sum(0)) <= 1e-14 * np.abs(mj).sum())
    torque = np.cross(s.x, ma)
    assert np.all(np.abs(torque.sum(0)) <= 1e-14 * np.abs(torque).sum())


def test_sum_over_j_is_linear_in_the_j_range(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(300, 5)
    il = np.array([0, 7, 150, 299], dtype=np.int64)
    a, j = orc.force(s.x, s.v, s.m, 1e-2, il)
    a1, j1 = orc.force(s.x, s.v, s.m, 1e-2, il, 0, 123)
    a2, j2 = orc.force(s.x, s.v, s.m, 1e-2, il, 123, 300)
    np.testing.assert_allclose(a1 + a2, a, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(j1 + j2, j, rtol=1e-13, atol=1e-15)


def test_self_term_and_coincident_bodies(orc):
    x = np.array([[0.3, -0.2, 0.1]])
    v = np.array([[1.0, 2.0, 3.0]])
    a, j = orc.force(x, v, np.array([1.0]), 1e-3)
    assert np.all(a == 0.0) and np.all(j == 0.0)
    # two bodies at the same point with eps > 0 exert no force on each other
    x2 = np.array([[0.3, -0.2, 0.1], [0.3, -0.2, 0.1]])
    v2 = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0]])
    a, j = orc.force(x2, v2, np.array([1.0, 2.0]), 1e-3)
    assert np.all(a == 0.0) and np.all(j == 0.0)
    # with different velocities the jerk is the softened closed form at r = 0:
    # d/dt [m r (r^2 + eps^2)^(-3/2)] = m (v_j - v_i) / eps^3 there
    v2[1] = [-0.5, 0.0, 4.0]
    a, j = orc.force(x2, v2, np.array([1.0, 2.0]), 1e-3)
    assert np.all(a == 0.0)
    np.testing.assert_allclose(j[0], 2.0 * (v2[1] - v2[0]) / 1e-9, rtol=1e-14)
    np.testing.assert_allclose(j[1], 1.0 * (v2[0] - v2[1]) / 1e-9, rtol=1e-14)


def test_two_body_magnitude_scales_like_softened_inverse_square(orc):
    # Along a line, |a| at separation d is m d / (d^2 + eps^2)^(3/2); check the
    # scaling law rather than the expression: the ratio between two separations.
    eps = 0.1
    def amag(d):
        x = np.array([[0.0, 0, 0], [d, 0, 0]])
        a, _ = orc.force(x, np.zeros((2, 3)), np.array([1.0, 1.0]), eps, np.array([0]))
        return a[0, 0]
    # large separations: inverse square law
    assert amag(200.0) / amag(100.0) == pytest.approx(0.25, rel=1e-5)
    # deep inside the softening length the force is harmonic (linear in d)
    assert amag(2e-5) / amag(1e-5) == pytest.approx(2.0, rel=1e-6)
    # the maximum of d/(d^2+eps^2)^(3/2) sits at d = eps/sqrt(2)
    ds = np.linspace(0.05, 0.09, 401)
    vals = np.array([amag(d) for d in ds])
    assert abs(ds[np.argmax(vals)] - eps / math.sqrt(2)) < 2e-4


def test_bad_ranges_raise(orc):
    x = np.zeros((4, 3))
    x[:, 0] = np.arange(4)
    with pytest.raises(orc.OracleError):
        orc.force(x, np.zeros((4, 3)), np.ones(4), 0.1, np.array([0]), 0, 5)
    with pytest.raises(orc.OracleError):
        orc.force(x, np.zeros((4, 3)), np.ones(4), 0.1, np.array([7]))


def test_force_scale_bounds_and_special_cases(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(200, 31)
    a, j = orc.force(s.x, s.v, s.m, 1e-3)
    sa, sj = orc.force_scale(s.x, s.v, s.m, 1e-3)
    # triangle inequality, with equality only when all terms are parallel
    assert np.all(sa >= np.linalg.norm(a, axis=1) * (1 - 1e-14))
    assert np.all(sj >= np.linalg.norm(j, axis=1) * (1 - 1e-14))
    # additive over the j-range like the sums themselves
    sa1, sj1 = orc.force_scale(s.x, s.v, s.m, 1e-3, None, 0, 77)
    sa2, sj2 = orc.force_scale(s.x, s.v, s.m, 1e-3, None, 77, 200)
    np.testing.assert_allclose(sa1 + sa2, sa, rtol=1e-13)
    np.testing.assert_allclose(sj1 + sj2, sj, rtol=1e-13)
    # bodies on one ray from body 0, moving along it: every term is parallel
    x = np.zeros((5, 3))
    x[:, 0] = [0.0, 0.5, 1.0, 2.0, 3.5]
    v = np.zeros((5, 3))
    v[:, 0] = [0.0, 0.3, -0.2, 0.7, 0.1]
    m = np.array([1.0, 0.5, 2.0, 1.0, 3.0])
    a, j = orc.force(x, v, m, 1e-3, np.array([0]))
    sa, sj = orc.force_scale(x, v, m, 1e-3, np.array([0]))
    assert sa[0] == pytest.approx(np.linalg.norm(a[0]), rel=1e-14)
    # a single pair: the scale is the magnitude of its one term
    a, j = orc.force(x[:2], v[:2], m[:2], 1e-3, np.array([0]))
    sa, sj = orc.force_scale(x[:2], v[:2], m[:2], 1e-3, np.array([0]))
    assert sa[0] == pytest.approx(np.linalg.norm(a[0]), rel=1e-15)
    assert sj[0] == pytest.approx(np.linalg.norm(j[0]), rel=1e-15)
