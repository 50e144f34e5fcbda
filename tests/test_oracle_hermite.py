"""Pins for the oracle's Hermite-4 predictor/corrector, step criterion and integrator.

Against: polynomial motion built from roots/coefficients with numpy's polynomial
class (the predictor must be exact for cubic motion, the corrector for quintic
motion, i.e. a cubic acceleration); the Kepler two-body closed form (Kepler's
equation solved by Newton's method); 4th-order convergence of the global error;
Aarseth's criterion on a circular orbit, where it reduces to sqrt(eta)/omega.
"""
import math

import numpy as np
import pytest
from numpy.polynomial import Polynomial as P


def _poly_motion(rng, deg, t0):
    """Three random polynomials of degree `deg` (one per axis), built from roots."""
    polys = []
    for _ in range(3):
        roots = rng.uniform(-2, 2, deg)
        polys.append(P.fromroots(roots) * rng.uniform(-1.5, 1.5))
    def val(t, k=0):
        return np.array([p.deriv(k)(t) if k else p(t) for p in polys])
    return val


def test_predictor_is_exact_for_cubic_motion(orc):
    rng = np.random.default_rng(7)
    n = 6
    t_i = np.array([0.25, 0.5, 0.0, 0.125, 0.375, 0.75])
    t_next = 1.0
    motions = [_poly_motion(rng, 3, 0) for _ in range(n)]
    x = np.array([mo(t_i[k]) for k, mo in enumerate(motions)])
    v = np.array([mo(t_i[k], 1) for k, mo in enumerate(motions)])
    a = np.array([mo(t_i[k], 2) for k, mo in enumerate(motions)])
    jk = np.array([mo(t_i[k], 3) for k, mo in enumerate(motions)])
    xp, vp = orc.predict(x, v, a, jk, t_i, t_next)
    for k, mo in enumerate(motions):
        np.testing.assert_allclose(xp[k], mo(t_next), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(vp[k], mo(t_next, 1), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("h", [0.5, 2.0 ** -4, 2.0 ** -9])
def test_corrector_is_exact_for_quintic_motion(orc, h):
    rng = np.random.default_rng(int(1 / h))
    n = 4
    t0 = 0.0
    motions = [_poly_motion(rng, 5, t0) for _ in range(n)]
    x = np.array([mo(t0) for mo in motions])
    v = np.array([mo(t0, 1) for mo in motions])
    a = np.array([mo(t0, 2) for mo in motions])
    jk = np.array([mo(t0, 3) for mo in motions])
    st = orc.State(x.copy(), v.copy(), np.ones(n), a.copy(), jk.copy(), np.zeros(n), np.full(n, h))
    xp, vp = orc.predict(x, v, a, jk, st.t, h)
    a1 = np.array([mo(h, 2) for mo in motions])
    j1 = np.array([mo(h, 3) for mo in motions])
    il = np.arange(n, dtype=np.int64)
    orc.correct(st, il, h, xp, vp, a1, j1, eta=0.02, dt_max=1.0, dt_min=2.0 ** -40)
    for k, mo in enumerate(motions):
        scale_x = np.abs(mo(h)).max() + 1
        scale_v = np.abs(mo(h, 1)).max() + 1
        np.testing.assert_allclose(st.x[k], mo(h), rtol=0, atol=2e-13 * scale_x)
        np.testing.assert_allclose(st.v[k], mo(h, 1), rtol=0, atol=2e-13 * scale_v)
    assert np.all(st.t == h)
    np.testing.assert_array_equal(st.a, a1)
    np.testing.assert_array_equal(st.j, j1)


# ---- Kepler two-body closed form -------------------------------------------------

def kepler_state(m1, m2, a, e, t, M0=0.0):
    """Positions/velocities of both bodies (CoM at rest at origin) at time t."""
    mt = m1 + m2
    nmean = math.sqrt(mt / a ** 3)
    M = M0 + nmean * t
    E = M if e < 0.8 else math.pi
    for _ in range(100):
        E -= (E - e * math.sin(E) - M) / (1 - e * math.cos(E))
    b = a * math.sqrt(1 - e * e)
    r = np.array([a * (math.cos(E) - e), b * math.sin(E), 0.0])
    edot = nmean / (1 - e * math.cos(E))
    w = np.array([-a * math.sin(E) * edot, b * math.cos(E) * edot, 0.0])
    x = np.array([m2 / mt * r, -m1 / mt * r])
    v = np.array([m2 / mt * w, -m1 / mt * w])
    return x, v


def _run_kepler(orc, e, t_end, eta, dt_max, eta_s=0.01, m1=0.5, m2=0.5):
    x0, v0 = kepler_state(m1, m2, 1.0, e, 0.0)
    p = orc.Params(eps=1e-10, eta=eta, eta_s=eta_s, dt_max=dt_max)
    st, steps, _ = orc.integrate(x0, v0, np.array([m1, m2]), t_end, p)
    xe, ve = kepler_state(m1, m2, 1.0, e, t_end)
    return st, xe, ve, steps


@pytest.mark.parametrize("e,tol", [(0.0, 2e-5), (0.5, 1e-5), (0.9, 5e-5)])
def test_kepler_orbit_matches_closed_form(orc, e, tol):
    st, xe, ve, steps = _run_kepler(orc, e, 6.25, eta=0.005, dt_max=2.0 ** -3)
    err = np.abs(st.x - xe).max()
    assert err < tol, (e, err, steps)
    assert np.all(st.t == 6.25)


def test_fixed_step_global_error_is_fourth_order(orc):
    errs = []
    for k in (6, 7, 8):
        h = 2.0 ** -k
        # huge eta/eta_s: every body keeps dt = dt_max = h (a fixed shared step)
        st, xe, ve, steps = _run_kepler(orc, 0.5, 6.25, eta=1e12, dt_max=h, eta_s=1e12)
        assert steps == int(6.25 / h)
        errs.append(np.abs(st.x - xe).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 20.0 and 12.0 < r2 < 20.0, errs


def test_energy_error_scales_like_eta_squared(orc):
    # dt ~ sqrt(eta) and the error per orbit ~ dt^4, so |dE| ~ eta^2.
    res = []
    for eta in (0.04, 0.01):
        st, xe, ve, steps = _run_kepler(orc, 0.5, 6.25, eta=eta, dt_max=2.0 ** -3)
        E = orc.energy(st.x, st.v, np.array([0.5, 0.5]), 1e-10)[2]
        res.append(abs(E - (-0.125)) / 0.125)
    ratio = res[0] / res[1]
    assert 4.0 < ratio < 64.0, res   # nominal 16, widened for power-of-two quantisation


def test_aarseth_step_on_circular_orbit(orc):
    # circular, a = 1, m1 + m2 = 1: omega = 1, so Aarseth's criterion gives sqrt(eta)
    eta = 0.02
    x0, v0 = kepler_state(0.5, 0.5, 1.0, 0.0, 0.0)
    p = orc.Params(eps=1e-10, eta=eta, eta_s=0.01, dt_max=2.0 ** -3)
    st = orc.startup(x0, v0, np.array([0.5, 0.5]), p)
    assert np.all(st.dt == 2.0 ** -7)      # eta_s |a|/|j| = 0.01 -> 2^-7
    seen = []
    for _ in range(12):
        t_next, il = orc.select(st.t, st.dt)
        xp, vp = orc.predict(st.x, st.v, st.a, st.j, st.t, t_next)
        acc, jerk = orc.force(xp, vp, st.m, p.eps, il)
        dta = orc.correct(st, il, t_next, xp, vp, acc, jerk, p.eta, p.dt_max, p.dt_min, want_dta=True)
        seen.extend(dta)
    np.testing.assert_allclose(seen, math.sqrt(eta), rtol=2e-2)
    assert np.all(st.dt == 2.0 ** -3)      # climbed by doublings to the largest allowed 2^k <= 0.1414
