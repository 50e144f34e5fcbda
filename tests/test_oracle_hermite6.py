"""Pins for the oracle's 6th-order Hermite scheme (the order of the paper's HiGPUs,
Sec. 2 item 1): snap, predictor, corrector, interpolated crackle, step criterion.

Against: the second time derivative of the softened potential's gradient taken
numerically at 40 digits along quadratic paths (snap); polynomial motion built
from roots with numpy's polynomial class (the predictor must be exact for
quintic motion, the corrector and the interpolated crackle for a quartic
acceleration); the Kepler closed form; 6th-order convergence of the global
error; the step criterion on circular orbits, where it reduces to eta / omega.
"""
import math

import mpmath as mp
import numpy as np
import pytest
from numpy.polynomial import Polynomial as P

from test_oracle_force import _phi_mp, _tiny_system
from test_oracle_hermite import kepler_state


def _poly_motion(rng, deg):
    polys = []
    for _ in range(3):
        polys.append(P.fromroots(rng.uniform(-2, 2, deg)) * rng.uniform(-1.5, 1.5))

    def val(t, k=0):
        return np.array([p.deriv(k)(t) if k else p(t) for p in polys])
    return val


# ---- snap --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", [5, 6])
def test_snap_is_second_time_derivative_of_acc(orc, seed):
    x, v, m = _tiny_system(seed)
    b = np.random.default_rng(seed + 100).normal(size=x.shape)   # any accelerations
    eps = 0.05
    _, _, snap = orc.force6(x, v, b, m, eps)
    mp.mp.dps = 40
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    vs = [[mp.mpf(float(c)) for c in row] for row in v]
    bs = [[mp.mpf(float(c)) for c in row] for row in b]
    ms = [mp.mpf(float(q)) for q in m]
    e = mp.mpf(eps)
    for i in range(len(m)):
        for c in range(3):
            # every body on x + v t + b t^2 / 2; snap_c = -d3F / dt2 du
            def F(t, u, i=i, c=c):
                moved = [[xs[k][d] + vs[k][d] * t + bs[k][d] * t * t / 2 for d in range(3)]
                         for k in range(len(ms))]
                y = list(moved[i])
                y[c] = y[c] + u
                return _phi_mp(i, y, moved, ms, e)
            g = -mp.diff(F, (0, 0), (2, 1))
            assert abs(float(g) - snap[i, c]) <= 1e-11 * np.linalg.norm(snap[i]), (i, c)


def test_acc_and_jerk_agree_with_the_fourth_order_pass(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(200, 31)
    b = np.random.default_rng(2).normal(size=s.x.shape)
    a4, j4 = orc.force(s.x, s.v, s.m, 1e-3)
    a6, j6, _ = orc.force6(s.x, s.v, b, s.m, 1e-3)
    sa, sj = orc.force_scale(s.x, s.v, s.m, 1e-3)
    assert np.all(np.abs(a6 - a4).max(axis=1) <= 1e-14 * sa)
    assert np.all(np.abs(j6 - j4).max(axis=1) <= 1e-14 * sj)


def test_snap_third_law_and_j_linearity(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(300, 32, masses=inputs.salpeter_masses(300, 33))
    a, _ = orc.force(s.x, s.v, s.m, 1e-2)
    _, _, sn = orc.force6(s.x, s.v, a, s.m, 1e-2)
    tot = (s.m[:, None] * sn).sum(axis=0)
    scale = (s.m[:, None] * np.abs(sn)).sum(axis=0)
    assert np.all(np.abs(tot) <= 1e-12 * scale)
    lo = orc.force6(s.x, s.v, a, s.m, 1e-2, j0=0, j1=123)[2]
    hi = orc.force6(s.x, s.v, a, s.m, 1e-2, j0=123, j1=300)[2]
    np.testing.assert_allclose(lo + hi, sn, rtol=0, atol=1e-12 * np.abs(sn).max())


def test_snap_scale_pins(orc):
    from paper_1411_5234_amd import inputs
    # one pair: the scale is the length of the only term
    rng = np.random.default_rng(41)
    x, v, b = rng.normal(size=(2, 3)), rng.normal(size=(2, 3)), rng.normal(size=(2, 3))
    m = np.array([0.7, 1.3])
    _, _, sn = orc.force6(x, v, b, m, 0.1)
    ss = orc.force6_scale(x, v, b, m, 0.1)
    np.testing.assert_allclose(ss, np.linalg.norm(sn, axis=1), rtol=1e-14)
    # many bodies: at least the length of the sum, additive over j-ranges, linear in m_j
    s = inputs.plummer(200, 42)
    a, _ = orc.force(s.x, s.v, s.m, 1e-2)
    _, _, sn = orc.force6(s.x, s.v, a, s.m, 1e-2)
    ss = orc.force6_scale(s.x, s.v, a, s.m, 1e-2)
    assert np.all(ss >= np.linalg.norm(sn, axis=1) * (1 - 1e-14))
    part = (orc.force6_scale(s.x, s.v, a, s.m, 1e-2, j0=0, j1=77)
            + orc.force6_scale(s.x, s.v, a, s.m, 1e-2, j0=77, j1=200))
    np.testing.assert_allclose(part, ss, rtol=1e-13)
    np.testing.assert_allclose(orc.force6_scale(s.x, s.v, a, 3.0 * s.m, 1e-2), 3.0 * ss,
                               rtol=1e-13)


# ---- predictor and corrector on polynomial motion ------------------------------------

def test_predictor6_is_exact_for_quintic_motion(orc):
    rng = np.random.default_rng(17)
    t_i = np.array([0.25, 0.5, 0.0, 0.125, 0.375, 0.75])
    mot = [_poly_motion(rng, 5) for _ in t_i]
    st = [np.array([mo(t_i[k], d) for k, mo in enumerate(mot)]) for d in range(6)]
    xp, vp, ap = orc.predict6(*st, t_i, 1.0)
    for k, mo in enumerate(mot):
        for got, d in ((xp, 0), (vp, 1), (ap, 2)):
            np.testing.assert_allclose(got[k], mo(1.0, d), rtol=1e-13, atol=1e-13)


def _correct_poly(orc, deg, h, seed):
    rng = np.random.default_rng(seed)
    n = 4
    mot = [_poly_motion(rng, deg) for _ in range(n)]
    d0 = [np.array([mo(0.0, d) for mo in mot]) for d in range(6)]
    st = orc.State6(d0[0].copy(), d0[1].copy(), np.ones(n), d0[2].copy(), d0[3].copy(),
                    np.zeros(n), np.full(n, h), d0[4].copy(), d0[5].copy())
    a1, j1, s1 = (np.array([mo(h, d) for mo in mot]) for d in (2, 3, 4))
    orc.correct6(st, np.arange(n, dtype=np.int64), h, a1, j1, s1, eta=0.14, dt_max=1.0,
                 dt_min=2.0 ** -40)
    return st, mot


@pytest.mark.parametrize("h", [0.5, 2.0 ** -4, 2.0 ** -9])
def test_corrector6_is_exact_for_quartic_acceleration(orc, h):
    st, mot = _correct_poly(orc, 6, h, int(3 / h))
    for k, mo in enumerate(mot):
        for got, d in ((st.x, 0), (st.v, 1), (st.c, 5)):
            scale = np.abs(mo(h, d)).max() + 1
            np.testing.assert_allclose(got[k], mo(h, d), rtol=0, atol=5e-13 * scale / h ** (d // 5 * 3))
    assert np.all(st.t == h)


@pytest.mark.parametrize("h", [0.5, 2.0 ** -4])
def test_corrector6_velocity_and_crackle_exact_for_quintic_acceleration(orc, h):
    st, mot = _correct_poly(orc, 7, h, int(5 / h))
    for k, mo in enumerate(mot):
        np.testing.assert_allclose(st.v[k], mo(h, 1), rtol=0, atol=5e-13 * (np.abs(mo(h, 1)).max() + 1))
        np.testing.assert_allclose(st.c[k], mo(h, 5), rtol=0,
                                   atol=5e-13 * (np.abs(mo(h, 5)).max() + 1) / h ** 3)
    # the position quadrature integrates v, a quintic here: not exact for this motion
    worst = max(np.abs(st.x[k] - mo(h)).max() for k, mo in enumerate(mot))
    assert worst > 1e-11 * h ** 7


# ---- Kepler -------------------------------------------------------------------------

def _run_kepler6(orc, e, t_end, eta, dt_max, eta_s=0.01, a=1.0):
    x0, v0 = kepler_state(0.5, 0.5, a, e, 0.0)
    p = orc.Params6(eps=1e-10, eta=eta, eta_s=eta_s, dt_max=dt_max)
    st, steps, _ = orc.integrate6(x0, v0, np.array([0.5, 0.5]), t_end, p)
    xe, _ = kepler_state(0.5, 0.5, a, e, t_end)
    return st, xe, steps


@pytest.mark.parametrize("e,tol", [(0.0, 4e-7), (0.5, 1.5e-7), (0.9, 1e-6)])
def test_kepler6_matches_closed_form(orc, e, tol):
    st, xe, steps = _run_kepler6(orc, e, 6.25, eta=0.14, dt_max=2.0 ** -3)
    err = np.abs(st.x - xe).max()
    assert err < tol, (e, err, steps)
    assert np.all(st.t == 6.25)


def test_fixed_step_global_error_is_sixth_order(orc):
    errs = []
    for k in (3, 4, 5):
        h = 2.0 ** -k
        st, xe, steps = _run_kepler6(orc, 0.0, 6.25, eta=1e12, dt_max=h, eta_s=1e12)
        assert steps == int(6.25 / h)
        errs.append(np.abs(st.x - xe).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 48.0 < r1 < 80.0 and 48.0 < r2 < 80.0, errs


def test_error_scales_like_eta_to_the_sixth(orc):
    errs = []
    for eta in (0.14, 0.07):
        st, xe, _ = _run_kepler6(orc, 0.5, 6.25, eta=eta, dt_max=2.0 ** -3)
        errs.append(np.abs(st.x - xe).max())
    assert 32.0 < errs[0] / errs[1] < 128.0, errs


@pytest.mark.parametrize("a", [0.5, 2.0])
def test_generalized_step_on_circular_orbits(orc, a):
    # circular, m1 + m2 = 1: omega = a^-1.5 and every |d^k acc/dt^k| = |acc| omega^k,
    # so the criterion reduces to eta / omega.  The crackle comes from the step's
    # interpolant, extrapolated to its end: off by O(omega h), and by more on the
    # first steps, whose prediction had no crackle yet.
    eta = 0.14
    omega = a ** -1.5
    x0, v0 = kepler_state(0.5, 0.5, a, 0.0, 0.0)
    p = orc.Params6(eps=1e-10, eta=eta, eta_s=0.01, dt_max=2.0 ** -3)
    st = orc.startup6(x0, v0, np.array([0.5, 0.5]), p)
    # startup: eta_s / omega, the largest power of two not above it
    assert np.all(st.dt == 2.0 ** math.floor(math.log2(min(0.01 / omega, 2.0 ** -3))))
    seen = []
    for _ in range(12):
        t_next, il = orc.select(st.t, st.dt)
        xp, vp, ap = orc.predict6(st.x, st.v, st.a, st.j, st.s, st.c, st.t, t_next)
        acc, jerk, snap = orc.force6(xp, vp, ap, st.m, p.eps, il)
        seen.extend(orc.correct6(st, il, t_next, acc, jerk, snap, p.eta, p.dt_max, p.dt_min,
                                 want_dta=True))
    np.testing.assert_allclose(seen[4:], eta / omega, rtol=5e-2)
    want = 2.0 ** math.floor(math.log2(min(eta / omega, 2.0 ** -3)))
    assert np.all(st.dt == want)


# ---- block steps ---------------------------------------------------------------------

def test_block_steps6_invariants_and_energy(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(48, 9)
    p = orc.Params6(eps=1e-2)
    log = []
    st, steps, inter = orc.integrate6(s.x, s.v, s.m, 0.25, p, log=log)
    assert np.all(st.t == 0.25)
    assert inter == 2 * 48 * 48 + sum(il.size * 48 for _, il in log)
    ts = [t for t, _ in log]
    assert all(b > a for a, b in zip(ts, ts[1:]))
    e0 = orc.energy(s.x, s.v, s.m, 1e-2)[2]
    e1 = orc.energy(st.x, st.v, st.m, 1e-2)[2]
    assert abs(e1 - e0) / abs(e0) < 1e-6
    k = np.log2(st.dt)
    assert np.all(k == np.round(k))
    # at the default eta the 6th order does at most 1.25x the pair work of the 4th
    # order (eta = 0.02) for a smaller energy error (4x here)
    st4, _, inter4 = orc.integrate(s.x, s.v, s.m, 0.25, orc.Params(eps=1e-2))
    e4 = orc.energy(st4.x, st4.v, st4.m, 1e-2)[2]
    assert inter < 1.25 * inter4
    assert abs(e1 - e0) < 0.5 * abs(e4 - e0)


# ---- close encounters and force noise -------------------------------------------------

def _flyby(orc, sep, eta, dt_max, t_end=0.0625):
    """Two light bodies (1e-6) meeting head-on at relative speed 2 with impact
    parameter 1e-3 (eps = 1e-4), in the strong field of a unit mass at distance 1,
    which dominates their acceleration."""
    m = np.array([1.0, 1e-6, 1e-6])
    x = np.array([[0.0, 0.0, 0.0], [1.0, -sep / 2, 0.0], [1.0, sep / 2, 1e-3]])
    v = np.array([[0.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, -1.0, 0.0]])
    p = orc.Params6(eps=1e-4, eta=eta, dt_max=dt_max)
    st, steps, _ = orc.integrate6(x, v, m, t_end, p)
    return st, steps


@pytest.mark.parametrize("sep,tol", [(0.1, 1e-6), (0.01, 5e-9)])
def test_close_encounter_in_a_strong_field_is_resolved(orc, sep, tol):
    # reference: the same scheme converged (eta = 0.01, steps <= 2^-14); the
    # encounter deflects the pair's velocities by about 1e-3.  At sep = 0.1 the
    # encounter lies ahead and only the crackle announces it; at sep = 0.01 it is
    # under way at t = 0 and the startup step must see it through the snap.
    ref, _ = _flyby(orc, sep, 0.01, 2.0 ** -14)
    st, steps = _flyby(orc, sep, 0.14, 2.0 ** -3)
    err = np.abs(st.v[1:] - ref.v[1:]).max()
    assert err < tol, (err, steps)


def test_force_noise_does_not_shrink_a_small_shared_step(orc):
    """Every body on the smallest startup step (far below its orbital time scale)
    with FP32-sized errors (1e-7 of each sum's magnitude scale) added to the
    forces: the interpolated crackle is then mostly noise, and the step must hold."""
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(256, 5)
    p = orc.Params6(eps=1e-3)
    st = orc.startup6(s.x, s.v, s.m, p)
    h = st.dt.min()
    p.dt_max = h
    st.dt[:] = h
    rng = np.random.default_rng(1)
    for _ in range(8):
        t_next, il = orc.select(st.t, st.dt)
        xp, vp, ap = orc.predict6(st.x, st.v, st.a, st.j, st.s, st.c, st.t, t_next)
        acc, jerk, snap = orc.force6(xp, vp, ap, st.m, p.eps, il)
        sa, sj = orc.force_scale(xp, vp, st.m, p.eps, il)
        ss = orc.force6_scale(xp, vp, ap, st.m, p.eps, il)
        acc = acc + 1e-7 * sa[:, None] * rng.normal(size=acc.shape)
        jerk = jerk + 1e-7 * sj[:, None] * rng.normal(size=jerk.shape)
        snap = snap + 1e-7 * ss[:, None] * rng.normal(size=snap.shape)
        orc.correct6(st, il, t_next, acc, jerk, snap, p.eta, p.dt_max, p.dt_min)
    assert np.all(st.dt == h)
