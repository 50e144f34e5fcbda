"""Pins for the oracle's treatment of tight pairs (the HiGPUs-R scheme of Sec. 3: tight
groups are taken out of the N-body integration and advanced separately).

Against: the second derivatives of the softened potential at 40 digits (tidal
tensor); the Kepler closed form (drift, isolated binary); the exact invariants of
the two-body problem, and the Jacobi-type integral |v|^2/2 - M/|r| - r.T.r/2 that a
constant linear tidal field conserves; second-order convergence of the splitting;
a hierarchical triple integrated directly with small steps.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from test_oracle_force import _phi_mp, _tiny_system
from test_oracle_hermite import kepler_state


# ---- tidal tensor -----------------------------------------------------------------------

@pytest.mark.parametrize("seed", [7, 8])
def test_tidal_is_minus_hessian_of_potential(orc, seed):
    x, v, m = _tiny_system(seed)
    eps = 0.05
    T = orc.tidal(x, m, eps)
    mp.mp.dps = 40
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    ms = [mp.mpf(float(q)) for q in m]
    e = mp.mpf(eps)
    for i in range(len(m)):
        for a in range(3):
            for b in range(3):
                def F(u, w, i=i, a=a, b=b):
                    y = list(xs[i])
                    y[a] = y[a] + u
                    y[b] = y[b] + w
                    return _phi_mp(i, y, xs, ms, e)
                h = -mp.diff(F, (0, 0), (1, 1))
                assert abs(float(h) - T[i, a, b]) <= 1e-12 * np.abs(T[i]).max(), (i, a, b)


def test_tidal_symmetry_trace_and_ranges(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(200, 9)
    eps = 1e-2
    T = orc.tidal(s.x, s.m, eps)
    assert np.allclose(T, np.transpose(T, (0, 2, 1)), rtol=0, atol=1e-13 * np.abs(T).max())
    # trace = -3 eps^2 sum_j m_j / s^(5/2): zero for eps = 0 (a harmonic field)
    r2 = ((s.x[None, :, :] - s.x[:, None, :]) ** 2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    want = -3.0 * eps * eps * (s.m[None, :] / (r2 + eps * eps) ** 2.5).sum(1)
    np.testing.assert_allclose(np.trace(T, axis1=1, axis2=2), want, rtol=1e-9,
                               atol=1e-12 * np.abs(T).max())
    T0 = orc.tidal(s.x, s.m, 0.0, ilist=[3, 4], j0=0, j1=200)
    assert np.all(np.abs(np.trace(T0, axis1=1, axis2=2)) <= 1e-12 * np.abs(T0).max())
    lo = orc.tidal(s.x, s.m, eps, j0=0, j1=77)
    hi = orc.tidal(s.x, s.m, eps, j0=77, j1=200)
    np.testing.assert_allclose(lo + hi, T, rtol=0, atol=1e-12 * np.abs(T).max())


def _phi_rest_mp(y, xs, ms, eps, skip):
    """Softened potential at point y from every body not in `skip` (40-digit)."""
    tot = mp.mpf(0)
    for j in range(len(ms)):
        if j in skip:
            continue
        d2 = sum((y[c] - xs[j][c]) ** 2 for c in range(3))
        tot -= ms[j] / mp.sqrt(d2 + eps * eps)
    return tot


def test_tidal_at_points_is_minus_hessian_of_the_rest(orc):
    """The tensor at a pair's centre of mass from the rest of the system: the second
    derivatives of the potential of the bodies not left out, at 40 digits."""
    x, v, m = _tiny_system(11, n=6)
    eps = 0.05
    cm = (m[0] * x[0] + m[1] * x[1]) / (m[0] + m[1])
    pts = np.array([cm, [0.3, -0.2, 0.7], x[4]])
    excl = np.array([[0, 1], [-1, -1], [4, -1]])
    T = orc.tidal_points(x, m, eps, pts, excl)
    mp.mp.dps = 40
    xs = [[mp.mpf(float(c)) for c in row] for row in x]
    ms = [mp.mpf(float(q)) for q in m]
    e = mp.mpf(eps)
    for k in range(3):
        skip = {int(q) for q in excl[k] if q >= 0}
        p = [mp.mpf(float(c)) for c in pts[k]]
        for a in range(3):
            for b in range(3):
                def F(u, w, a=a, b=b, p=p, skip=skip):
                    y = list(p)
                    y[a] = y[a] + u
                    y[b] = y[b] + w
                    return _phi_rest_mp(y, xs, ms, e, skip)
                h = -mp.diff(F, (0, 0), (1, 1))
                assert abs(float(h) - T[k, a, b]) <= 1e-12 * np.abs(T[k]).max(), (k, a, b)
    # the bodies left out do not matter, wherever they are
    x2 = x.copy()
    x2[0] += 10.0
    x2[1] -= 3.0
    T2 = orc.tidal_points(x2, m, eps, pts[:1], excl[:1])
    assert np.array_equal(T2[0], T[0])


def _nearest_brute(x, rows, row_end, dt, dt_cap):
    """Plain loops: the least (dx dx + dy dy) + dz dz over every other body, the lowest
    index first among equals."""
    out_j, out_d = [], []
    for i in rows:
        best, bd = -1, math.inf
        if i < row_end and (dt is None or dt[i] <= dt_cap):
            for j in range(len(x)):
                if j == i:
                    continue
                dx = float(x[j][0]) - float(x[i][0])
                dy = float(x[j][1]) - float(x[i][1])
                dz = float(x[j][2]) - float(x[i][2])
                d = dx * dx + dy * dy + dz * dz
                if d < bd:
                    best, bd = j, d
        out_j.append(best)
        out_d.append(bd)
    return np.array(out_j), np.array(out_d)


def test_nearest_is_the_brute_force_scan(orc):
    rng = np.random.default_rng(5)
    n = 60
    x = rng.normal(size=(n, 3))
    x[7] = x[3]                           # coincident bodies: distance 0
    x[10] = [0.5, 0.25, 0.125]            # two bodies at exactly equal distance from 10
    x[20] = [0.5, 0.25, 0.125 + 2.0 ** -10]
    x[30] = [0.5, 0.25, 0.125 - 2.0 ** -10]
    x[41] = x[40] * (1.0 + 1e-15)         # a near tie far from the origin
    dt = rng.choice([2.0 ** -12, 2.0 ** -6], n)
    for rows, row_end, dtv, cap in ((np.arange(n), n, None, math.inf),
                                    (np.array([3, 7, 10, 40, 41, 59, 0]), 45, dt, 2.0 ** -10)):
        nn, r2 = orc.nearest(x, rows, row_end, dtv, cap)
        wj, wd = _nearest_brute(x.tolist(), rows.tolist(), row_end, dtv, cap)
        assert np.array_equal(nn, wj)
        assert np.array_equal(r2, wd)
    nn, r2 = orc.nearest(x, [3, 7, 10])
    assert nn.tolist() == [7, 3, 20] and r2[0] == 0.0 and r2[1] == 0.0
    assert orc.nearest(x[:1], [0])[0].tolist() == [-1]      # no other body


# ---- Kepler drift -----------------------------------------------------------------------

def _rel(m1, m2, a, e, t, M0=0.0):
    x, v = kepler_state(m1, m2, a, e, t, M0)
    return x[1] - x[0], v[1] - v[0]


@pytest.mark.parametrize("e", [0.0, 0.3, 0.9, 0.995])
@pytest.mark.parametrize("t", [0.01, 1.7, -2.3, 40.0])
def test_kepler_drift_matches_closed_form(orc, e, t):
    r0, v0 = _rel(0.3, 0.7, 1.3, e, 0.0, M0=0.4)
    r1, v1 = orc.kepler_drift(1.0, r0, v0, t)
    re, ve = _rel(0.3, 0.7, 1.3, e, t, M0=0.4)
    scale = 1.0 + abs(t)
    assert np.abs(r1 - re).max() <= 1e-12 * scale * 1.3
    assert np.abs(v1 - ve).max() <= 1e-12 * scale / (1.0 - e) ** 0.5 * 2.0


def test_kepler_drift_invariants_and_reversibility(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        r0 = rng.normal(size=3)
        v0 = rng.normal(size=3) * 0.4
        M = 2.0
        if np.dot(v0, v0) / 2 - M / np.linalg.norm(r0) >= 0:
            continue
        dt = rng.uniform(-5, 5)
        r1, v1 = orc.kepler_drift(M, r0, v0, dt)
        E0 = np.dot(v0, v0) / 2 - M / np.linalg.norm(r0)
        E1 = np.dot(v1, v1) / 2 - M / np.linalg.norm(r1)
        assert abs(E1 - E0) <= 1e-12 * abs(E0)
        np.testing.assert_allclose(np.cross(r1, v1), np.cross(r0, v0), rtol=0, atol=1e-12)
        r2, v2 = orc.kepler_drift(M, r1, v1, -dt)
        np.testing.assert_allclose(r2, r0, rtol=0, atol=1e-11)
        np.testing.assert_allclose(v2, v0, rtol=0, atol=1e-11)
        ra, va = orc.kepler_drift(M, r0, v0, 0.37 * dt)
        rb, vb = orc.kepler_drift(M, ra, va, 0.63 * dt)
        np.testing.assert_allclose(rb, r1, rtol=0, atol=1e-11)


def test_kepler_drift_refuses_unbound_pairs(orc):
    with pytest.raises(orc.OracleError):
        orc.kepler_drift(1.0, np.array([1.0, 0, 0]), np.array([0, 2.0, 0]), 0.1)


# ---- relative orbit in a tidal field ----------------------------------------------------

def test_group_advance_without_tide_is_kepler(orc):
    r0, v0 = _rel(0.5, 0.5, 1.0, 0.6, 0.0)
    Z = np.zeros((3, 3))
    r1, v1 = orc.group_advance(1.0, r0, v0, 7.5, 13, Z, Z)
    re, ve = _rel(0.5, 0.5, 1.0, 0.6, 7.5)
    np.testing.assert_allclose(r1, re, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v1, ve, rtol=0, atol=1e-12)


def _jacobi(M, r, v, T):
    return np.dot(v, v) / 2 - M / np.linalg.norm(r) - 0.5 * r @ T @ r


def test_group_advance_conserves_the_jacobi_integral_of_a_constant_tide(orc):
    # constant symmetric tidal field: |v|^2/2 - M/|r| - r.T.r/2 is an exact integral;
    # the kick-drift-kick splitting keeps it to O(h^2)
    rng = np.random.default_rng(5)
    A = rng.normal(size=(3, 3)) * 0.02
    T = A + A.T
    for e in (0.0, 0.5):
        r0, v0 = _rel(0.5, 0.5, 1.0, e, 0.0)
        J0 = _jacobi(1.0, r0, v0, T)
        errs = []
        for nsub in (128, 256):
            r1, v1 = orc.group_advance(1.0, r0, v0, 0.9 * 2 * math.pi, nsub, T, T)
            errs.append(abs(_jacobi(1.0, r1, v1, T) - J0) / abs(J0))
        assert errs[1] < 2e-4, errs
        assert 3.0 < errs[0] / errs[1] < 5.0, errs


def test_group_advance_is_second_order(orc):
    rng = np.random.default_rng(6)
    A = rng.normal(size=(3, 3)) * 0.05
    T0, T1 = A + A.T, (A + A.T) * 0.3 + np.eye(3) * 0.01
    r0, v0 = _rel(0.5, 0.5, 1.0, 0.4, 0.0)
    H = 0.9 * 2 * math.pi
    ref = orc.group_advance(1.0, r0, v0, H, 1 << 15, T0, T1)
    e = [np.abs(orc.group_advance(1.0, r0, v0, H, k, T0, T1)[0] - ref[0]).max()
         for k in (32, 64, 128)]
    assert 3.3 < e[0] / e[1] < 4.7 and 3.3 < e[1] / e[2] < 4.7, e


# ---- grouped block-step integration ------------------------------------------------------

def test_isolated_binary_grouped_is_the_closed_form(orc):
    x0, v0 = kepler_state(0.4, 0.6, 1e-2, 0.7, 0.0)
    vcm = np.array([0.3, -0.1, 0.2])
    v0 = v0 + vcm
    p = orc.Params(eps=1e-10)
    xo, vo, steps, g = orc.group_integrate(x0, v0, np.array([0.4, 0.6]), [(0, 1)], 0.5, p)
    xe, ve = kepler_state(0.4, 0.6, 1e-2, 0.7, 0.5)
    np.testing.assert_allclose(xo, xe + 0.5 * vcm, rtol=0, atol=1e-12)
    np.testing.assert_allclose(vo, ve + vcm, rtol=0, atol=5e-10)   # about 80 orbits


def _triple():
    # inner binary (0.3 + 0.2, a = 0.01, e = 0.5) and a third body 0.5 at distance 1
    xb, vb = kepler_state(0.3, 0.2, 0.01, 0.5, 0.0)
    M, m3, R = 0.5, 0.5, 1.0
    vorb = math.sqrt((M + m3) / R)
    x = np.zeros((3, 3))
    v = np.zeros((3, 3))
    x[:2] = xb + np.array([-m3 / (M + m3) * R, 0, 0])
    v[:2] = vb + np.array([0, -m3 / (M + m3) * vorb, 0])
    x[2] = np.array([M / (M + m3) * R, 0, 0])
    v[2] = np.array([0, M / (M + m3) * vorb, 0])
    return x, v, np.array([0.3, 0.2, 0.5])


def _elements(M, r, v):
    E = np.dot(v, v) / 2 - M / np.linalg.norm(r)
    a = -M / (2 * E)
    h = np.cross(r, v)
    e = math.sqrt(max(0.0, 1 + 2 * E * np.dot(h, h) / M ** 2))
    return a, e


def test_hierarchical_triple_against_direct_integration(orc):
    x, v, m = _triple()
    t_end = 0.5
    # direct: the inner binary resolved with small steps
    std, _, _ = orc.integrate(x, v, m, t_end, orc.Params(eps=1e-10, eta=0.005, dt_max=2.0 ** -6))
    xo, vo, steps, g = orc.group_integrate(x, v, m, [(0, 1)], t_end,
                                           orc.Params(eps=1e-10, dt_max=2.0 ** -6))
    # the outer orbit and the inner orbit's elements agree to the order of the
    # terms the grouping leaves out ((a/R)^2 ~ 1e-4 of the outer forces)
    assert np.abs(xo[2] - std.x[2]).max() < 1e-5
    ad, ed = _elements(0.5, std.x[1] - std.x[0], std.v[1] - std.v[0])
    ag, eg = _elements(0.5, xo[1] - xo[0], vo[1] - vo[0])
    assert abs(ag - ad) / ad < 1e-4 and abs(eg - ed) < 1e-3
    assert steps < 200


@pytest.mark.parametrize("a_hi", [1e-3, 3e-4])
def test_cluster_with_hard_binaries_conserves_the_scheme_energy(orc, a_hi):
    """N = 160 Plummer cluster with 16 hard binaries (a in [1e-4, a_hi], thermal e,
    eps = 1e-5): the grouped run takes a few hundred block steps (integrated
    directly, the same cluster takes ~8e5) and conserves its energy."""
    from paper_1411_5234_amd import inputs
    s = inputs.with_binaries(160, 10, frac_members=0.2, a_lo=1e-4, a_hi=a_hi, imf="equal")
    pairs = [(2 * k, 2 * k + 1) for k in range(16)]
    eps = 1e-5
    p = orc.Params(eps=eps)
    g0 = orc.group_startup(s.x, s.v, s.m, pairs, p)
    e0 = orc.group_energy(g0, s.m, eps)
    xo, vo, steps, g = orc.group_integrate(s.x, s.v, s.m, pairs, 0.125, p)
    e1 = orc.group_energy(g, s.m, eps)
    assert abs(e1 - e0) / abs(e0) < 1e-6, abs(e1 - e0) / abs(e0)
    assert np.all(g.tpair == 0.125) and steps < 400


def test_kepler_drift_invariants_at_high_eccentricity(orc):
    """e up to 1 - 1e-4, any phase and |dt| up to 20 periods/2pi: energy, angular
    momentum and the Laplace-Runge-Lenz vector are kept, and the mean anomaly
    advances by n dt."""
    rng = np.random.default_rng(0)
    for _ in range(400):
        e = 1.0 - 10.0 ** rng.uniform(-4, -0.3)
        r0, v0 = _rel(0.5, 0.5, 1.0, e, 0.0, M0=rng.uniform(0, 2 * math.pi))
        t = rng.uniform(-20, 20)
        r1, v1 = orc.kepler_drift(1.0, r0, v0, t)
        for (ra, va), (rb, vb) in [((r0, v0), (r1, v1))]:
            Ea = np.dot(va, va) / 2 - 1.0 / np.linalg.norm(ra)
            Eb = np.dot(vb, vb) / 2 - 1.0 / np.linalg.norm(rb)
            assert abs(Eb - Ea) < 1e-10
            ha, hb = np.cross(ra, va), np.cross(rb, vb)
            assert np.abs(hb - ha).max() < 1e-12
            la = np.cross(va, ha) - ra / np.linalg.norm(ra)
            lb = np.cross(vb, hb) - rb / np.linalg.norm(rb)
            assert np.abs(lb - la).max() < 1e-11

        def mean_anomaly(r, v):
            a = 1.0 / (2.0 / np.linalg.norm(r) - np.dot(v, v))
            ec, es = 1.0 - np.linalg.norm(r) / a, np.dot(r, v) / math.sqrt(a)
            return math.atan2(es, ec) - es
        d = (mean_anomaly(r1, v1) - mean_anomaly(r0, v0) - t) % (2 * math.pi)
        assert min(d, 2 * math.pi - d) < 1e-10
