"""Checks of the seeded input generators (Plummer, IMFs, binaries, request streams)."""
import math

import numpy as np
import pytest

from paper_1411_5234_amd import inputs


def test_same_seed_same_bytes():
    a = inputs.plummer(1000, 5)
    b = inputs.plummer(1000, 5)
    assert a.x.tobytes() == b.x.tobytes() and a.v.tobytes() == b.v.tobytes()
    c = inputs.plummer(1000, 6)
    assert a.x.tobytes() != c.x.tobytes()


def test_plummer_virial_units(orc):
    s = inputs.plummer(4096, 1)
    assert s.m.sum() == pytest.approx(1.0)
    np.testing.assert_allclose((s.m[:, None] * s.x).sum(0), 0, atol=1e-15)
    np.testing.assert_allclose((s.m[:, None] * s.v).sum(0), 0, atol=1e-15)
    T, W, E = orc.energy(s.x, s.v, s.m, 0.0)
    assert E == pytest.approx(-0.25, abs=0.02)
    assert 2 * T / -W == pytest.approx(1.0, abs=0.06)
    # half-mass radius of the Henon-scaled Plummer model: 1.305 * 3 pi / 16
    r = np.sort(np.linalg.norm(s.x, axis=1))
    assert r[len(r) // 2] == pytest.approx(1.305 * 3 * math.pi / 16, rel=0.05)


def test_plummer_isotropy():
    s = inputs.plummer(20000, 2)
    for arr in (s.x, s.v):
        sq = (arr ** 2).mean(0)
        assert np.all(np.abs(sq / sq.mean() - 1) < 0.06)


def _loglog_slope(m, lo, hi):
    edges = np.logspace(np.log10(lo), np.log10(hi), 15)
    h, _ = np.histogram(m, edges)
    centers = np.sqrt(edges[1:] * edges[:-1])
    dens = h / np.diff(edges)
    ok = h > 50
    return np.polyfit(np.log(centers[ok]), np.log(dens[ok]), 1)[0]


def test_salpeter_slope_and_range():
    m = inputs.salpeter_masses(200000, 3)
    assert m.sum() == pytest.approx(1.0)
    assert m.max() / m.min() <= 100.0 + 1e-9
    raw = m / m.min()
    assert _loglog_slope(raw, 1.0, 100.0) == pytest.approx(-2.35, abs=0.08)


def test_kroupa_segments():
    raw = inputs._kroupa_raw(np.random.default_rng(1), 400000)
    assert raw.min() >= 0.08 and raw.max() <= 100.0
    assert _loglog_slope(raw[raw < 0.5], 0.08, 0.5) == pytest.approx(-1.3, abs=0.1)
    assert _loglog_slope(raw[raw > 0.5], 0.5, 100.0) == pytest.approx(-2.3, abs=0.1)
    assert inputs.kroupa_masses(1000, 2).sum() == pytest.approx(1.0)


def test_binaries_recover_orbital_elements():
    s = inputs.with_binaries(2000, 7)
    npairs = s.meta["n_pairs"]
    assert npairs == 100
    m1, m2 = s.m[0:2 * npairs:2], s.m[1:2 * npairs:2]
    r = s.x[0:2 * npairs:2] - s.x[1:2 * npairs:2]
    w = s.v[0:2 * npairs:2] - s.v[1:2 * npairs:2]
    mt = m1 + m2
    rn = np.linalg.norm(r, axis=1)
    eps_orb = 0.5 * (w ** 2).sum(1) - mt / rn           # specific orbital energy
    a = -mt / (2 * eps_orb)
    hvec = np.cross(r, w)
    e = np.sqrt(np.maximum(0, 1 + 2 * eps_orb * (hvec ** 2).sum(1) / mt ** 2))
    np.testing.assert_allclose(a, s.meta["a"], rtol=1e-9)
    np.testing.assert_allclose(e, s.meta["e"], rtol=1e-7, atol=1e-9)
    assert s.meta["a"].min() >= 1e-4 and s.meta["a"].max() <= 1e-2
    assert s.m.sum() == pytest.approx(1.0)


def test_request_stream_shape():
    reqs = inputs.request_stream(4096, 4, 256, 32768, rate=100.0, eps=1e-3, t_end=1.0)
    ns = np.array([r.n for r in reqs])
    assert ns.min() >= 256 and ns.max() <= 32768
    assert np.all(np.diff([r.arrival for r in reqs]) >= 0)
    # log-uniform: median near sqrt(256 * 32768)
    assert np.median(ns) == pytest.approx(math.sqrt(256 * 32768), rel=0.1)
    again = inputs.request_stream(4096, 4, 256, 32768, rate=100.0, eps=1e-3, t_end=1.0)
    assert [r.n for r in again] == list(ns)
    # the same requests at any arrival rate (closed batch vs Poisson replay)
    closed = inputs.request_stream(4096, 4, 256, 32768, rate=0.0, eps=1e-3, t_end=1.0)
    assert [r.n for r in closed] == list(ns) and all(r.arrival == 0.0 for r in closed)
