"""Pins for the oracle's power-of-two block time steps (Sec. 2 item 2).

Invariants checked at every block step of a small Plummer run: every step is a power
of two no larger than dt_max; every body's time is a multiple of its step; the
active block is exactly the set of bodies due at the block time (checked by a brute
scan, not by the oracle's own selection); block times increase; everything is
synchronised at t_end; energy is conserved to the integrator's accuracy.
"""
import math

import numpy as np
import pytest


def _is_pow2(x):
    m, e = math.frexp(x)
    return m == 0.5


def test_select_against_brute_scan(orc):
    rng = np.random.default_rng(3)
    n = 500
    dt = 2.0 ** -rng.integers(2, 9, n).astype(float)
    t = np.floor(rng.uniform(0, 1, n) / dt) * dt
    t_next, il = orc.select(t, dt)
    due = t + dt
    assert t_next == min(due)
    assert list(il) == [i for i in range(n) if due[i] == t_next]
    assert np.all(np.diff(il) > 0)


def test_block_step_invariants_over_a_run(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(64, 9)
    p = orc.Params(eps=1e-2, eta=0.02, eta_s=0.01, dt_max=2.0 ** -3)
    st = orc.startup(s.x, s.v, s.m, p)
    E0 = orc.energy(st.x, st.v, st.m, p.eps)[2]
    t_end = 0.5
    last = 0.0
    steps = 0
    while np.any(st.t < t_end):
        due = st.t + st.dt
        expect = np.flatnonzero(due == due.min())
        rec = orc.block_step(st, p)
        steps += 1
        assert rec.t_next > last
        last = rec.t_next
        np.testing.assert_array_equal(rec.ilist, expect)
        assert np.all(st.t[rec.ilist] == rec.t_next)
        for i in range(st.n):
            assert _is_pow2(st.dt[i]) and st.dt[i] <= p.dt_max
            assert math.fmod(st.t[i], st.dt[i]) == 0.0
    assert np.all(st.t == t_end)
    assert steps > 10
    E1 = orc.energy(st.x, st.v, st.m, p.eps)[2]
    assert abs(E1 - E0) / abs(E0) < 1e-5


def test_step_below_dt_min_is_an_error(orc):
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(32, 4)
    p = orc.Params(eps=1e-3, eta=0.02, eta_s=0.01, dt_max=2.0 ** -3, dt_min=2.0 ** -4)
    with pytest.raises(orc.OracleError):
        orc.integrate(s.x, s.v, s.m, 0.25, p)


def test_plummer_c1_energy_drift_small(orc):
    # N = 1024 Plummer, eps = 1e-3, eta = 0.02 to t = 1 (the small reference workload)
    from paper_1411_5234_amd import inputs
    s = inputs.plummer(1024, 1)
    p = orc.Params(eps=1e-3)
    E0 = orc.energy(s.x, s.v, s.m, p.eps)[2]
    st, steps, inter = orc.integrate(s.x, s.v, s.m, 1.0, p)
    E1 = orc.energy(st.x, st.v, st.m, p.eps)[2]
    assert abs(E1 - E0) / abs(E0) < 1e-6
    assert inter > 1024 * 1024 and steps > 100
