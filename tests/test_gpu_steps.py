"""GPU parity of the block-step kernels against the oracle.

Selection must be bit-exact (integer work on exact dyadic times); the predictor and
corrector are FP64 and must agree to rounding; the power-of-two steps decided by
the corrector and the startup rule are compared exactly; the energy is FP64 with
compensated sums.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import device_system
from paper_1411_5234_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


def _set_rows(sys, **rows):
    for k, v in rows.items():
        sys.row(k).copy_(torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64))


@pytest.mark.parametrize("n,seed", [(1, 0), (255, 1), (4096, 2), (100003, 3), (1 << 20, 4)])
def test_select_matches_oracle_exactly(ctx, orc, n, seed):
    rng = np.random.default_rng(seed)
    dt = 2.0 ** -rng.integers(3, 12, n).astype(float)
    t = np.floor(rng.uniform(0, 0.5, n) / dt) * dt
    sys = device_system(np.zeros((n, 3)), np.zeros((n, 3)), np.ones(n))
    _set_rows(sys, t=t, dt=dt)
    idx = torch.zeros(n, dtype=torch.int32, device="cuda")
    tn, m = ctx.select_active(sys, idx)
    otn, oil = orc.select(t, dt)
    assert tn == otn and m == oil.size
    np.testing.assert_array_equal(idx[:m].cpu().numpy(), oil)


def test_select_all_due_and_empty(ctx):
    n = 5000
    sys = device_system(np.zeros((n, 3)), np.zeros((n, 3)), np.ones(n))
    _set_rows(sys, t=np.zeros(n), dt=np.full(n, 0.125))
    idx = torch.zeros(n, dtype=torch.int32, device="cuda")
    tn, m = ctx.select_active(sys, idx)
    assert tn == 0.125 and m == n
    np.testing.assert_array_equal(idx.cpu().numpy(), np.arange(n))
    empty = device_system(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0))
    tn, m = ctx.select_active(empty, idx)
    assert m == 0


def _random_state(n, seed):
    rng = np.random.default_rng(seed)
    s = inputs.plummer(n, seed)
    a = rng.normal(size=(n, 3))
    jk = rng.normal(size=(n, 3)) * 10
    dt = 2.0 ** -rng.integers(3, 10, n).astype(float)
    t = np.floor(rng.uniform(0, 0.5, n) / dt) * dt
    return s, a, jk, t, dt


def test_predict_matches_oracle(ctx, orc):
    n = 70001
    s, a, jk, t, dt = _random_state(n, 5)
    sys = device_system(s.x, s.v, s.m)
    _set_rows(sys, ax=a[:, 0], ay=a[:, 1], az=a[:, 2], jx=jk[:, 0], jy=jk[:, 1], jz=jk[:, 2], t=t, dt=dt)
    t_next = 0.5
    ctx.predict(sys, t_next)
    ctx.sync()
    st = sys.state_numpy()
    xp, vp = orc.predict(s.x, s.v, a, jk, t, t_next)
    np.testing.assert_allclose(st["xp"], xp, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(st["vp"], vp, rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(sys.row("vxp32").cpu().numpy(), st["vp"][:, 0].astype(np.float32))
    np.testing.assert_array_equal(sys.row("m32").cpu().numpy(), s.m.astype(np.float32))


def test_startup_steps_match_oracle(ctx, orc):
    s = inputs.plummer(3000, 6)
    sys = device_system(s.x, s.v, s.m)
    acc = torch.empty(3 * s.n, dtype=torch.float64, device="cuda")
    jerk = torch.empty_like(acc)
    ctx.force_active(sys, None, s.n, 0, s.n, 1e-3, "fp64", acc, jerk)
    ctx.init_steps(sys, acc, jerk, 0.01, 2.0 ** -3, 2.0 ** -40)
    ctx.sync()
    st = sys.state_numpy()
    odt = orc.init_dt(st["a"], st["j"], 0.01, 2.0 ** -3, 2.0 ** -40)
    np.testing.assert_array_equal(st["dt"], odt)
    assert np.all(st["t"] == 0.0)
    np.testing.assert_array_equal(st["a"], acc.view(3, -1).T.cpu().numpy())


def test_correct_matches_oracle(ctx, orc):
    # one real block step of a Plummer sphere: both sides correct the same inputs
    s = inputs.plummer(2048, 7)
    p = orc.Params(eps=1e-3)
    ost = orc.startup(s.x, s.v, s.m, p)
    t_next, il = orc.select(ost.t, ost.dt)
    xp, vp = orc.predict(ost.x, ost.v, ost.a, ost.j, ost.t, t_next)
    acc, jerk = orc.force(xp, vp, ost.m, p.eps, il)
    sys = device_system(ost.x, ost.v, ost.m)
    _set_rows(sys, ax=ost.a[:, 0], ay=ost.a[:, 1], az=ost.a[:, 2], jx=ost.j[:, 0], jy=ost.j[:, 1],
              jz=ost.j[:, 2], t=ost.t, dt=ost.dt, xp=xp[:, 0], yp=xp[:, 1], zp=xp[:, 2],
              vxp=vp[:, 0], vyp=vp[:, 1], vzp=vp[:, 2])
    m = il.size
    idx = torch.as_tensor(il.astype(np.int32), device="cuda")
    gacc = torch.as_tensor(np.ascontiguousarray(acc.T).ravel(), device="cuda")
    gjerk = torch.as_tensor(np.ascontiguousarray(jerk.T).ravel(), device="cuda")
    ctx.correct(sys, idx, m, gacc, gjerk, t_next, p.eta, p.dt_max, p.dt_min)
    ctx.sync()
    orc.correct(ost, il, t_next, xp, vp, acc, jerk, p.eta, p.dt_max, p.dt_min)
    st = sys.state_numpy()
    np.testing.assert_allclose(st["x"], ost.x, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(st["v"], ost.v, rtol=1e-14, atol=1e-15)
    np.testing.assert_array_equal(st["a"], ost.a)
    np.testing.assert_array_equal(st["j"], ost.j)
    np.testing.assert_array_equal(st["t"], ost.t)
    np.testing.assert_array_equal(st["dt"], ost.dt)


def test_step_below_dt_min_is_reported(ctx):
    from paper_1411_5234_amd._lib import NbError
    s = inputs.plummer(256, 8)
    sys = device_system(s.x, s.v, s.m)
    acc = torch.empty(3 * s.n, dtype=torch.float64, device="cuda")
    jerk = torch.empty_like(acc)
    ctx.force_active(sys, None, s.n, 0, s.n, 1e-3, "fp64", acc, jerk)
    with pytest.raises(NbError) as e:
        ctx.init_steps(sys, acc, jerk, 0.01, 2.0 ** -3, 2.0 ** -4)
        ctx.sync()
    assert e.value.name == "NB_ERANGE"


@pytest.mark.parametrize("n,eps", [(1, 1e-3), (333, 1e-3), (4096, 1e-4), (20000, 0.0)])
def test_energy_matches_oracle(ctx, orc, n, eps):
    s = inputs.plummer(n, 9)
    sys = device_system(s.x, s.v, s.m)
    gT, gW, gE = ctx.energy(sys, eps)
    oT, oW, oE = orc.energy(s.x, s.v, s.m, eps)
    assert gT == pytest.approx(oT, rel=1e-13, abs=1e-300)
    assert gW == pytest.approx(oW, rel=1e-12, abs=1e-300)


def test_energy_at_2pow20_matches_stored_oracle(ctx):
    """nb_energy on the N = 2^20 Plummer sphere (seed 3, eps = 1e-4, the benchmarked
    workload) against the oracle's value stored by
    tests/golden/make_energy_plummer_2pow20.py (5.5e11 pairs on the CPU)."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "energy_plummer_2pow20_seed3.json")
    with open(path) as f:
        rec = json.load(f)["energy"]["0.0001"]
    s = inputs.plummer(1 << 20, 3)
    sys = device_system(s.x, s.v, s.m)
    gT, gW, gE = ctx.energy(sys, 1e-4)
    print("N=2^20: W gpu %.17g oracle %.17g (rel %.2e)" % (
        gW, rec["potential"], abs(gW - rec["potential"]) / abs(rec["potential"])), flush=True)
    assert gT == pytest.approx(rec["kinetic"], rel=1e-13)
    assert gW == pytest.approx(rec["potential"], rel=1e-12)
    del sys
    torch.cuda.empty_cache()
