"""Block-step Hermite-4 integration on the GPU in lockstep with the oracle.

N = 1024 equal-mass Plummer sphere, eps = 1e-3, eta = 0.02, eta_s = 0.01,
dt_max = 1/8, to t = 1.  At every block step both sides must pick the same block
time and the same active bodies; the GPU force on the GPU's predicted state must
match the oracle's force on that same state to the FP64 gate; at the end the two
final states and energies are compared.  The run is chaotic, so the final-state
difference is reported and bounded loosely, while the schedule must be identical.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import TOL, device_system, rel_err
from paper_1411_5234_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


def test_lockstep_fp64_plummer_1024(ctx, orc):
    from paper_1411_5234_amd.nbody import Integrator, Params
    s = inputs.plummer(1024, 1)
    eps = 1e-3
    op = orc.Params(eps=eps)
    ost = orc.startup(s.x, s.v, s.m, op)
    sys = device_system(s.x, s.v, s.m)
    it = Integrator(ctx, sys, Params(eps=eps, precision="fp64"))
    it.startup()
    st = sys.state_numpy()
    np.testing.assert_array_equal(st["dt"], ost.dt)
    E0 = orc.energy(s.x, s.v, s.m, eps)[2]
    worst = 0.0
    steps = 0
    while True:
        t_next, m = ctx.select_active(sys, it.i_idx)
        ot, oil = orc.select(ost.t, ost.dt)
        assert t_next == ot
        if t_next > 1.0:
            break
        gil = it.i_idx[:m].cpu().numpy()
        np.testing.assert_array_equal(gil, oil)
        it._advance(t_next, m)
        if steps % 97 == 0:   # force parity on the GPU's own predicted state
            g = sys.state_numpy()
            ga = it.acc.view(-1)[: 3 * m].view(3, m).T.cpu().numpy()
            gj = it.jerk.view(-1)[: 3 * m].view(3, m).T.cpu().numpy()
            oa, oj = orc.force(g["xp"], g["vp"], g["m"], eps, oil)
            worst = max(worst, rel_err(ga, oa).max(), rel_err(gj, oj).max())
        orc.block_step(ost, op)
        steps += 1
    ctx.sync()
    g = sys.state_numpy()
    assert np.all(g["t"] == 1.0) and np.all(ost.t == 1.0)
    np.testing.assert_array_equal(g["dt"], ost.dt)
    assert worst <= TOL["fp64"], worst
    dx = np.abs(g["x"] - ost.x).max()
    gE = ctx.energy(sys, eps)[2]
    oE = orc.energy(ost.x, ost.v, ost.m, eps)[2]
    print("steps %d  max|dx| %.3e  force worst %.3e  E0 %.15f  E_gpu %.15f  E_orc %.15f  "
          "drift gpu %.3e orc %.3e" % (steps, dx, worst, E0, gE, oE, abs(gE - E0) / abs(E0),
                                       abs(oE - E0) / abs(E0)), flush=True)
    assert dx < 1e-6
    assert abs(gE - oE) / abs(oE) < 1e-9


def test_mixed_integration_energy_drift(ctx, orc):
    from paper_1411_5234_amd.nbody import Integrator, Params
    s = inputs.plummer(1024, 1)
    eps = 1e-3
    E0 = orc.energy(s.x, s.v, s.m, eps)[2]
    res = {}
    for prec in ("fp64", "mixed"):
        sys = device_system(s.x, s.v, s.m)
        it = Integrator(ctx, sys, Params(eps=eps, precision=prec))
        it.startup()
        steps, inter = it.run(1.0)
        E1 = ctx.energy(sys, eps)[2]
        res[prec] = abs(E1 - E0) / abs(E0)
        print("%s: steps %d interactions %d drift %.3e" % (prec, steps, inter, res[prec]), flush=True)
    # the mixed path's drift stays at the integrator's level, not the FP32 round-off floor
    assert res["fp64"] < 1e-6
    assert res["mixed"] < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_native_steps_equal_separate_calls(ctx, precision):
    """Integrator.run steps through nb_step_batch (one native call per block step)
    unless a log is asked for; both routes give the same block sequence and the
    same final state, bitwise."""
    from paper_1411_5234_amd.nbody import Integrator, Params
    s = inputs.plummer(2000, 31, masses=inputs.salpeter_masses(2000, 32))
    out = []
    for use_log in (False, True):
        sys = device_system(s.x, s.v, s.m)
        it = Integrator(ctx, sys, Params(eps=1e-3, precision=precision))
        it.startup()
        seen = []
        steps, inter = it.run(0.25, log=[] if use_log else None,
                              progress=lambda t, k: seen.append((t, k)))
        st = sys.state_numpy()
        out.append((steps, inter, st, [t for t, _ in seen]))
    (s0, i0, st0, t0), (s1, i1, st1, t1) = out
    print("%s: %d steps, %d interactions" % (precision, s0, i0), flush=True)
    assert s0 == s1 and i0 == i1 and t0 == t1 and len(t0) == s0
    for k in st0:
        assert st0[k].tobytes() == st1[k].tobytes(), k


def test_n_2pow20_integration_force_parity_sampled(ctx, orc):
    """The benchmarked N = 2^20 Plummer system (eps = 1e-4, mixed precision) in its
    real block-step integration: at several block steps, up to 64 of the active
    bodies' forces, computed by the production launch on the GPU's own predicted
    state, against the oracle on that state."""
    from gpu_helpers import check
    from paper_1411_5234_amd.nbody import Integrator, Params
    n = 1 << 20
    s = inputs.plummer(n, 3)
    sys = device_system(s.x, s.v, s.m)
    it = Integrator(ctx, sys, Params(eps=1e-4, precision="mixed"))
    it.startup()
    rng = np.random.default_rng(40)
    checked = 0
    for step in range(60):
        t_next, m = ctx.select_active(sys, it.i_idx)
        it._advance(t_next, m)
        if step % 12 != 11:
            continue
        g = sys.state_numpy()
        il = it.i_idx[:m].cpu().numpy().astype(np.int64)
        pick = np.sort(rng.choice(m, min(m, 64), replace=False))
        ga = it.acc.view(-1)[: 3 * m].view(3, m).T.cpu().numpy()[pick]
        gj = it.jerk.view(-1)[: 3 * m].view(3, m).T.cpu().numpy()[pick]
        check(orc, "mixed", ga, gj, g["xp"], g["vp"], g["m"], 1e-4, il[pick],
              tag="N=2^20 step %d t=%.3e m=%d" % (step, t_next, m))
        checked += 1
    assert checked == 5
    del sys
    torch.cuda.empty_cache()
