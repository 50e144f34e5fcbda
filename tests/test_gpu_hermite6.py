"""GPU parity of the 6th-order Hermite path (nb_predict6, nb_force6_active,
nb_init_steps6, nb_correct6) against the FP64 oracle.

Force gates as the 4th-order path (see gpu_helpers.check6): acceleration
relative error, jerk and snap error over their magnitude scales, 1e-12 for FP64
and 1e-6 for the mixed and double-single forms.  Predictor and corrector are
FP64 on both sides and are compared to ~1e-13; the new power-of-two steps and
the block sequence of a whole FP64 integration must be identical.
"""
import numpy as np
import pytest
import torch

from gpu_helpers import check6, device_system6, gpu_force6
from paper_1411_5234_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


def _with_acc(orc, s, eps):
    a, _ = orc.force(s.x, s.v, s.m, eps)
    return a


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_force6_plummer_1024_all_active(ctx, orc, precision):
    s = inputs.plummer(1024, 61)
    ap = _with_acc(orc, s, 1e-3)
    sys, h6 = device_system6(s.x, s.v, s.m, ap)
    g = gpu_force6(ctx, sys, h6, 1e-3, precision)
    check6(orc, precision, g, s.x, s.v, ap, s.m, 1e-3, tag="N=1024")


@pytest.mark.parametrize("precision", ["mixed", "ds", "fp64"])
def test_force6_plummer_2pow20_all_active_sampled(ctx, orc, precision):
    """The 6th-order launch of `bench.py --order 6` (m = N = 2^20) on 256 random
    bodies and on the 128 bodies whose acceleration or jerk cancels most.  The
    predicted accelerations are the smooth mean field of the Plummer model,
    -r / (r^2 + a^2)^(3/2) with a = 3 pi / 16, a seeded input that both sides take
    (an oracle pass over all 2^20 bodies would take the CPU too long)."""
    from test_gpu_force import top_kappa_2pow20
    n = 1 << 20
    s = inputs.plummer(n, 3)
    a2 = (3.0 * np.pi / 16.0) ** 2
    ap = -s.x / ((s.x ** 2).sum(1) + a2)[:, None] ** 1.5
    sys, h6 = device_system6(s.x, s.v, s.m, ap)
    g = gpu_force6(ctx, sys, h6, 1e-4, precision)
    pick = np.sort(np.random.default_rng(31).choice(n, 256, replace=False))
    check6(orc, precision, tuple(q[pick] for q in g), s.x, s.v, ap, s.m, 1e-4, pick,
           tag="N=2^20 all active (256 sampled)")
    top_a, top_j = top_kappa_2pow20()
    top = np.unique(np.concatenate([top_a, top_j]))
    check6(orc, precision, tuple(q[top] for q in g), s.x, s.v, ap, s.m, 1e-4, top,
           tag="N=2^20 all active (the 128 largest kappa)")


@pytest.fixture(scope="module")
def salpeter16k(orc):
    n = 16384
    s = inputs.plummer(n, 62, masses=inputs.salpeter_masses(n, 63))
    return s, _with_acc(orc, s, 1e-4)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
@pytest.mark.parametrize("m", [64, 1000, 16384])
def test_force6_salpeter_active_blocks(ctx, orc, salpeter16k, precision, m):
    s, ap = salpeter16k
    il = np.sort(np.random.default_rng(m).permutation(s.n)[:m])
    sys, h6 = device_system6(s.x, s.v, s.m, ap)
    g = gpu_force6(ctx, sys, h6, 1e-4, precision, il)
    pick = np.arange(m) if m <= 1000 else np.random.default_rng(64).choice(m, 512, replace=False)
    g = tuple(q[pick] for q in g)
    check6(orc, precision, g, s.x, s.v, ap, s.m, 1e-4, il[pick], tag="N=16384 m=%d" % m)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_force6_every_plan_shape(ctx, orc, precision):
    s = inputs.plummer(3000, 65, masses=inputs.salpeter_masses(3000, 66))
    ap = _with_acc(orc, s, 1e-2)
    sys, h6 = device_system6(s.x, s.v, s.m, ap)
    il = np.sort(np.random.default_rng(67).choice(3000, 333, replace=False))
    for plan in [(1, 1, 1), (2, 1, 3), (4, 1, 2), (1, 4, 1), (2, 16, 5), (1, 64, 2), (4, 64, 1)]:
        g = gpu_force6(ctx, sys, h6, 1e-2, precision, il, plan=plan)
        check6(orc, precision, g, s.x, s.v, ap, s.m, 1e-2, il, tag="plan %s" % (plan,))


@pytest.mark.parametrize("precision", ["fp64", "mixed", "ds"])
def test_force6_many_j_chunks(ctx, orc, salpeter16k, precision):
    """A small active block over 32 j-chunks: nine partial sums per body reduced
    with two lanes per output value."""
    s, ap = salpeter16k
    il = np.sort(np.random.default_rng(70).permutation(s.n)[:50])
    sys, h6 = device_system6(s.x, s.v, s.m, ap)
    for plan in [(1, 64, 32), (2, 16, 32), (1, 4, 20)]:
        g = gpu_force6(ctx, sys, h6, 1e-4, precision, il, plan=plan)
        check6(orc, precision, g, s.x, s.v, ap, s.m, 1e-4, il, tag="chunks %s" % (plan,))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_force6_ragged_j_ranges_and_repeatability(ctx, orc, precision):
    s = inputs.plummer(1000, 68, masses=inputs.salpeter_masses(1000, 69))
    ap = _with_acc(orc, s, 1e-2)
    sys, h6 = device_system6(s.x, s.v, s.m, ap)
    il = np.sort(np.random.default_rng(70).choice(1000, 77, replace=False))
    for j0, j1 in [(13, 911), (0, 1), (999, 1000), (511, 513)]:
        g = gpu_force6(ctx, sys, h6, 1e-2, precision, il, j0, j1)
        check6(orc, precision, g, s.x, s.v, ap, s.m, 1e-2, il, j0, j1,
               tag="ragged [%d,%d)" % (j0, j1))
    a = gpu_force6(ctx, sys, h6, 1e-2, precision, il)
    b = gpu_force6(ctx, sys, h6, 1e-2, precision, il)
    for p, q in zip(a, b):
        assert p.tobytes() == q.tobytes()


def _random_state(rng, n):
    st = {k: rng.normal(size=(n, 3)) for k in ("x", "v", "a", "j", "s", "c")}
    st["m"] = rng.uniform(0.5, 1.5, n) / n
    return st


def _load_state(sys, h6, st, t, dt):
    n = sys.n
    host = sys.buf64.cpu()
    for k, key in enumerate(("x", "v", "a", "j")):
        host[3 * k:3 * k + 3, :n] = torch.from_numpy(st[key].T.copy())
    host[12, :n] = torch.from_numpy(st["m"])
    host[13, :n] = torch.from_numpy(t)
    host[14, :n] = torch.from_numpy(dt)
    sys.buf64.copy_(host)
    h = h6.buf64.cpu()
    h[0:3, :n] = torch.from_numpy(st["s"].T.copy())
    h[3:6, :n] = torch.from_numpy(st["c"].T.copy())
    h6.buf64.copy_(h)


def test_predict6_matches_oracle(ctx, orc):
    from paper_1411_5234_amd.nbody import Hermite6, System
    rng = np.random.default_rng(71)
    n = 1537
    st = _random_state(rng, n)
    dt = 2.0 ** -rng.integers(2, 12, n)
    t_next = 0.75
    t = t_next - dt * rng.integers(1, 3, n)
    sys = System(n, "cuda")
    h6 = Hermite6(sys)
    _load_state(sys, h6, st, t, dt)
    ctx.predict6(sys, h6, t_next)
    ctx.sync()
    xp, vp, ap = orc.predict6(st["x"], st["v"], st["a"], st["j"], st["s"], st["c"], t, t_next)
    g = sys.state_numpy()
    gh = h6.state_numpy()
    for got, want in ((g["xp"], xp), (g["vp"], vp), (gh["ap"], ap)):
        np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-15)
    # FP32 copies are the roundings of the FP64 values
    assert np.array_equal(sys.buf32[0:3, :n].cpu().numpy(), g["vp"].T.astype(np.float32))
    assert np.array_equal(h6.buf32[:, :n].cpu().numpy(), gh["ap"].T.astype(np.float32))


def test_correct6_matches_oracle(ctx, orc):
    """One real block step of a Plummer sphere: state, forces and steps from the oracle."""
    from paper_1411_5234_amd.nbody import Hermite6, System
    s = inputs.plummer(2048, 72)
    p = orc.Params6(eps=1e-2)
    st = orc.startup6(s.x, s.v, s.m, p)
    for _ in range(3):   # a few steps so that the crackle is set
        orc.block_step6(st, p)
    t_next, il = orc.select(st.t, st.dt)
    xp, vp, ap = orc.predict6(st.x, st.v, st.a, st.j, st.s, st.c, st.t, t_next)
    acc, jerk, snap = orc.force6(xp, vp, ap, st.m, p.eps, il)
    sys = System(st.n, "cuda")
    h6 = Hermite6(sys)
    _load_state(sys, h6, {"x": st.x, "v": st.v, "a": st.a, "j": st.j, "s": st.s, "c": st.c,
                          "m": st.m}, st.t, st.dt)
    dev = lambda q: torch.from_numpy(np.ascontiguousarray(q.T)).cuda().view(-1)
    idx = torch.as_tensor(il.astype(np.int32), device="cuda")
    ctx.correct6(sys, h6, idx, il.size, dev(acc), dev(jerk), dev(snap), t_next, p.eta, p.dt_max,
                 p.dt_min)
    ctx.sync()
    want = st.copy()
    orc.correct6(want, il, t_next, acc, jerk, snap, p.eta, p.dt_max, p.dt_min)
    g, gh = sys.state_numpy(), h6.state_numpy()
    for key, got in (("x", g["x"]), ("v", g["v"]), ("a", g["a"]), ("j", g["j"]), ("s", gh["s"])):
        ref = getattr(want, key)
        scale = np.abs(ref).max(axis=1, keepdims=True) + 1e-300
        assert np.all(np.abs(got - ref) <= 1e-13 * scale), key
    # crackle: closed form on the GPU, a linear solve in the oracle; both round
    # the same differences of size |a|/h^3
    h = (t_next - st.t[il])[:, None]
    sc = (np.abs(acc) / h ** 3 + np.abs(jerk) / h ** 2 + np.abs(snap) / h).max(axis=1)
    dc = np.abs(gh["c"][il] - want.c[il]).max(axis=1)
    assert np.all(dc <= 1e-12 * sc), (dc / sc).max()
    assert np.array_equal(g["t"], want.t)
    assert np.array_equal(g["dt"], want.dt)


def test_integrate6_fp64_lockstep_with_oracle(ctx, orc):
    from paper_1411_5234_amd.nbody import Integrator6, Params6, System
    s = inputs.plummer(384, 73)
    p = Params6(eps=1e-2, precision="fp64")
    sys = System.from_arrays(s.x, s.v, s.m, fp32_copies=False)
    it = Integrator6(ctx, sys, p)
    it.startup()
    glog = []
    steps, inter = it.run(0.25, log=glog)
    olog = []
    ost, osteps, ointer = orc.integrate6(s.x, s.v, s.m, 0.25, orc.Params6(eps=1e-2), log=olog)
    print("GPU %d steps, oracle %d steps" % (steps, osteps), flush=True)
    assert steps == osteps and inter == ointer
    for (tg, ig), (to, io) in zip(glog, olog):
        assert tg == to and np.array_equal(ig, io)
    g = sys.state_numpy()
    assert np.abs(g["x"] - ost.x).max() <= 1e-10
    assert np.abs(g["v"] - ost.v).max() <= 1e-10
    assert np.array_equal(g["t"], ost.t) and np.array_equal(g["dt"], ost.dt)


@pytest.mark.parametrize("precision", ["mixed", "ds"])
def test_integrate6_reduced_precision_energy(ctx, orc, precision):
    from paper_1411_5234_amd.nbody import Integrator6, Params6, System
    s = inputs.plummer(1024, 74)
    sys = System.from_arrays(s.x, s.v, s.m)
    it = Integrator6(ctx, sys, Params6(eps=1e-3, precision=precision))
    it.startup()
    steps, _ = it.run(0.25)
    e0 = orc.energy(s.x, s.v, s.m, 1e-3)[2]
    g = sys.state_numpy()
    e1 = orc.energy(g["x"], g["v"], g["m"], 1e-3)[2]
    print("%s: %d steps, |dE/E| = %.3e" % (precision, steps, abs(e1 - e0) / abs(e0)), flush=True)
    assert np.all(g["t"] == 0.25)
    assert abs(e1 - e0) / abs(e0) < 1e-5


def test_hermite6_argument_errors(ctx):
    from paper_1411_5234_amd import _lib
    from paper_1411_5234_amd.nbody import Hermite6, System
    s = inputs.plummer(64, 75)
    sys = System.from_arrays(s.x, s.v, s.m)
    h6 = Hermite6(sys)
    out = torch.zeros(3 * 64, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.NbError) as e:
        rc = ctx.L.nb_force6_active(ctx.h, sys.ref, h6.ref, None, 64, 0, 64, 1e-2, 1,
                                    out.data_ptr(), out.data_ptr(), None)
        ctx._check(rc)
    assert e.value.name == "NB_EINVAL"
    rc = ctx.L.nb_force6_active(ctx.h, sys.ref, None, None, 64, 0, 64, 1e-2, 1, out.data_ptr(),
                                out.data_ptr(), out.data_ptr())
    assert rc == -1
    h6_64 = Hermite6(sys, fp32_copies=False)
    with pytest.raises(_lib.NbError):
        ctx.force6_active(sys, h6_64, None, 64, 0, 64, 1e-2, "mixed", out, out, out)
    with pytest.raises(_lib.NbError):
        ctx.correct6(sys, h6, None, 65, out, out, out, 0.125, 0.14, 0.125, 2.0 ** -40)
    ctx.sync()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step6_native_equals_separate_calls(ctx, precision):
    """Integrator6.run steps through nb_step6 unless a log is asked for; both routes
    give the same block sequence and the same final state, bitwise."""
    from paper_1411_5234_amd.nbody import Integrator6, Params6, System
    s = inputs.plummer(1500, 71, masses=inputs.salpeter_masses(1500, 72))
    out = []
    for use_log in (False, True):
        sys = System.from_arrays(s.x, s.v, s.m)
        it = Integrator6(ctx, sys, Params6(eps=1e-3, precision=precision))
        it.startup()
        seen = []
        steps, inter = it.run(0.125, log=[] if use_log else None,
                              progress=lambda t, k: seen.append(t))
        out.append((steps, inter, sys.state_numpy(), it.h6.state_numpy(), seen))
    (s0, i0, st0, h0, t0), (s1, i1, st1, h1, t1) = out
    print("%s: %d steps" % (precision, s0), flush=True)
    assert s0 == s1 and i0 == i1 and t0 == t1 and len(t0) == s0 > 0
    for k in st0:
        assert st0[k].tobytes() == st1[k].tobytes(), k
    for k in h0:
        assert h0[k].tobytes() == h1[k].tobytes(), k


def test_step6_reports_done_and_bad_arguments(ctx):
    import ctypes as C

    from paper_1411_5234_amd._lib import PRECISIONS
    from paper_1411_5234_amd.nbody import Integrator6, Params6, System
    s = inputs.plummer(200, 73)
    sys = System.from_arrays(s.x, s.v, s.m)
    it = Integrator6(ctx, sys, Params6(eps=1e-3))
    it.startup()
    tn, m, done = C.c_double(), C.c_int32(), C.c_int32()
    base = [ctx.h, sys.ref, it.h6.ref, it.i_idx.data_ptr(), it.acc.data_ptr(), it.jerk.data_ptr(),
            it.snap.data_ptr(), 1e-3, PRECISIONS["mixed"], 0.14, 0.125, 2.0 ** -40]
    # t_end before the first block time: nothing is enqueued
    assert ctx.L.nb_step6(*base, -1.0, C.byref(tn), C.byref(m), C.byref(done)) == 0
    assert done.value == 1 and tn.value > 0 and m.value > 0
    # bad step parameters, missing done pointer
    bad = list(base)
    bad[9] = -0.1
    assert ctx.L.nb_step6(*bad, 1.0, C.byref(tn), C.byref(m), C.byref(done)) == -1
    assert ctx.L.nb_step6(*base, 1.0, C.byref(tn), C.byref(m), None) == -1
