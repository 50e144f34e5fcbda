"""Continuous-batching server on the GPU.

A request's result must be bitwise the same alone and in a mix that is admitted
and retired while it runs; the served result must equal the single-system
block-step integrator's (which is checked against the oracle in
test_gpu_integrate); admission must respect the memory budget; a failing request
must fail alone.
"""
import math

import numpy as np
import pytest

from paper_1411_5234_amd import inputs

pytestmark = pytest.mark.gpu

FIELDS = ("x", "v", "a", "j", "t", "dt")


@pytest.fixture(scope="module")
def ctx():
    from paper_1411_5234_amd.nbody import Context
    c = Context(0)
    yield c
    c.close()


def _req(rid, n, seed, arrival=0.0, t_end=0.25, eps=1e-3, kind="plummer"):
    return inputs.Request(rid, arrival, n, seed, eps, t_end, kind)


def _serve(ctx, reqs, precision="mixed", **kw):
    from paper_1411_5234_amd.serve import Server
    srv = Server(ctx, precision=precision, keep_state=True, **kw)
    res = srv.run(reqs, realtime=False)
    return {r.rid: r for r in res}, srv


@pytest.mark.parametrize("precision", ["mixed", "ds", "fp64"])
def test_same_result_alone_and_in_a_mix(ctx, precision):
    target = _req(0, 700, 11)
    alone, _ = _serve(ctx, [target], precision)
    mix = [_req(1, 300, 12), _req(2, 1500, 13), target, _req(3, 256, 14, t_end=0.125),
           _req(4, 900, 15), _req(5, 2048, 16, t_end=0.5), _req(6, 333, 17)]
    # three slots: systems are admitted while others are mid-run and retired
    mixed, srv = _serve(ctx, mix, precision, max_slots=3)
    assert all(r.error is None for r in mixed.values())
    a, b = alone[0].final, mixed[0].final
    for f in FIELDS:
        assert a[f].tobytes() == b[f].tobytes(), f
    assert alone[0].steps == mixed[0].steps
    assert np.all(b["t"] == 0.25)
    # the same mix on two pipes (two streams, systems split between them)
    two, srv2 = _serve(ctx, mix, precision, max_slots=3, pipes=2)
    assert len(srv2._pipes) == 2
    for rid, r in mixed.items():
        assert two[rid].error is None
        for f in FIELDS:
            assert r.final[f].tobytes() == two[rid].final[f].tobytes(), (rid, f)
        assert (r.steps, r.interactions, r.energy1) == (two[rid].steps, two[rid].interactions,
                                                        two[rid].energy1)


@pytest.mark.parametrize("order", [4, 6])
def test_lane_target_alone_and_in_a_mix(ctx, order):
    """A server with a smaller force-plan lane target: plans change (so the test
    exercises other launch shapes) and a system's result is still bitwise the same
    alone and in a mix."""
    from paper_1411_5234_amd import _lib
    from paper_1411_5234_amd.serve import Server
    lanes = 1 << 14
    # the startup step and blocks of 1024 bodies or more get other plans at N = 2048
    assert _lib.force_plan(2048, 2048, "mixed", lanes) != _lib.force_plan(2048, 2048, "mixed")
    assert _lib.force_plan(2048, 1024, "mixed", lanes) != _lib.force_plan(2048, 1024, "mixed")
    target = _req(0, 2048, 11, t_end=0.125)
    alone, _ = _serve(ctx, [target], "mixed", lanes=lanes, order=order)
    mix = [_req(1, 300, 12, t_end=0.125), target, _req(2, 1500, 13, t_end=0.125),
           _req(3, 256, 14, t_end=0.125)]
    mixed, _ = _serve(ctx, mix, "mixed", max_slots=2, lanes=lanes, order=order)
    assert all(r.error is None for r in mixed.values())
    a, b = alone[0].final, mixed[0].final
    for f in FIELDS:
        assert a[f].tobytes() == b[f].tobytes(), f
    two, _ = _serve(ctx, mix, "mixed", max_slots=3, lanes=lanes, order=order, pipes=2)
    for f in FIELDS:
        assert a[f].tobytes() == two[0].final[f].tobytes(), f
    assert alone[0].steps == mixed[0].steps
    assert np.all(b["t"] == 0.125)
    assert alone[0].energy_error < 1e-5
    with pytest.raises(_lib.NbError):
        Server(ctx, lanes=3)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_equals_single_system_integrator(ctx, precision):
    from paper_1411_5234_amd.nbody import Integrator, Params, System
    req = _req(0, 512, 21, t_end=0.25)
    served, _ = _serve(ctx, [req, _req(1, 1024, 22)], precision)
    snap = req.snapshot()
    sys_ = System.from_arrays(snap.x, snap.v, snap.m, fp32_copies=(precision != "fp64"))
    it = Integrator(ctx, sys_, Params(eps=req.eps, precision=precision))
    it.startup()
    steps, inter = it.run(req.t_end)
    st = sys_.state_numpy()
    for f in FIELDS:
        assert st[f].tobytes() == served[0].final[f].tobytes(), f
    assert served[0].steps == steps and served[0].interactions == inter


def _target_log(rid):
    """An on_iteration hook recording, for request `rid`, the block time and the
    active bodies of every block step the server ran for it (its first iteration is
    the startup step)."""
    log, seen = [], []

    def hook(srv):
        for sl in srv.slots:
            if sl.req.rid != rid:
                continue
            if not seen:
                seen.append(True)       # admitted this iteration: the startup step
                return
            # the item array of the slot's pipe is rebuilt after a retirement; its
            # values are then in sl.item
            p = sl.pipe
            k = p.slots.index(sl)
            t_next, m, done, err = ((float(p.view["t_next"][k]), int(p.view["m"][k]),
                                     int(p.view["done"][k]), int(p.view["error"][k]))
                                    if p.arr is not None else
                                    (sl.item.t_next, sl.item.m, sl.item.done, sl.item.error))
            if not done and not err:
                log.append((t_next, sl.i_idx[:m].cpu().numpy().astype(np.int64)))
    return log, hook


def test_served_in_a_mix_against_the_oracle(ctx, orc):
    """A request served while others are admitted and retired around it, against
    the oracle's block-step integration of the same initial condition (Sec. 2 items
    1-2).  FP64: the same block times and active bodies at every step, the same
    final steps, and the final state and energy within the lockstep bound.  Mixed
    precision, served in the same mix: the same number of block steps within a few
    percent and an energy error of the oracle's order."""
    from paper_1411_5234_amd.serve import Server
    target = _req(0, 512, 21, t_end=0.25)
    snap = target.snapshot()
    olog = []
    ost, osteps, _ = orc.integrate(snap.x, snap.v, snap.m, target.t_end,
                                   orc.Params(eps=target.eps), log=olog)
    E0 = orc.energy(snap.x, snap.v, snap.m, target.eps)[2]
    o_drift = abs(orc.energy(ost.x, ost.v, ost.m, target.eps)[2] - E0) / abs(E0)
    # two short requests retire while the target runs; two more are admitted then
    mix = [_req(1, 300, 12, t_end=0.125), _req(2, 700, 13, t_end=0.125), target,
           _req(3, 1500, 14), _req(4, 256, 15, t_end=0.5)]
    res = {}
    for precision in ("fp64", "mixed"):
        log, hook = _target_log(0)
        srv = Server(ctx, precision=precision, keep_state=True, max_slots=3)
        out = {r.rid: r for r in srv.run(mix, realtime=False, on_iteration=hook)}
        assert all(r.error is None for r in out.values())
        # requests 3 and 4 wait for the slots that requests 1 and 2 free
        first_free = min(out[1].finished, out[2].finished)
        assert out[3].admitted >= first_free and out[4].admitted >= first_free
        assert out[3].admitted < out[0].finished     # admitted while the target runs
        res[precision] = (out[0], log)
    r, log = res["fp64"]
    assert len(log) == len(olog) == osteps == r.steps
    for (gt, gil), (ot, oil) in zip(log, olog):
        assert gt == ot
        np.testing.assert_array_equal(gil, oil)
    g = r.final
    np.testing.assert_array_equal(g["t"], ost.t)
    np.testing.assert_array_equal(g["dt"], ost.dt)
    dx = np.abs(g["x"] - ost.x).max()
    dv = np.abs(g["v"] - ost.v).max()
    print("fp64 served: %d steps, max|dx| %.3e max|dv| %.3e, energy error %.3e (oracle %.3e)"
          % (r.steps, dx, dv, r.energy_error, o_drift), flush=True)
    assert dx < 1e-10 and dv < 1e-10
    assert abs(r.energy1 - orc.energy(ost.x, ost.v, ost.m, target.eps)[2]) <= 1e-10 * abs(E0)
    rm, _ = res["mixed"]
    print("mixed served: %d steps (oracle %d), energy error %.3e (oracle %.3e)"
          % (rm.steps, osteps, rm.energy_error, o_drift), flush=True)
    assert abs(rm.steps - osteps) <= 0.05 * osteps
    assert rm.energy_error <= 10 * o_drift + 1e-8


def test_admission_respects_memory_budget(ctx):
    from paper_1411_5234_amd.serve import Server, footprint_bytes
    reqs = [_req(k, 600 + 50 * k, 30 + k, t_end=0.125) for k in range(8)]
    budget = footprint_bytes(700, "mixed") * 2 + 10
    seen = []
    srv = Server(ctx, precision="mixed", memory_budget=budget)
    res = srv.run(reqs, realtime=False,
                  on_iteration=lambda s: seen.append((len(s.slots), s.used)))
    assert len(res) == 8 and all(r.error is None for r in res)
    assert max(k for k, _ in seen) <= 2
    assert max(u for _, u in seen) <= budget
    with pytest.raises(ValueError):
        srv.submit(_req(99, 10 ** 6, 1))


class _NaNRequest(inputs.Request):
    def snapshot(self):
        s = inputs.plummer(self.n, self.seed)
        s.x[3, 1] = float("nan")
        return s


def test_a_failing_request_fails_alone(ctx):
    bad = _NaNRequest(1, 0.0, 400, 41, 1e-3, 0.25)
    good = _req(0, 500, 42)
    alone, _ = _serve(ctx, [good])
    both, _ = _serve(ctx, [good, bad, _req(2, 300, 43)])
    assert both[1].error is not None
    assert both[0].error is None and both[2].error is None
    for f in FIELDS:
        assert alone[0].final[f].tobytes() == both[0].final[f].tobytes(), f


def test_poisson_stream_latency_and_throughput(ctx):
    from paper_1411_5234_amd.serve import Server, summarize
    import time
    reqs = inputs.request_stream(24, 4, 256, 2048, rate=200.0, eps=1e-3, t_end=0.25,
                                 ic_seed_base=4000)
    srv = Server(ctx, precision="mixed", max_slots=16)
    t0 = time.perf_counter()
    res = srv.run(reqs, realtime=True)
    s = summarize(res, time.perf_counter() - t0)
    print(s, flush=True)
    assert s["completed"] == 24 and s["failed"] == 0
    assert 0 < s["latency_p50_s"] <= s["latency_p99_s"]
    assert s["energy_error_max"] < 1e-4
    assert all(r.admitted >= r.arrival - 1e-9 for r in res)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_sixth_order_served_equals_integrator6_alone_and_in_a_mix(ctx, precision):
    """nb_step6_batch: a system served at 6th order in a mix (admitted and retired
    around it) gets the same bits as the single-system 6th-order integrator."""
    from paper_1411_5234_amd.nbody import Integrator6, Params6, System
    target = _req(0, 600, 51, t_end=0.25)
    mix = [_req(1, 300, 52), target, _req(2, 1200, 53, t_end=0.125), _req(3, 256, 54),
           _req(4, 800, 55, t_end=0.5)]
    served, _ = _serve(ctx, mix, precision, max_slots=3, order=6)
    assert all(r.error is None for r in served.values())
    snap = target.snapshot()
    sys_ = System.from_arrays(snap.x, snap.v, snap.m, fp32_copies=(precision != "fp64"))
    it = Integrator6(ctx, sys_, Params6(eps=target.eps, precision=precision))
    it.startup()
    steps, inter = it.run(target.t_end)
    st = sys_.state_numpy()
    for f in FIELDS:
        assert st[f].tobytes() == served[0].final[f].tobytes(), f
    assert served[0].steps == steps and served[0].interactions == inter
    assert served[0].energy_error < 1e-6


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_grouped_pairs_alone_in_a_mix_and_as_the_integrator(ctx, precision):
    """Requests with primordial binaries served with the pairs carried as
    centre-of-mass bodies (their orbits advanced on the CPU thread from batched
    tidal tensors): the target's reduced state and pair orbits are bitwise the same
    served alone, served in a mix that is admitted and retired around it, and run
    by the single-system grouped integrator (which is checked against the oracle's
    grouped integration in test_gpu_groups)."""
    from paper_1411_5234_amd.groups import GroupedIntegrator
    from paper_1411_5234_amd.nbody import Params
    from paper_1411_5234_amd.serve import Server

    def bin_req(rid, n, seed, t_end=0.125):
        return inputs.Request(rid, 0.0, n, seed, 1e-5, t_end, "kroupa_binaries")

    target = bin_req(0, 1500, 5101)
    keys = FIELDS + ("pair_r", "pair_w", "members_x", "members_v")
    # every pair grouped and none returned, as the single-system integrator does
    kw = dict(precision=precision, keep_state=True, groups=True, group_gamma=float("inf"),
              split_gamma=0.0)
    srv = Server(ctx, **kw)
    alone = srv.run([target], realtime=False)[0]
    assert alone.error is None and alone.pairs == 75
    mix = [_req(1, 300, 12, t_end=0.125), bin_req(2, 1100, 5102), target,
           _req(3, 2048, 14, t_end=0.25), bin_req(4, 900, 5103)]
    srv = Server(ctx, max_slots=2, **kw)
    out = {r.rid: r for r in srv.run(mix, realtime=False)}
    assert all(r.error is None for r in out.values()), {k: r.error for k, r in out.items()}
    b = out[0]
    for f in keys:
        assert alone.final[f].tobytes() == b.final[f].tobytes(), f
    assert alone.steps == b.steps
    snap = target.snapshot()
    gi = GroupedIntegrator(ctx, snap.x, snap.v, snap.m, snap.meta["pairs"],
                           Params(eps=target.eps, precision=precision))
    gi.startup()
    steps, _ = gi.run(target.t_end)
    st = gi.sys.state_numpy()
    for f in FIELDS:
        assert st[f].tobytes() == b.final[f].tobytes(), f
    assert gi.r.tobytes() == b.final["pair_r"].tobytes()
    assert gi.w.tobytes() == b.final["pair_w"].tobytes()
    assert steps == b.steps
    e_scheme = abs(b.energy1 - b.energy0) / abs(b.energy0)
    e_direct = abs(b.direct1 - b.direct0) / abs(b.direct0)
    print("%s grouped: %d block steps, scheme energy error %.3e, direct %.3e" %
          (precision, b.steps, e_scheme, e_direct), flush=True)
    assert abs(b.energy1 - gi.energy()) <= 1e-14 * abs(b.energy1)
    assert e_scheme < 1e-4


def test_pairs_return_to_the_n_body_system(ctx):
    """Grouped pairs whose perturbation grows past the split threshold rejoin the
    N-body system as two bodies mid-run (here a low threshold makes many do so):
    the run completes, the result is bitwise the same alone and in a mix, and the
    scheme's conserved quantity (with the known change at each return) and the
    full N-body energy stay conserved."""
    from paper_1411_5234_amd.serve import Server

    def bin_req(rid, n, seed, t_end=0.125):
        return inputs.Request(rid, 0.0, n, seed, 1e-5, t_end, "kroupa_binaries")

    target = bin_req(0, 1500, 5101)
    keys = FIELDS + ("pair_r", "pair_w", "members_x", "members_v")
    kw = dict(precision="fp64", keep_state=True, groups=True, split_gamma=1e-4)
    alone = Server(ctx, **kw).run([target], realtime=False)[0]
    assert alone.error is None, alone.error
    print("grouped %d pairs, %d returned, %d block steps; conserved quantity error %.3e "
          "(return offset %.3e), direct %.3e" % (
              alone.pairs, alone.splits, alone.steps, alone.energy_error, alone.split_energy,
              abs(alone.direct1 - alone.direct0) / abs(alone.direct0)), flush=True)
    assert 0 < alone.splits < alone.pairs
    assert alone.final["pair_r"].shape[0] == alone.pairs - alone.splits
    mix = [_req(1, 300, 12, t_end=0.125), bin_req(2, 1100, 5102), target, bin_req(4, 900, 5103)]
    out = {r.rid: r for r in Server(ctx, max_slots=2, **kw).run(mix, realtime=False)}
    assert all(r.error is None for r in out.values()), {k: r.error for k, r in out.items()}
    b = out[0]
    for f in keys:
        assert alone.final[f].tobytes() == b.final[f].tobytes(), f
    assert (alone.steps, alone.splits) == (b.steps, b.splits)
    assert alone.energy_error < 1e-4
    # with captures too: returns and captures in several systems of one iteration
    # move segments of the shared pair table under each other
    kc = dict(kw, capture_every=1)
    solo = Server(ctx, **kc).run([target], realtime=False)[0]
    outc = {r.rid: r for r in Server(ctx, max_slots=3, **kc).run(mix, realtime=False)}
    assert solo.error is None and all(r.error is None for r in outc.values()), \
        {k: r.error for k, r in outc.items()}
    print("with captures: %d returned, %d captured; conserved quantity error %.3e" % (
        solo.splits, solo.captures, solo.energy_error), flush=True)
    for f in keys + ("pairs",):
        assert solo.final[f].tobytes() == outc[0].final[f].tobytes(), f
    assert solo.energy_error < 1e-4
    # admission keeps only pairs below the grouping threshold
    few = Server(ctx, precision="fp64", groups=True, group_gamma=1e-5).run([target],
                                                                            realtime=False)[0]
    assert few.error is None and few.pairs < alone.pairs


def _forming_ic(n=600, seed=7301):
    """A cluster with hard binaries that no one has declared as pairs, plus two
    single bodies on a fast (unbound) close flyby of each other."""
    from dataclasses import dataclass
    b = inputs.with_binaries(n, seed, frac_members=0.02, a_lo=1e-4, a_hi=3e-4, imf="equal")
    x, v, m = b.x.copy(), b.v.copy(), b.m.copy()
    planted = [tuple(int(i) for i in q) for q in b.meta["pairs"]]
    i, j = n - 1, n - 2                        # singles of the sample
    x[j] = x[i] + [2e-4, 0.0, 0.0]
    w = 3.0 * math.sqrt((m[i] + m[j]) / 2e-4)  # well above the escape speed
    v[j] = v[i] + [0.0, w, 0.0]
    snap = inputs.Snapshot(x, v, m, {"kind": "binaries, undeclared"})

    @dataclass
    class _Req(inputs.Request):
        def snapshot(self):
            return snap
    return snap, planted, (j, i), _Req


def test_pairs_form_during_the_run(ctx, orc):
    """Bound pairs that nobody declared are found during the run and carried as one
    body: each captured pair is one of the planted binaries (mutual nearest
    neighbours, bound, weakly perturbed), never the unbound flyby; the tidal
    tensor a new pair starts with matches the oracle's at its centre of mass; the
    result is bitwise the same alone and in a mix; and the conserved quantity,
    with the known change at each capture, stays conserved."""
    import time
    from paper_1411_5234_amd.serve import Server
    snap, planted, flyby, Req = _forming_ic()
    eps = 1e-5
    target = Req(0, 0.0, snap.n, 0, eps, 0.125, "custom")
    kw = dict(precision="fp64", keep_state=True, groups=True, capture_every=1)
    # step by step up to the first capture: the new pairs' starting tensors
    srv = Server(ctx, **kw)
    srv.t0 = time.perf_counter()
    srv.submit(target)
    srv._admit()
    slot = srv.slots[0]
    for _ in range(2000):
        srv.step()
        if slot.result.captures:
            break
    k = slot.result.captures
    assert k > 0
    ps = slot.ps
    st = slot.sys.state_numpy()
    rows = np.arange(ps.cm0 + ps.np - k, ps.cm0 + ps.np)
    T_or = orc.tidal(st["xp"], st["m"], eps, rows)
    T_gpu = ps.T[ps.np - k:].reshape(k, 3, 3)
    err = np.abs(T_gpu - T_or).max() / np.abs(T_or).max()
    print("first capture: %d pairs at t = %.6g; tensor vs oracle %.3e" % (
        k, ps.tpair[ps.np - 1], err), flush=True)
    assert err <= 1e-12
    assert np.all(st["t"][rows] == ps.tpair[ps.np - k:])
    # whole runs, alone and in a mix
    alone = Server(ctx, **kw).run([target], realtime=False)[0]
    assert alone.error is None, alone.error
    got = {tuple(sorted(int(i) for i in q)) for q in alone.final["pairs"]}
    print("captured %d, returned %d, held at the end %s of planted %s; energy error %.3e "
          "(capture offset %.3e), direct %.3e" % (
              alone.captures, alone.splits, sorted(got), sorted(planted), alone.energy_error,
              alone.capture_energy, abs(alone.direct1 - alone.direct0) / abs(alone.direct0)),
          flush=True)
    assert alone.captures >= 1 and got and got <= set(planted)
    assert tuple(sorted(flyby)) not in got
    assert alone.energy_error < 1e-4
    mix = [_req(1, 300, 12, t_end=0.125), target, _req(2, 800, 13, t_end=0.125)]
    out = {r.rid: r for r in Server(ctx, max_slots=2, **kw).run(mix, realtime=False)}
    assert all(r.error is None for r in out.values()), {k: r.error for k, r in out.items()}
    b = out[0]
    for f in FIELDS + ("pair_r", "pair_w", "members_x", "members_v", "pairs"):
        assert alone.final[f].tobytes() == b.final[f].tobytes(), f
    assert (alone.steps, alone.captures, alone.splits) == (b.steps, b.captures, b.splits)
