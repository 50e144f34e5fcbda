"""Benchmark: pair-interactions/s of the Hermite-4 block-step hot path at N = 2^20.

Workload: N = 1,048,576 equal-mass Plummer sphere (seed 3, Henon units), eps = 1e-4,
mixed precision (FP64 positions and differences, FP32 pair arithmetic, FP64
accumulation).  One step is one block step of the whole path -- select the active
block, predict all bodies, acceleration + jerk of the block, Hermite correction and
new steps -- in which the whole system is the active block: the run uses one shared
power-of-two step h, the smallest startup step of any body, so every body is due at
every block time (m = N).  Inputs are resident in HBM before timing starts.

Prints one JSON line (see the keys below).  `value` = sum over timed steps of m * N
divided by the wall time of the K timed steps.  The roofline object refers to the
force kernel, timed with HIP events on the stream it is launched on; algorithmic
work is 41 flops per pair interaction.  cpu_baseline times the oracle on a bounded
sample of the same workload (the first 4096 bodies against all N) and reports the
sample's relative errors of the GPU result against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "pair-interactions/s & % FP32 peak at N=1M; ensemble solves/s, p99 latency"
FLOPS_PER_INTERACTION = 41
# 6th order (acc + jerk + snap): 9 differences, s (6), r.w, w.w, r.b (15), rsqrt, r^-2 and
# m s^-3/2 (4), alpha (1), beta (4), -3 alpha, -6 alpha, -3 beta (3), acc (6), u (6),
# jerk (6), snap term (12) and snap (6), with FMA = 2
FLOPS_PER_INTERACTION6 = 78
# The count other Hermite GPU codes quote for one acc + jerk interaction; reported
# beside the algorithmic count, labelled, never as the roofline.
FLOPS_CONVENTION4 = 60
PEAK_FP32_TFLOPS = 157.3     # MI355X dense FP32 vector (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_FP64_TFLOPS = 78.6

# HBM bytes per force launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (scaled by a
# plain-copy calibration: x2.0 fetch, x1.0 write), keyed by the hash of the force
# kernel's sources, the precision, N and the launch plan.  Reported only for that
# exact kernel and launch; null otherwise.  Taken with the current sources.
TRAFFIC = {("5fcf579e3352ce45", "mixed", 1 << 20, (2, 1, 4)): 2.7712e9 + 2.0133e8}


def _kernel_source_hash(order=4):
    import hashlib
    h = hashlib.sha256()
    base = os.path.join(ROOT, "paper_1411_5234_amd", "csrc")
    for f in ("nb_internal.h", "pair.h", "force.hip" if order == 4 else "force6.hip"):
        with open(os.path.join(base, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--precision", choices=["mixed", "ds", "fp64"], default="mixed")
    ap.add_argument("--order", type=int, choices=[4, 6], default=4,
                    help="Hermite order of the step, integrate and serve modes (6: acc + jerk + snap, 6th-order corrector)")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="bodies of the oracle's CPU baseline sample (0 = skip)")
    ap.add_argument("--no-energy", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="step mode: serve the first R requests of the C4 stream after the "
                         "headline (closed batch, Poisson replay, one-at-a-time FP64 on the "
                         "first --baseline-requests) and report them as `serving` (0 = skip)")
    ap.add_argument("--mode", choices=["step", "sweep", "integrate", "serve", "copy", "groups"],
                    default="step",
                    help="step: the headline (default); sweep: active-block sizes 2^6..2^16 at "
                         "N=65536 (Salpeter), FP64 vs mixed, planned j-split vs none; integrate: "
                         "block-step integration of the N=2^20 Plummer sphere to t_end with energy "
                         "drift; serve: Poisson request stream through the continuous-batching server; "
                         "copy: a plain 1 GiB device copy (calibrates the HBM traffic counters); "
                         "groups: a cluster with hard binaries integrated directly and with the "
                         "pairs carried as centre-of-mass bodies (CPU pair work overlapped or not)")
    ap.add_argument("--t-end", type=float, default=0.125)
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--stream", choices=["c4", "c5"], default="c4")
    ap.add_argument("--slots", type=int, default=256)
    ap.add_argument("--baseline-requests", type=int, default=32)
    ap.add_argument("--lanes", type=int, default=None,
                    help="serve mode: force-plan lane target of every batched system "
                         "(0: the library default, sized for one system alone; default "
                         "for the C4 stream 2^18 at 4th order and 2^16 at 6th, the fastest "
                         "targets tried there; 0 for C5)")
    ap.add_argument("--groups", action="store_true",
                    help="serve mode, C5 stream: carry each primordial binary as one body at its "
                         "centre of mass, its relative orbit advanced on CPU threads")
    ap.add_argument("--capture-every", type=int, default=64,
                    help="serve mode, C5 stream with --groups: every that many block steps of "
                         "a system, single bodies of its block that are each other's nearest "
                         "neighbours, bound and weakly perturbed become a pair (0: off; "
                         "64 was the fastest of 4, 16, 32, 64, 128 and off)")
    ap.add_argument("--precisions", default="mixed,fp64",
                    help="serve mode, C5 stream: the precisions each request is served in")
    ap.add_argument("--pipes", type=int, default=1, choices=[1, 2],
                    help="serving: split the resident systems between this many contexts "
                         "(streams), stepped one after the other")
    ap.add_argument("--closed-only", action="store_true",
                    help="serve mode: the closed batch alone (no Poisson replay, baselines "
                         "or reruns), e.g. for a kernel trace")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.mode == "sweep":
        return mode_sweep(args)
    if args.mode == "integrate":
        return mode_integrate(args)
    if args.mode == "serve":
        return mode_serve(args)
    if args.mode == "copy":
        return mode_copy(args)
    if args.mode == "groups":
        return mode_groups(args)

    return mode_step(args)


def mode_step(args):
    """The headline: shared-step block steps with the whole system active."""
    import numpy as np
    import torch

    from paper_1411_5234_amd import _lib, inputs
    from paper_1411_5234_amd.nbody import (Context, Integrator, Integrator6, Params, Params6,
                                           System)

    h6 = args.order == 6
    flops = FLOPS_PER_INTERACTION6 if h6 else FLOPS_PER_INTERACTION
    n = args.n
    snap = inputs.plummer(n, args.seed)
    system = System.from_arrays(snap.x, snap.v, snap.m, device="cuda")
    ctx = Context(0)
    stream = ctx.stream
    if h6:
        p = Params6(eps=args.eps, precision=args.precision)
        it = Integrator6(ctx, system, p)
    else:
        p = Params(eps=args.eps, precision=args.precision)
        it = Integrator(ctx, system, p)
    it.startup()
    ctx.sync()
    dt0 = system.row("dt")
    h = float(dt0.min().item())
    # shared step: every body gets h (the smallest startup step), dt_max = h
    p.dt_max = h
    a3, j3 = it.acc.view(-1)[: 3 * n], it.jerk.view(-1)[: 3 * n]
    if h6:
        ctx.init_steps6(system, it.h6, a3, j3, it.snap.view(-1)[: 3 * n], p.eta_s, h, p.dt_min)
    else:
        ctx.init_steps(system, a3, j3, p.eta_s, h, p.dt_min)
    ctx.sync()

    E0 = None
    if not args.no_energy:
        E0 = ctx.energy(system, args.eps)[2]

    ev = []
    inter = 0

    def force(m, prec, plan=None):
        acc = it.acc.view(-1)[: 3 * m]
        jerk = it.jerk.view(-1)[: 3 * m]
        if h6:
            sn = it.snap.view(-1)[: 3 * m]
            ctx.force6_active(system, it.h6, it.i_idx, m, 0, n, p.eps, prec, acc, jerk, sn, plan)
            return acc, jerk, sn
        ctx.force_active(system, it.i_idx, m, 0, n, p.eps, prec, acc, jerk, plan)
        return acc, jerk

    def one_step(timed):
        nonlocal inter
        t_next, m = ctx.select_active(system, it.i_idx)
        if h6:
            ctx.predict6(system, it.h6, t_next)
        else:
            ctx.predict(system, t_next)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = force(m, p.precision)
        e1.record(stream)
        if h6:
            ctx.correct6(system, it.h6, it.i_idx, m, *out, t_next, p.eta, p.dt_max, p.dt_min)
        else:
            ctx.correct(system, it.i_idx, m, *out, t_next, p.eta, p.dt_max, p.dt_min)
        if timed:
            ev.append((e0, e1))
            inter += m * n
        return m

    for _ in range(args.warmup):
        one_step(False)
    ctx.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = []
    for _ in range(args.steps):
        ms.append(one_step(True))
    ctx.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    force_ms = [a.elapsed_time(b) for a, b in ev]
    value = inter / wall
    favg_s = float(np.mean(force_ms)) / 1e3
    per_launch = float(np.mean(ms)) * n
    achieved_tflops = flops * per_launch / favg_s / 1e12
    peak = PEAK_FP32_TFLOPS if args.precision != "fp64" else PEAK_FP64_TFLOPS

    extra = {}
    alt_sample = {}
    if ms[-1] == n:
        # the other precisions on the same predicted state and launch shape: one
        # warm-up and two HIP-event-timed force launches each
        alt = {}
        for prec in ("fp64", "ds", "mixed"):
            if prec == args.precision:
                continue
            force(n, prec)
            ctx.sync()
            best = float("inf")
            for _ in range(2):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                force(n, prec)
                e1.record(stream)
                ctx.sync()
                best = min(best, e0.elapsed_time(e1) / 1e3)
            alt[prec] = {"kernel_ms": best * 1e3, "interactions_per_s": n * n / best,
                         "tflops": flops * n * n / best / 1e12,
                         "plan": list(_lib.force_plan(n, n, prec))}
            if args.cpu_sample > 0:
                k = min(args.cpu_sample, n)
                alt_sample[prec] = (it.acc.view(-1)[: 3 * n].view(3, n)[:, :k].T.cpu().numpy(),
                                    it.jerk.view(-1)[: 3 * n].view(3, n)[:, :k].T.cpu().numpy())
        extra["other_precisions_same_state"] = alt
        # leave the results of the benchmarked precision in place for the CPU check
        force(n, args.precision)
        ctx.sync()
    if E0 is not None:
        E1 = ctx.energy(system, args.eps)[2]
        extra["energy_drift_over_timed_steps"] = abs(E1 - E0) / abs(E0)

    cpu = None
    if args.cpu_sample > 0:
        import oracle
        k = min(args.cpu_sample, n)
        st = system.state_numpy()
        il = np.arange(k, dtype=np.int64)
        # the oracle evaluates the sample from the same predicted j-set the last GPU step used
        tc = time.perf_counter()
        if h6:
            ap = it.h6.state_numpy()["ap"]
            oa, oj, osn = oracle.force6(st["xp"], st["vp"], ap, st["m"], args.eps, il)
        else:
            oa, oj = oracle.force(st["xp"], st["vp"], st["m"], args.eps, il)
        tcpu = time.perf_counter() - tc
        cpu = {"value": k * n / tcpu, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
               "kind": "oracle", "build": "gcc " + " ".join(oracle.CFLAGS),
               "sample": "%s of the first %d bodies against all %d predicted bodies (FP64, "
                         "compensated sums), %.1f s" % ("acc+jerk+snap" if h6 else "acc+jerk",
                                                         k, n, tcpu)}
        if ms[-1] == n:   # the last block was the whole system, in index order
            ga_all = it.acc.view(-1)[: 3 * n].view(3, n).T.cpu().numpy()
            gj_all = it.jerk.view(-1)[: 3 * n].view(3, n).T.cpu().numpy()
            ga, gj = ga_all[:k], gj_all[:k]
            ea = np.linalg.norm(ga - oa, axis=1) / np.linalg.norm(oa, axis=1)
            ej = np.linalg.norm(gj - oj, axis=1) / np.linalg.norm(oj, axis=1)
            extra["error_vs_oracle_sample"] = {
                "bodies": k, "acc_rel_max": float(ea.max()),
                "acc_rel_rms": float(np.sqrt((ea ** 2).mean())),
                "jerk_rel_max": float(ej.max()), "jerk_rel_rms": float(np.sqrt((ej ** 2).mean()))}
            if not h6:
                ssa, ssj = oracle.force_scale(st["xp"], st["vp"], st["m"], args.eps, il)
                extra["error_vs_oracle_sample"].update(accuracy_summary(ga, gj, oa, oj, ssa, ssj))
                top = top_kappa_bodies(n, args.seed, args.eps)
                if top is not None:
                    ta, tj = oracle.force(st["xp"], st["vp"], st["m"], args.eps, top)
                    tsa, tsj = oracle.force_scale(st["xp"], st["vp"], st["m"], args.eps, top)
                    extra["error_vs_oracle_top_kappa"] = {
                        "bodies": int(top.size),
                        "chosen": "the 64 largest sum|a_ij|/|a_i| and the 64 largest "
                                  "sum|jerk_ij|/|jerk_i| of a full oracle scan of the t = 0 state",
                        **accuracy_summary(ga_all[top], gj_all[top], ta, tj, tsa, tsj)}
            if h6:
                gs = it.snap.view(-1)[: 3 * n].view(3, n)[:, :k].T.cpu().numpy()
                ss = oracle.force6_scale(st["xp"], st["vp"], ap, st["m"], args.eps, il)
                es = np.linalg.norm(gs - osn, axis=1) / ss
                extra["error_vs_oracle_sample"]["snap_over_scale_max"] = float(es.max())
            # the other precisions' results on the same sample
            for prec, (pa, pj) in alt_sample.items():
                ea = np.linalg.norm(pa - oa, axis=1) / np.linalg.norm(oa, axis=1)
                ej = np.linalg.norm(pj - oj, axis=1) / np.linalg.norm(oj, axis=1)
                extra["other_precisions_same_state"][prec]["error_vs_oracle_sample"] = {
                    "acc_rel_max": float(ea.max()), "acc_rel_rms": float(np.sqrt((ea ** 2).mean())),
                    "jerk_rel_max": float(ej.max()),
                    "jerk_rel_rms": float(np.sqrt((ej ** 2).mean()))}
                if not h6 and prec != "fp64":
                    extra["other_precisions_same_state"][prec]["error_vs_oracle_sample"].update(
                        accuracy_summary(pa, pj, oa, oj, ssa, ssj))

    kname = "force%s_%s_kernel" % ("6" if h6 else "",
                                   "fp64" if args.precision == "fp64" else "mixed")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"mixed": "f64+f32", "ds": "f32x2+f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "plummer_n%d_eps%g_%s_hermite%d_shared_step_full_block"
                               % (n, args.eps, args.precision, args.order),
                   "n": n, "eps": args.eps, "precision": args.precision, "order": args.order,
                   "active_block": "m=N", "shared_step": h},
        "fp32_peak_frac": value * flops / (PEAK_FP32_TFLOPS * 1e12),
        "fp32_peak_frac_at_60_flops_convention": (
            value * FLOPS_CONVENTION4 / (PEAK_FP32_TFLOPS * 1e12) if not h6 else None),
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved_tflops / peak,
                     "traffic": TRAFFIC.get((_kernel_source_hash(args.order), args.precision, n,
                                             _lib.force_plan(n, n, args.precision))),
                     "kernel": kname,
                     "kernel_ms_avg": float(np.mean(force_ms)),
                     "flops_per_interaction": flops,
                     "interactions_per_launch": per_launch},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    if args.serving_requests > 0 and not h6 and args.precision == "mixed":
        # the serving half of the metric: a bounded sample of the C4 stream
        print("serving: first %d requests of the C4 stream" % args.serving_requests,
              file=sys.stderr, flush=True)
        sv = serving_runs(ctx, "c4", args.serving_requests, baseline=args.baseline_requests,
                          pipes=args.pipes)
        out["serving"] = {"workload": "c4: equal-mass Plummer, N log-uniform in [256, 32768], "
                                      "eps = 1e-3, to t = 1, first %d requests" % args.serving_requests,
                          "precision": "mixed", "lanes": default_lanes("c4", 4),
                          "pipes": args.pipes, **sv}
    ctx.close()
    print(json.dumps(out), flush=True)


ACC_GATE = 1e-6           # per-body relative error of the mixed path (acceleration and jerk)


def accuracy_summary(ga, gj, oa, oj, sa, sj):
    """Plain per-body relative errors |g - o| / |o|, the errors over the magnitude
    scales sum_j |a_ij| and sum_j |jerk_ij|, the share of bodies within the plain
    1e-6, and the cancellation factors kappa = scale / |o| of the worst bodies."""
    import numpy as np
    na, nj = np.linalg.norm(oa, axis=1), np.linalg.norm(oj, axis=1)
    ea = np.linalg.norm(ga - oa, axis=1) / na
    ej = np.linalg.norm(gj - oj, axis=1) / nj
    wa, wj = int(np.argmax(ea)), int(np.argmax(ej))
    return {"acc_rel_max": float(ea.max()), "jerk_rel_max": float(ej.max()),
            "acc_over_scale_max": float((np.linalg.norm(ga - oa, axis=1) / sa).max()),
            "jerk_over_scale_max": float((np.linalg.norm(gj - oj, axis=1) / sj).max()),
            "share_acc_rel_le_1e-6": float((ea <= ACC_GATE).mean()),
            "share_jerk_rel_le_1e-6": float((ej <= ACC_GATE).mean()),
            "share_both_rel_le_1e-6": float(((ea <= ACC_GATE) & (ej <= ACC_GATE)).mean()),
            "kappa_acc_of_worst_acc_body": float(sa[wa] / na[wa]),
            "kappa_jerk_of_worst_jerk_body": float(sj[wj] / nj[wj])}


def top_kappa_bodies(n, seed, eps):
    """Indices of the bodies with the largest cancellation factors of the N = 2^20
    Plummer sphere (seed 3, eps = 1e-4), as written by the oracle-only script
    tests/golden/make_kappa_plummer_2pow20.py; None for other workloads."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", "kappa_plummer_2pow20_seed3.json")
    if (n, seed, eps) != (1 << 20, 3, 1e-4) or not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    idx = rec["top_kappa_acc"]["index"] + rec["top_kappa_jerk"]["index"]
    return np.unique(np.asarray(idx, dtype=np.int64))


def _timed_force(ctx, system, idx, m, eps, precision, acc, jerk, plan=None, reps=5):
    import torch
    ctx.force_active(system, idx, m, 0, system.n, eps, precision, acc, jerk, plan)
    ctx.sync()
    best = float("inf")
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.force_active(system, idx, m, 0, system.n, eps, precision, acc, jerk, plan)
        e1.record(ctx.stream)
        ctx.sync()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    return best


def mode_copy(args):
    """Plain device-to-device copy of 1 GiB, three times: the calibration kernel for
    the FETCH_SIZE / WRITE_SIZE counters (each copy reads and writes 2^30 bytes)."""
    import torch
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / 3
    print(json.dumps({"mode": "copy", "bytes_read_per_copy": 1 << 30, "bytes_written_per_copy": 1 << 30,
                      "GB_per_s": 2 * (1 << 30) / dt / 1e9}), flush=True)


def mode_sweep(args):
    """Active-block sweep (the paper's Fig. 1 analogue): N = 65536 Salpeter cluster,
    eps = 1e-4, m = 2^6 .. 2^16 bodies (first m of a seeded permutation)."""
    import numpy as np
    import torch

    from paper_1411_5234_amd import _lib, inputs
    from paper_1411_5234_amd.nbody import Context, System
    n = 65536
    snap = inputs.plummer(n, 2, masses=inputs.salpeter_masses(n, 2))
    ctx = Context(0)
    system = System.from_arrays(snap.x, snap.v, snap.m)
    perm = np.random.default_rng(20).permutation(n)
    acc = torch.empty(3 * n, dtype=torch.float64, device="cuda")
    jerk = torch.empty_like(acc)
    rows = []
    for k in range(6, 17):
        m = 1 << k
        idx = torch.as_tensor(np.sort(perm[:m]).astype(np.int32), device="cuda")
        for prec in ("mixed", "fp64"):
            planned = _lib.force_plan(n, m, prec)
            t_plan = _timed_force(ctx, system, idx, m, 1e-4, prec, acc, jerk)
            t_one = _timed_force(ctx, system, idx, m, 1e-4, prec, acc, jerk, plan=(planned[0], 1, 1))
            rows.append({"m": m, "precision": prec, "plan": list(planned),
                         "interactions_per_s": m * n / t_plan,
                         "interactions_per_s_no_split": m * n / t_one,
                         "us": t_plan * 1e6, "us_no_split": t_one * 1e6})
            print("m=%6d %-5s plan %-12s %.3e int/s (%.1f us)   no split %.3e int/s (%.1f us)"
                  % (m, prec, planned, m * n / t_plan, t_plan * 1e6, m * n / t_one, t_one * 1e6),
                  file=sys.stderr, flush=True)
    ctx.close()
    print(json.dumps({"metric": "pair-interactions/s vs active-block size (N=65536 Salpeter)",
                      "mode": "sweep", "rows": rows}), flush=True)


def mode_integrate(args):
    """Block-step Hermite integration (order 4, or 6 with --order 6) of the N=2^20
    Plummer sphere to t_end."""
    import torch

    from paper_1411_5234_amd import inputs
    from paper_1411_5234_amd.nbody import (Context, Integrator, Integrator6, Params, Params6,
                                           System)
    n = args.n
    snap = inputs.plummer(n, args.seed)
    ctx = Context(0)
    system = System.from_arrays(snap.x, snap.v, snap.m)
    if args.order == 6:
        p = Params6(eps=args.eps, precision=args.precision)
        it = Integrator6(ctx, system, p)
    else:
        p = Params(eps=args.eps, precision=args.precision)
        it = Integrator(ctx, system, p)
    E0 = ctx.energy(system, args.eps)[2]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    it.startup()
    last = [time.perf_counter()]

    def progress(step_t, steps):
        now = time.perf_counter()
        if now - last[0] > 10:
            last[0] = now
            print("t=%.6f steps=%d interactions=%.3e wall=%.1fs" % (step_t, steps, it.interactions,
                                                                   now - t0), file=sys.stderr, flush=True)

    it.run(args.t_end, progress=progress)
    wall = time.perf_counter() - t0
    E1 = ctx.energy(system, args.eps)[2]
    ctx.close()
    out = {"metric": "pair-interactions/s over a block-step integration", "mode": "integrate",
           "value": it.interactions / wall, "unit": "pair-interactions/s",
           "config": {"workload": "plummer_n%d_eps%g_%s_hermite%d_to_t%g"
                                  % (n, args.eps, args.precision, args.order, args.t_end),
                      "n": n, "eps": args.eps, "precision": args.precision, "order": args.order,
                      "t_end": args.t_end,
                      "eta": p.eta, "eta_s": p.eta_s, "dt_max": p.dt_max},
           "flops_per_interaction": FLOPS_PER_INTERACTION6 if args.order == 6 else FLOPS_PER_INTERACTION,
           "block_steps": it.steps, "interactions": it.interactions, "wall_s": wall,
           "energy0": E0, "energy1": E1, "energy_drift": abs(E1 - E0) / abs(E0)}
    print(json.dumps(out), flush=True)


SERVE_SPECS = {
    "c4": dict(n_lo=256, n_hi=32768, eps=1e-3, t_end=1.0, kind="plummer", seed=4, base=4000),
    "c5": dict(n_lo=1024, n_hi=65536, eps=1e-5, t_end=0.125, kind="kroupa_binaries", seed=5,
               base=5000),
}


def default_lanes(stream, order):
    """Force-plan lane target of the batched systems: with up to 256 C4 systems
    resident the batch fills the GPU and shorter splits win (measured fastest:
    2^18 at 4th order, 2^16 at 6th); the C5 runs keep few systems resident, where
    the library default (one system fills the GPU) was faster."""
    return 0 if stream == "c5" else (1 << 16 if order == 6 else 1 << 18)


def serve_stream(stream, rate, count):
    from paper_1411_5234_amd import inputs
    spec = SERVE_SPECS[stream]
    return inputs.request_stream(count, spec["seed"], spec["n_lo"], spec["n_hi"], rate=rate,
                                 eps=spec["eps"], t_end=spec["t_end"], kind=spec["kind"],
                                 ic_seed_base=spec["base"])


def _progress():
    last = [time.perf_counter()]

    def progress(srv):
        now = time.perf_counter()
        if now - last[0] > 10:
            last[0] = now
            print("  iteration %d: %d resident, %d queued, %d done" % (
                srv.iterations, len(srv.slots), len(srv.queue), len(srv.results)),
                file=sys.stderr, flush=True)
    return progress


def serving_runs(ctx, stream, requests, precision="mixed", order=4, slots=256, lanes=None,
                 baseline=32, closed_only=False, pipes=1):
    """The first `requests` requests of a serving stream, served four ways:
    - closed batch: all arrive at t = 0 (saturated throughput);
    - Poisson replay in real time at 0.8 x the closed-batch rate;
    - one at a time in FP64 (the first `baseline` requests, one after another);
    - the same `baseline` requests through the batched server, for a like-for-like rate.
    Returns the summaries (solves/s, p50/p99 latency, interactions, energy errors)."""
    from paper_1411_5234_amd.serve import Server, summarize
    lanes = default_lanes(stream, order) if lanes is None else lanes
    progress = _progress()
    out = {}
    srv = Server(ctx, precision=precision, max_slots=slots, energy=True, order=order, lanes=lanes,
                 pipes=pipes)
    t0 = time.perf_counter()
    res = srv.run(serve_stream(stream, 0.0, requests), realtime=False, on_iteration=progress)
    out["closed_batch"] = summarize(res, time.perf_counter() - t0)
    print("closed batch: %s" % out["closed_batch"], file=sys.stderr, flush=True)
    if closed_only:
        return out
    rate = 0.8 * out["closed_batch"]["solves_per_s"]
    srv = Server(ctx, precision=precision, max_slots=slots, energy=True, order=order, lanes=lanes,
                 pipes=pipes)
    t0 = time.perf_counter()
    res = srv.run(serve_stream(stream, rate, requests), realtime=True, on_iteration=progress)
    out["poisson"] = summarize(res, time.perf_counter() - t0)
    out["poisson"]["arrival_rate_per_s"] = rate
    print("poisson at %.2f/s: %s" % (rate, out["poisson"]), file=sys.stderr, flush=True)
    k = min(baseline, requests)
    if k > 0:
        srv = Server(ctx, precision="fp64", max_slots=1, energy=True, order=order)
        t0 = time.perf_counter()
        res = srv.run(serve_stream(stream, 0.0, requests)[:k], realtime=False,
                      on_iteration=progress)
        out["one_at_a_time_fp64"] = summarize(res, time.perf_counter() - t0)
        out["one_at_a_time_fp64"]["requests_served"] = k
        print("one at a time fp64: %s" % out["one_at_a_time_fp64"], file=sys.stderr, flush=True)
        srv = Server(ctx, precision=precision, max_slots=slots, energy=True, order=order,
                     lanes=lanes, pipes=pipes)
        t0 = time.perf_counter()
        res = srv.run(serve_stream(stream, 0.0, requests)[:k], realtime=False)
        out["batched_same_requests"] = summarize(res, time.perf_counter() - t0)
        out["batched_same_requests"]["requests_served"] = k
    return out


def mode_serve(args):
    """Serve a request stream through the continuous-batching server.

    c4: equal-mass Plummer clusters, N log-uniform in [256, 32768], eps = 1e-3, to
    t = 1.  c5: Kroupa IMF with 10% binaries, N log-uniform in [1024, 65536],
    eps = 1e-5, to t = 1/8.  The stream is first served as a closed batch to
    measure saturated throughput, then replayed in real time with arrivals at
    0.8 x that rate; a one-at-a-time FP64 baseline serves the first
    --baseline-requests requests alone, one after another."""
    from paper_1411_5234_amd.nbody import Context
    from paper_1411_5234_amd.serve import Server
    if args.lanes is None:
        args.lanes = default_lanes(args.stream, args.order)
    if args.stream == "c5":
        return mode_serve_c5(args)
    spec = SERVE_SPECS[args.stream]
    ctx = Context(0)
    out = {"metric": "ensemble solves/s and p50/p99 latency", "mode": "serve",
           "config": {"workload": args.stream, "requests": args.requests, "slots": args.slots,
                      "precision": args.precision, "order": args.order, "lanes": args.lanes,
                      **{k: v for k, v in spec.items() if k != "base"}}}
    out.update(serving_runs(ctx, args.stream, args.requests, args.precision, args.order,
                            args.slots, args.lanes, args.baseline_requests, args.closed_only,
                            pipes=args.pipes))
    closed = out["closed_batch"]
    if args.closed_only:
        ctx.close()
        out["value"] = closed["solves_per_s"]
        out["unit"] = "solves/s"
        print(json.dumps(out), flush=True)
        return
    progress = _progress()
    worst = closed.get("energy_error_worst_request")
    if worst is not None:
        # the request with the largest energy error, served alone in FP64 and in the
        # run's precision: tells the integrator's error from the pair arithmetic's
        req = [q for q in serve_stream(args.stream, 0.0, args.requests) if q.rid == worst["rid"]]
        row = dict(worst)
        for prec in dict.fromkeys(("fp64", args.precision)):
            srv = Server(ctx, precision=prec, max_slots=1, energy=True, order=args.order,
                         lanes=args.lanes)
            r = srv.run(req, realtime=False)[0]
            row["energy_error_" + prec] = r.energy_error if r.error is None else r.error
        out["worst_request_alone"] = row
        print("worst request alone: %s" % row, file=sys.stderr, flush=True)
    ctx.close()
    out["value"] = out["poisson"]["solves_per_s"]
    out["unit"] = "solves/s"
    print(json.dumps(out), flush=True)


def mode_serve_c5(args):
    """The precision-stress stream (C5): Kroupa clusters with 10% of the bodies in
    primordial binaries, N log-uniform in [1024, 65536], eps = 1e-5, to t = 1/8.
    The first --requests requests are served as a closed batch in each precision of
    --precisions, directly (every body in the block-step system) or with --groups
    (each binary carried as one body at its centre of mass, its orbit advanced on
    CPU threads).  Reported: solves/s per precision and, per request, the energy
    error in each precision (grouped: the scheme's conserved quantity and the full
    N-body energy of the reconstructed members), with its distribution."""
    import numpy as np

    from paper_1411_5234_amd.nbody import Context
    from paper_1411_5234_amd.serve import Server, summarize
    spec = SERVE_SPECS["c5"]
    precs = [p for p in args.precisions.split(",") if p]
    reqs = serve_stream("c5", 0.0, args.requests)
    ctx = Context(0)
    out = {"metric": "ensemble solves/s and energy error per request, mixed vs FP64",
           "mode": "serve", "config": {"workload": "c5", "requests": args.requests,
                                       "slots": args.slots, "groups": args.groups,
                                       "capture_every": args.capture_every,
                                       "lanes": args.lanes, "precisions": precs,
                                       **{k: v for k, v in spec.items() if k != "base"}}}
    progress = _progress()
    per = {}
    for prec in precs:
        srv = Server(ctx, precision=prec, max_slots=args.slots, energy=True, lanes=args.lanes,
                     groups=args.groups, capture_every=args.capture_every)
        t0 = time.perf_counter()
        res = srv.run(reqs, realtime=False, on_iteration=progress)
        out["closed_batch_" + prec] = summarize(res, time.perf_counter() - t0)
        print("%s closed batch: %s" % (prec, out["closed_batch_" + prec]), file=sys.stderr,
              flush=True)
        per[prec] = {r.rid: r for r in res}
    rows = []
    for q in reqs:
        row = {"rid": q.rid, "n": q.n}
        for prec in precs:
            r = per[prec].get(q.rid)
            if r is None or r.error is not None:
                row["error_" + prec] = r.error if r is not None else "missing"
                continue
            row["pairs"] = r.pairs
            row["steps_" + prec] = r.steps
            if args.groups:
                row["returns_" + prec] = r.splits
                row["captures_" + prec] = r.captures
            row["energy_error_" + prec] = r.energy_error
            if args.groups:
                row["direct_energy_error_" + prec] = abs(r.direct1 - r.direct0) / abs(r.direct0)
        rows.append(row)
    out["energy_error_per_request"] = rows
    dist = {}
    for key in ["energy_error_" + p for p in precs] + (
            ["direct_energy_error_" + p for p in precs] if args.groups else []):
        vals = np.array([r[key] for r in rows if key in r])
        if vals.size:
            worst = max((r for r in rows if key in r), key=lambda r: r[key])
            dist[key] = {"requests": int(vals.size), "median": float(np.median(vals)),
                         "p90": float(np.quantile(vals, 0.9)), "max": float(vals.max()),
                         "worst_request": {"rid": worst["rid"], "n": worst["n"]}}
    if "mixed" in precs and "fp64" in precs:
        both = [r for r in rows if "energy_error_mixed" in r and "energy_error_fp64" in r]
        ratio = np.array([r["energy_error_mixed"] / max(r["energy_error_fp64"], 1e-300)
                          for r in both])
        if ratio.size:
            dist["mixed_over_fp64"] = {"median": float(np.median(ratio)),
                                       "min": float(ratio.min()), "max": float(ratio.max())}
    out["energy_error_distribution"] = dist
    ctx.close()
    out["value"] = out["closed_batch_" + precs[0]]["solves_per_s"]
    out["unit"] = "solves/s"
    print(json.dumps(out), flush=True)


def mode_groups(args):
    """Kroupa cluster of --n bodies (default 16384 here) with 10% of them in hard
    binaries (a log-uniform in [1e-4, 1e-3], thermal e), eps = 1e-5, to --t-end
    (default 1/64 here): integrated directly, then with the pairs carried as
    centre-of-mass bodies whose relative orbits advance on CPU threads.  Then, to
    8 x t_end, the grouped run with the CPU pair work overlapped with the GPU
    block steps against the same work run between them (best of two each)."""
    import numpy as np

    from paper_1411_5234_amd import inputs
    from paper_1411_5234_amd.groups import GroupedIntegrator
    from paper_1411_5234_amd.nbody import Context, Integrator, Params, System
    n = args.n if args.n != (1 << 20) else 16384
    t_end = args.t_end if args.t_end != 0.125 else 1.0 / 64
    eps = 1e-5
    s = inputs.with_binaries(n, 6, frac_members=0.1, a_lo=1e-4, a_hi=1e-3, imf="kroupa")
    npairs = s.meta["n_pairs"]
    pairs = [(2 * k, 2 * k + 1) for k in range(npairs)]
    ctx = Context(0)
    out = {"metric": "block steps, wall time and energy error with and without grouped pairs",
           "mode": "groups",
           "config": {"workload": "kroupa_binaries_n%d_eps%g_to_t%g" % (n, eps, t_end), "n": n,
                      "pairs": npairs, "a_range": [1e-4, 1e-3], "eps": eps, "t_end": t_end,
                      "precision": args.precision}}
    last = [time.perf_counter()]

    def progress(tag, t, steps):
        now = time.perf_counter()
        if now - last[0] > 10:
            last[0] = now
            print("  %s: t=%.6f steps=%d" % (tag, t, steps), file=sys.stderr, flush=True)

    # direct
    system = System.from_arrays(s.x, s.v, s.m)
    it = Integrator(ctx, system, Params(eps=eps, precision=args.precision))
    E0 = ctx.energy(system, eps)[2]
    t0 = time.perf_counter()
    it.startup()
    while True:
        t_next, m = ctx.select_active(system, it.i_idx)
        if t_next > t_end:
            break
        it._advance(t_next, m)
        progress("direct", t_next, it.steps)
    ctx.sync()
    wall = time.perf_counter() - t0
    E1 = ctx.energy(system, eps)[2]
    out["direct"] = {"block_steps": it.steps, "interactions": it.interactions, "wall_s": wall,
                     "energy_error": abs(E1 - E0) / abs(E0)}
    print("direct: %s" % out["direct"], file=sys.stderr, flush=True)
    del it, system
    def grouped(overlap, t_stop, per_period=32):
        gi = GroupedIntegrator(ctx, s.x, s.v, s.m, pairs, Params(eps=eps, precision=args.precision),
                               overlap=overlap, per_period=per_period)
        t0 = time.perf_counter()
        gi.startup()
        e0 = gi.energy()
        steps, inter = gi.run(t_stop)
        wall = time.perf_counter() - t0
        e1 = gi.energy()
        res = {"block_steps": steps, "interactions": inter, "wall_s": wall,
               "cpu_pair_advances": gi.cpu_pairs_advanced, "per_period": per_period,
               "scheme_energy_error": abs(e1 - e0) / abs(e0)}
        if overlap:
            res["host_blocked_on_pairs_s"] = gi.wait_seconds
        else:
            res["pair_advance_cpu_s"] = gi.cpu_seconds
        del gi
        return res

    grouped(True, t_end / 8)                       # warm-up (first launches, thread start)
    out["grouped"] = grouped(True, t_end)
    print("grouped: %s" % out["grouped"], file=sys.stderr, flush=True)
    # the CPU pair work overlapped with the GPU block steps, or run between them: a
    # longer run, best of two of each, alternating; with 32 substeps per orbital
    # period (the default) and with 256 (eight times the CPU work)
    t_long = 8 * t_end
    for per_period in (32, 256):
        runs = {True: [], False: []}
        for overlap in (True, False, True, False):
            runs[overlap].append(grouped(overlap, t_long, per_period))
        for overlap, key in ((True, "overlapped"), (False, "serialized")):
            best = min(runs[overlap], key=lambda r: r["wall_s"])
            best["t_end"] = t_long
            out["grouped_%s_%d" % (key, per_period)] = best
            print("%s %d: %s" % (key, per_period, best), file=sys.stderr, flush=True)
    ctx.close()
    out["speedup_grouped_vs_direct"] = out["direct"]["wall_s"] / out["grouped"]["wall_s"]
    for per_period in (32, 256):
        ser, ovl = out["grouped_serialized_%d" % per_period], out["grouped_overlapped_%d" % per_period]
        out["overlap_%d" % per_period] = {
            "wall_saved_s": ser["wall_s"] - ovl["wall_s"],
            "pair_advance_cpu_s": ser["pair_advance_cpu_s"],
            "hidden_fraction": 1.0 - ovl["host_blocked_on_pairs_s"] / max(ser["pair_advance_cpu_s"], 1e-12)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
