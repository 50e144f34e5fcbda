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
PEAK_FP32_TFLOPS = 157.3     # MI355X dense FP32 vector (256 CU x 2.4 GHz x 256 flop/clk)
PEAK_FP64_TFLOPS = 78.6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=1 << 20)
    ap.add_argument("--eps", type=float, default=1e-4)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--seed", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="bodies of the oracle's CPU baseline sample (0 = skip)")
    ap.add_argument("--no-energy", action="store_true")
    return ap.parse_args()


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1411_5234_amd import inputs
    from paper_1411_5234_amd.nbody import Context, Integrator, Params, System

    n = args.n
    snap = inputs.plummer(n, args.seed)
    system = System.from_arrays(snap.x, snap.v, snap.m, device="cuda")
    ctx = Context(0)
    stream = ctx.stream
    p = Params(eps=args.eps, precision=args.precision)
    it = Integrator(ctx, system, p)
    it.startup()
    ctx.sync()
    dt0 = system.row("dt")
    h = float(dt0.min().item())
    # shared step: every body gets h (the smallest startup step), dt_max = h
    p.dt_max = h
    ctx.init_steps(system, it.acc.view(-1)[: 3 * n], it.jerk.view(-1)[: 3 * n], p.eta_s, h, p.dt_min)
    ctx.sync()

    E0 = None
    if not args.no_energy:
        E0 = ctx.energy(system, args.eps)[2]

    ev = []
    force_ms = []
    inter = 0

    def one_step(timed):
        nonlocal inter
        t_next, m = ctx.select_active(system, it.i_idx)
        ctx.predict(system, t_next)
        acc = it.acc.view(-1)[: 3 * m]
        jerk = it.jerk.view(-1)[: 3 * m]
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        ctx.force_active(system, it.i_idx, m, 0, n, p.eps, p.precision, acc, jerk)
        e1.record(stream)
        ctx.correct(system, it.i_idx, m, acc, jerk, t_next, p.eta, p.dt_max, p.dt_min)
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
    achieved_tflops = FLOPS_PER_INTERACTION * per_launch / favg_s / 1e12
    peak = PEAK_FP32_TFLOPS if args.precision == "mixed" else PEAK_FP64_TFLOPS

    extra = {}
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
        oa, oj = oracle.force(st["xp"], st["vp"], st["m"], args.eps, il)
        tcpu = time.perf_counter() - tc
        ga = it.acc.view(-1)[: 3 * n].view(3, n)[:, :k].T.cpu().numpy()
        gj = it.jerk.view(-1)[: 3 * n].view(3, n)[:, :k].T.cpu().numpy()
        ea = np.linalg.norm(ga - oa, axis=1) / np.linalg.norm(oa, axis=1)
        ej = np.linalg.norm(gj - oj, axis=1) / np.linalg.norm(oj, axis=1)
        cpu = {"value": k * n / tcpu, "unit": "pair-interactions/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "acc+jerk of the first %d bodies against all %d predicted bodies (FP64, "
                         "compensated sums), %.1f s" % (k, n, tcpu)}
        extra["error_vs_oracle_sample"] = {
            "bodies": k, "acc_rel_max": float(ea.max()), "acc_rel_rms": float(np.sqrt((ea ** 2).mean())),
            "jerk_rel_max": float(ej.max()), "jerk_rel_rms": float(np.sqrt((ej ** 2).mean()))}

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
        "dtype": "f64+f32" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "plummer_n%d_eps%g_%s_shared_step_full_block" % (n, args.eps, args.precision),
                   "n": n, "eps": args.eps, "precision": args.precision, "active_block": "m=N",
                   "shared_step": h},
        "fp32_peak_frac": value * FLOPS_PER_INTERACTION / (PEAK_FP32_TFLOPS * 1e12),
        "roofline": {"bound": "alu", "achieved": achieved_tflops, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved_tflops / peak, "traffic": None,
                     "kernel": "force_%s_kernel" % args.precision,
                     "kernel_ms_avg": float(np.mean(force_ms)),
                     "flops_per_interaction": FLOPS_PER_INTERACTION,
                     "interactions_per_launch": per_launch},
        "cpu_baseline": cpu,
    }
    out.update(extra)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
