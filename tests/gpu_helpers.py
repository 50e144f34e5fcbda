"""Shared helpers of the GPU parity tests (call the HIP path through the C ABI)."""
import numpy as np
import torch

# Per-body gates.  FP64 path: |g - o| / |o| <= 1e-12 for acceleration and jerk.
# Mixed path: acceleration |g - o| / |o| <= 1e-6; jerk |g - o| / S_j <= 1e-6 with
# S_j = sum_j |jerk_ij| (FP32 pair terms carry a few ulp of error each, and the
# jerk of a body can be a sum of terms up to ~60x larger than the result).
TOL = {"fp64": 1e-12, "mixed": 1e-6}


def device_system(x, v, m, fp32=True):
    from paper_1411_5234_amd.nbody import System
    return System.from_arrays(x, v, m, device="cuda", fp32_copies=fp32)


def gpu_force(ctx, sys, eps, precision, ilist=None, j0=0, j1=None, plan=None):
    n = sys.n
    m = n if ilist is None else len(ilist)
    idx = None if ilist is None else torch.as_tensor(np.asarray(ilist, dtype=np.int32), device="cuda")
    acc = torch.full((3 * max(m, 1),), np.nan, dtype=torch.float64, device="cuda")
    jerk = torch.full((3 * max(m, 1),), np.nan, dtype=torch.float64, device="cuda")
    ctx.force_active(sys, idx, m, j0, n if j1 is None else j1, eps, precision, acc, jerk, plan)
    ctx.sync()
    a = acc[: 3 * m].view(3, m).T.cpu().numpy()
    j = jerk[: 3 * m].view(3, m).T.cpu().numpy()
    return a, j


def rel_err(g, o):
    return np.linalg.norm(g - o, axis=1) / np.linalg.norm(o, axis=1)


def report(tag, g_a, g_j, o_a, o_j):
    ea, ej = rel_err(g_a, o_a), rel_err(g_j, o_j)
    if ea.size == 0:
        print("%s: no bodies with a non-zero force" % tag, flush=True)
        return ea, ej
    line = "%s: acc max %.3e p99.9 %.3e rms %.3e | jerk max %.3e p99.9 %.3e rms %.3e" % (
        tag, ea.max(), np.quantile(ea, 0.999), np.sqrt((ea ** 2).mean()),
        ej.max(), np.quantile(ej, 0.999), np.sqrt((ej ** 2).mean()))
    print(line, flush=True)
    return ea, ej


def check(orc, precision, ga, gj, x, v, m, eps, ilist=None, j0=0, j1=None, tag=""):
    """Compare GPU acc/jerk of bodies `ilist` with the oracle under the gates above."""
    oa, oj = orc.force(x, v, m, eps, ilist, j0, j1)
    keep = np.linalg.norm(oa, axis=1) > 0
    ea, ej = report(tag + " " + precision, ga[keep], gj[keep], oa[keep], oj[keep])
    if precision == "fp64":
        assert ea.max(initial=0) <= TOL["fp64"] and ej.max(initial=0) <= TOL["fp64"], (ea.max(), ej.max())
    else:
        sa, sj = orc.force_scale(x, v, m, eps, ilist, j0, j1)
        nj = np.linalg.norm(gj[keep] - oj[keep], axis=1) / sj[keep]
        print("   mixed jerk error / sum|jerk_ij|: max %.3e" % nj.max(initial=0), flush=True)
        assert ea.max(initial=0) <= TOL["mixed"], ea.max()
        assert nj.max(initial=0) <= TOL["mixed"], nj.max()
    return oa, oj
