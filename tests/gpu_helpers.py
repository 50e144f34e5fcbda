"""Shared helpers of the GPU parity tests (call the HIP path through the C ABI)."""
import numpy as np
import torch

# Per-body gates.  FP64 path: |g - o| / |o| <= 1e-12 for acceleration and jerk.
# Mixed and DS paths, two gates:
#  - every body: |g - o| / S <= 1e-6, with S_a = sum_j |a_ij| and S_j = sum_j |jerk_ij|
#    the magnitude scales of the pair sums;
#  - every body whose cancellation factor kappa = S / |o| is at most KAPPA_PLAIN:
#    the plain |g - o| / |o| <= 1e-6.
# Why both: each FP32 pair term carries a few units of FP32 rounding (2^-24 =
# 6e-8), so |g - o| is a few 1e-8 of the largest terms, and the plain relative
# error grows with kappa.  An FP32 emulation of the kernel's arithmetic on 4800
# bodies of the N = 2^20 Plummer sphere found |g - o| / S up to 4.8e-7 (jerk) and
# 2.9e-7 (acceleration), and plain errors up to 4.5e-6 on bodies with kappa_j ~ 160;
# with only the mandated FP32 rounding of r_j - r_i (and every later operation in
# FP64) the worst of them still reaches 1.4e-6.  Every emulated body with
# kappa_a <= 10 kept the plain acceleration error <= 3.4e-7, and every one with
# kappa_j <= 5 the plain jerk error <= 6.9e-7.
# The jerk gates of the mixed and DS paths also allow the one error that does not
# come from the pair arithmetic: the velocity differences are formed from FP32
# copies of the predicted velocities (Sec. 2 item 4 keeps only the position
# differences and the sums in FP64), which moves each jerk term by at most
# 2 u m_j (|v_i| + |v_j|) / s^(3/2) (tests/test_fp32_floor.py derives the bound and
# shows a C5 binary member at 1.03e-6 from that rounding alone).  Both jerk gates
# are applied to the error less that bound, summed over j.
KAPPA_PLAIN = {"acc": 10.0, "jerk": 5.0}
U32 = 2.0 ** -24
TOL = {"fp64": 1e-12, "mixed": 1e-6, "ds": 1e-6}
# Snap (6th order): |g - o| / S_s with S_s = sum_j |snap_ij|.  A pair's snap term
# passes through about a dozen FP32 roundings (the hardware reciprocal square root,
# mu, alpha, beta, u and the three-part snap term) before joining an FP32 run sum
# of up to 32 terms, so its error is bounded by about 32 u = 32 * 2^-24 = 1.9e-6
# of S_s; a CPU emulation of the same FP32 operations reaches 0.84e-6 on the
# N = 1024 Plummer sphere.
TOL_SNAP = {"fp64": 1e-12, "mixed": 2e-6, "ds": 2e-6}


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


def velocity_bound(orc, x, v, m, eps, ilist, j0=0, j1=None):
    """Per listed body: 2 u sum_{j != i} m_j (|v_i| + |v_j|) / (|r_ij|^2 + eps^2)^(3/2)
    over j in [j0, j1), the most the FP32 rounding of the velocities can move its
    jerk."""
    return 2.0 * U32 * orc.velocity_scale(x, v, m, eps, ilist, j0, j1)


def plain_gate(tag, g, o, scale, kmax, tol=1e-6, allow=None):
    """Assert |g - o| / |o| <= tol for every body with scale / |o| <= kmax, and
    |g - o| / scale <= tol for every body, with |g - o| less `allow` (a bound on an
    error from outside the pair arithmetic, none by default); print both and the
    share of all bodies within the plain tol."""
    no = np.linalg.norm(o, axis=1)
    raw = np.linalg.norm(g - o, axis=1)
    err = raw if allow is None else np.maximum(raw - allow, 0.0)
    plain, over = err / no, err / scale
    kappa = scale / no
    low = kappa <= kmax
    rp = raw / no
    print("   %s: plain max %.3e (kappa %.1f), within 1e-6: %d/%d, /scale max %.3e | gated%s: "
          "kappa<=%g plain max %.3e, /scale max %.3e" % (
              tag, rp.max(), kappa[np.argmax(rp)], int((rp <= tol).sum()), rp.size,
              (raw / scale).max(), "" if allow is None else " (less the velocity bound)", kmax,
              plain[low].max(initial=0), over.max()), flush=True)
    assert over.max(initial=0) <= tol, (tag, over.max())
    assert plain[low].max(initial=0) <= tol, (tag, plain[low].max())


def check(orc, precision, ga, gj, x, v, m, eps, ilist=None, j0=0, j1=None, tag=""):
    """Compare GPU acc/jerk of bodies `ilist` with the oracle under the gates above."""
    oa, oj = orc.force(x, v, m, eps, ilist, j0, j1)
    keep = np.linalg.norm(oa, axis=1) > 0
    ea, ej = report(tag + " " + precision, ga[keep], gj[keep], oa[keep], oj[keep])
    if precision == "fp64":
        assert ea.max(initial=0) <= TOL["fp64"] and ej.max(initial=0) <= TOL["fp64"], (ea.max(), ej.max())
    else:
        sa, sj = orc.force_scale(x, v, m, eps, ilist, j0, j1)
        il = np.arange(len(m)) if ilist is None else np.asarray(ilist)
        vb = velocity_bound(orc, x, v, m, eps, il[keep], j0, j1)
        plain_gate("acc", ga[keep], oa[keep], sa[keep], KAPPA_PLAIN["acc"], TOL[precision])
        plain_gate("jerk", gj[keep], oj[keep], sj[keep], KAPPA_PLAIN["jerk"], TOL[precision],
                   allow=vb)
    return oa, oj


# ---- 6th order -------------------------------------------------------------------

def device_system6(x, v, m, ap, fp32=True):
    """A System whose predicted set is (x, v) and a Hermite6 whose predicted
    acceleration is `ap` (FP64 and FP32 copies)."""
    from paper_1411_5234_amd.nbody import Hermite6
    sys = device_system(x, v, m, fp32)
    h6 = Hermite6(sys, fp32_copies=fp32)
    if sys.n:
        h6.buf64[6:9, : sys.n] = torch.from_numpy(np.ascontiguousarray(np.asarray(ap).T)).cuda()
        if fp32:
            h6.buf32[:, : sys.n] = h6.buf64[6:9, : sys.n].float()
    return sys, h6


def gpu_force6(ctx, sys, h6, eps, precision, ilist=None, j0=0, j1=None, plan=None):
    n = sys.n
    m = n if ilist is None else len(ilist)
    idx = None if ilist is None else torch.as_tensor(np.asarray(ilist, dtype=np.int32), device="cuda")
    out = [torch.full((3 * max(m, 1),), np.nan, dtype=torch.float64, device="cuda") for _ in range(3)]
    ctx.force6_active(sys, h6, idx, m, j0, n if j1 is None else j1, eps, precision, *out, plan=plan)
    ctx.sync()
    return tuple(o[: 3 * m].view(3, m).T.cpu().numpy() for o in out)


def check6(orc, precision, g, x, v, ap, m, eps, ilist=None, j0=0, j1=None, tag=""):
    """Compare GPU (acc, jerk, snap) with the oracle.  FP64: relative acceleration
    and jerk errors per body.  Mixed and DS: acceleration, jerk and snap errors over
    the magnitude scale sum_j |term_ij| of each sum (each can be a sum of terms much
    larger than the result), gated by TOL and TOL_SNAP."""
    ga, gj, gs = g
    oa, oj, os_ = orc.force6(x, v, ap, m, eps, ilist, j0, j1)
    keep = np.linalg.norm(oa, axis=1) > 0
    ea = rel_err(ga[keep], oa[keep])
    sa, sj = orc.force_scale(x, v, m, eps, ilist, j0, j1)
    na = np.linalg.norm(ga[keep] - oa[keep], axis=1) / sa[keep]
    ss = orc.force6_scale(x, v, ap, m, eps, ilist, j0, j1)
    vb = None
    if precision != "fp64":
        il = np.arange(len(m)) if ilist is None else np.asarray(ilist)
        vb = velocity_bound(orc, x, v, m, eps, il[keep], j0, j1)
    dj = np.linalg.norm(gj[keep] - oj[keep], axis=1)
    nj = (dj if vb is None else np.maximum(dj - vb, 0.0)) / sj[keep]
    ns = np.linalg.norm(gs[keep] - os_[keep], axis=1) / ss[keep]
    es = rel_err(gs[keep], os_[keep])
    print("%s %s: acc rel max %.3e, acc/scale max %.3e | jerk/scale max %.3e | snap/scale max "
          "%.3e (snap rel max %.3e)" % (tag, precision, ea.max(initial=0), na.max(initial=0),
                                        nj.max(initial=0), ns.max(initial=0), es.max(initial=0)),
          flush=True)
    tol = TOL[precision]
    assert (ea if precision == "fp64" else na).max(initial=0) <= tol
    assert nj.max(initial=0) <= tol, nj.max()
    if precision != "fp64":
        plain_gate("acc", ga[keep], oa[keep], sa[keep], KAPPA_PLAIN["acc"], tol)
        plain_gate("jerk", gj[keep], oj[keep], sj[keep], KAPPA_PLAIN["jerk"], tol, allow=vb)
    assert ns.max(initial=0) <= TOL_SNAP[precision], ns.max()
    if precision == "fp64":
        ej = rel_err(gj[keep], oj[keep])
        assert ej.max(initial=0) <= tol, ej.max()
    assert np.all(ga[~keep] == 0.0) and np.all(gj[~keep] == 0.0) and np.all(gs[~keep] == 0.0)
    return oa, oj, os_
