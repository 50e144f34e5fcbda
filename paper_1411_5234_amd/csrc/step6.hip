// Predictor, corrector and startup of the 6th-order Hermite scheme (the
// integrator of the paper's HiGPUs, Sec. 2 item 1), over item tables like the
// 4th-order kernels.  All FP64; one thread per body (predictor, startup) or per
// active body (corrector).
#include "nb_internal.h"
#include "launch.h"

namespace nbk {

// Every body to the block time: position to the crackle term, velocity and
// acceleration (the acceleration is what the snap of the pair sum needs).  The
// block time is the item's t_next, or, with sel (the device selection results of
// the same items), sel[k].t_next when that is not past the item's t_next field
// (then its horizon), as in the 4th-order predictor.
__global__ __launch_bounds__(WG) void predict6_kernel(const Item *items, const int64_t *starts,
                                                      int n_items, const SelResult *sel)
{
    const int k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[k];
    const int64_t i = ((int64_t)blockIdx.x - starts[k]) * WG + threadIdx.x;
    const nb_system &s = p.s;
    const nb_hermite6 &h = p.h6;
    double tn = p.t_next;
    if (sel) {
        tn = sel[k].t_next;
        if (!(tn <= p.t_next))
            return;
    }
    if (i >= s.n)
        return;
    const double d = tn - s.t[i];
    // Taylor coefficients d^n / n!
    const double c2 = d * d * 0.5, c3 = c2 * d * (1.0 / 3.0), c4 = c3 * d * 0.25,
                 c5 = c4 * d * 0.2;
    const double *x[3] = {s.x, s.y, s.z}, *v[3] = {s.vx, s.vy, s.vz};
    const double *a[3] = {s.ax, s.ay, s.az}, *j[3] = {s.jx, s.jy, s.jz};
    const double *sn[3] = {h.sx, h.sy, h.sz}, *cr[3] = {h.cx, h.cy, h.cz};
    double *xp[3] = {s.xp, s.yp, s.zp}, *vp[3] = {s.vxp, s.vyp, s.vzp};
    double *ap[3] = {h.axp, h.ayp, h.azp};
    float *vp32[3] = {s.vxp32, s.vyp32, s.vzp32}, *ap32[3] = {h.axp32, h.ayp32, h.azp32};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double vi = v[c][i], ai = a[c][i], ji = j[c][i], si = sn[c][i], ci = cr[c][i];
        xp[c][i] = x[c][i] + vi * d + ai * c2 + ji * c3 + si * c4 + ci * c5;
        const double pv = vi + ai * d + ji * c2 + si * c3 + ci * c4;
        const double pa = ai + ji * d + si * c2 + ci * c3;
        vp[c][i] = pv;
        ap[c][i] = pa;
        if (s.vxp32) vp32[c][i] = (float)pv;
        if (h.axp32) ap32[c][i] = (float)pa;
    }
    if (s.m32)
        s.m32[i] = (float)s.m[i];
}

hipError_t launch_predict6(const Table &t, const SelResult *sel, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(predict6_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items,
                       t.starts, t.n, sel);
    return hipGetLastError();
}

__device__ __forceinline__ double len3(const double (&u)[3])
{
    return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

// Corrector of the active bodies.  The two-point quadratures use (a, j, s) at
// both ends of the step; the crackle at the step's end is that of the degree-5
// polynomial matching (a, j, s) at both ends, written out in closed form.  New
// step: the lowest generalized Aarseth form with that crackle,
// eta (sqrt(|a||s|) + |j|) / (sqrt(|j||c|) + |s|), which anticipates approaching
// encounters, floored at one eighth of the form with |j|^2/|a| in place of the
// crackle term (computed derivatives only), so that rounding noise in the
// interpolated crackle cannot drive the step down; kept a power of two as in
// the 4th-order corrector.
__global__ __launch_bounds__(WG) void correct6_kernel(const Item *items, const int64_t *starts,
                                                      int n_items, double eta, double dt_max,
                                                      double dt_min)
{
    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int64_t k = ((int64_t)blockIdx.x - starts[it_k]) * WG + threadIdx.x;
    const int64_t m = p.m;
    if (k >= m)
        return;
    const nb_system &s = p.s;
    const nb_hermite6 &hh = p.h6;
    const int64_t i = p.i_idx ? (int64_t)p.i_idx[k] : k;
    if (i < 0 || i >= s.n) {
        atomicOr(p.status, (int)NBK_EINDEX);
        return;
    }
    const double t_next = p.t_next;
    const double h = t_next - s.t[i];
    const double h2 = h * h, h3 = h2 * h;
    const double ih = 1.0 / h, ih3 = ih * ih * ih;
    double *x[3] = {s.x, s.y, s.z}, *v[3] = {s.vx, s.vy, s.vz};
    double *a[3] = {s.ax, s.ay, s.az}, *j[3] = {s.jx, s.jy, s.jz};
    double *sn[3] = {hh.sx, hh.sy, hh.sz}, *cr[3] = {hh.cx, hh.cy, hh.cz};
    double a1v[3], j1v[3], s1v[3], c1v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a0 = a[c][i], j0 = j[c][i], s0 = sn[c][i];
        const double a1 = p.acc[c * m + k], j1 = p.jerk[c * m + k], s1 = p.snap[c * m + k];
        const double v0 = v[c][i];
        const double v1 = v0 + 0.5 * h * (a0 + a1) - 0.1 * h2 * (j1 - j0) +
                          (h3 / 120.0) * (s0 + s1);
        const double x1 = x[c][i] + 0.5 * h * (v0 + v1) - 0.1 * h2 * (a1 - a0) +
                          (h3 / 120.0) * (j0 + j1);
        const double da = a0 - a1;
        c1v[c] = -3.0 * (20.0 * da + h2 * (s0 - 3.0 * s1) + h * (8.0 * j0 + 12.0 * j1)) * ih3;
        x[c][i] = x1;
        v[c][i] = v1;
        a[c][i] = a1;
        j[c][i] = j1;
        sn[c][i] = s1;
        cr[c][i] = c1v[c];
        a1v[c] = a1; j1v[c] = j1; s1v[c] = s1;
    }
    const double an = len3(a1v), jn = len3(j1v), sN = len3(s1v);
    const double num = sqrt(an * sN) + jn;
    const double den_d = sN + (an > 0.0 ? jn * jn / an : 0.0);
    const double den_c = sN + sqrt(jn * len3(c1v));
    const double dt_d = den_d > 0.0 ? eta * (num / den_d) : INFINITY;
    double dta = den_c > 0.0 ? eta * (num / den_c) : INFINITY;
    if (dta < 0.125 * dt_d)
        dta = 0.125 * dt_d;
    int err = 0;
    if (isnan(dta) || !isfinite(an) || !isfinite(jn) || !isfinite(sN))
        err |= NBK_ENAN;
    double step = h;
    if (step > dta) {
        while (step > dta && step >= dt_min)
            step *= 0.5;
    } else if (dta >= 2.0 * h && 2.0 * h <= dt_max) {
        const double q = t_next / (2.0 * h);   // exact: 2h is a power of two
        if (q == floor(q))
            step = 2.0 * h;
    }
    if (step < dt_min)
        err |= NBK_ERANGE;
    s.t[i] = t_next;
    s.dt[i] = step;
    if (err)
        atomicOr(p.status, err);
}

hipError_t launch_correct6(const Table &t, double eta, double dt_max, double dt_min,
                           hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(correct6_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items,
                       t.starts, t.n, eta, dt_max, dt_min);
    return hipGetLastError();
}

// Startup: store acceleration, jerk and snap, zero the crackle, and take the
// largest power of two not above min(eta_s (sqrt(|a||s|) + |j|) / (|s| +
// |j|^2/|a|), dt_max): no crackle exists yet, and the snap shows a neighbour
// that is already close.
__global__ __launch_bounds__(WG) void init_steps6_kernel(const Item *items, const int64_t *starts,
                                                         int n_items, double eta_s, double dt_max,
                                                         double dt_min)
{
    const int k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[k];
    const int64_t i = ((int64_t)blockIdx.x - starts[k]) * WG + threadIdx.x;
    const nb_system &s = p.s;
    const nb_hermite6 &h = p.h6;
    const int64_t n = s.n;
    if (i >= n)
        return;
    double *a[3] = {s.ax, s.ay, s.az}, *j[3] = {s.jx, s.jy, s.jz};
    double *sn[3] = {h.sx, h.sy, h.sz}, *cr[3] = {h.cx, h.cy, h.cz};
    double av[3], jv[3], sv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        av[c] = p.acc[c * n + i];
        jv[c] = p.jerk[c * n + i];
        sv[c] = p.snap[c * n + i];
        a[c][i] = av[c];
        j[c][i] = jv[c];
        sn[c][i] = sv[c];
        cr[c][i] = 0.0;
    }
    const double an = len3(av), jn = len3(jv), sN = len3(sv);
    int err = 0;
    if (!isfinite(an) || !isfinite(jn) || !isfinite(sN))
        err |= NBK_ENAN;
    const double top = sqrt(an * sN) + jn, bottom = sN + (an > 0.0 ? jn * jn / an : 0.0);
    double want = bottom > 0.0 ? eta_s * (top / bottom) : dt_max;
    if (want > dt_max)
        want = dt_max;
    double step = dt_max;
    while (step > want && step >= dt_min)
        step *= 0.5;
    if (step < dt_min)
        err |= NBK_ERANGE;
    s.t[i] = 0.0;
    s.dt[i] = step;
    if (err)
        atomicOr(p.status, err);
}

hipError_t launch_init_steps6(const Table &t, double eta_s, double dt_max, double dt_min,
                              hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_steps6_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items,
                       t.starts, t.n, eta_s, dt_max, dt_min);
    return hipGetLastError();
}

}  // namespace nbk
