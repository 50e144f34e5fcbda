// Block-time-step kernels (Sec. 2 items 1-2 of the paper): active-block
// selection, Hermite-4 predictor for all bodies, corrector plus new
// power-of-two step for the active block, and the startup step.  All FP64.
// These are memory- or latency-bound one-pass kernels.
#include "nb_internal.h"

namespace nbk {

// ---- selection ---------------------------------------------------------------
// Pass 1: per-workgroup minimum of t + dt over a contiguous slice.
// Pass 2: every workgroup reduces the per-workgroup minima to t_next (identical
//         arithmetic in every workgroup) and counts its bodies due at t_next.
// Pass 3: every workgroup adds the counts of the workgroups before it and writes
//         its due bodies' indices in ascending order (ordered compaction with a
//         wave ballot and an LDS prefix over the four waves).

struct SelShape {
    int blocks;
    int64_t slice;  // bodies per workgroup
};

static SelShape sel_shape(int64_t n)
{
    int64_t blocks = (n + 4095) / 4096;
    if (blocks < 1) blocks = 1;
    if (blocks > SEL_BLOCKS) blocks = SEL_BLOCKS;
    int64_t slice = (n + blocks - 1) / blocks;
    slice = (slice + WG - 1) / WG * WG;
    blocks = (n + slice - 1) / slice;
    if (blocks < 1) blocks = 1;
    return {(int)blocks, slice};
}

__device__ double wg_min(double v, double *lds)
{
    for (int off = 32; off >= 1; off >>= 1)
        v = fmin(v, __shfl_xor(v, off, 64));
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    v = lds[0];
    for (int k = 1; k < WG / 64; ++k) v = fmin(v, lds[k]);
    return v;
}

__device__ int wg_sum_int(int v, int *lds)
{
    for (int off = 32; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, 64);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    __syncthreads();
    if (l == 0) lds[w] = v;
    __syncthreads();
    int t = 0;
    for (int k = 0; k < WG / 64; ++k) t += lds[k];
    return t;
}

__global__ __launch_bounds__(WG) void select_min_kernel(const double *t, const double *dt,
                                                        int64_t n, int64_t slice, nb_small *sm)
{
    __shared__ double lds[WG / 64];
    const int64_t b0 = (int64_t)blockIdx.x * slice;
    const int64_t b1 = min(b0 + slice, n);
    double v = INFINITY;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += WG)
        v = fmin(v, t[i] + dt[i]);
    v = wg_min(v, lds);
    if (threadIdx.x == 0)
        sm->blockval[blockIdx.x] = v;
}

__device__ double global_tnext(const nb_small *sm, int nblocks, double *lds)
{
    double v = INFINITY;
    for (int k = threadIdx.x; k < nblocks; k += WG)
        v = fmin(v, sm->blockval[k]);
    return wg_min(v, lds);
}

__global__ __launch_bounds__(WG) void select_count_kernel(const double *t, const double *dt,
                                                          int64_t n, int64_t slice, int nblocks,
                                                          nb_small *sm)
{
    __shared__ double lds[WG / 64];
    __shared__ int ldi[WG / 64];
    const double tn = global_tnext(sm, nblocks, lds);
    const int64_t b0 = (int64_t)blockIdx.x * slice;
    const int64_t b1 = min(b0 + slice, n);
    int c = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += WG)
        c += (t[i] + dt[i] == tn) ? 1 : 0;
    c = wg_sum_int(c, ldi);
    if (threadIdx.x == 0) {
        sm->blockcnt[blockIdx.x] = c;
        if (blockIdx.x == 0)
            sm->t_next = tn;
    }
}

__global__ __launch_bounds__(WG) void select_scatter_kernel(const double *t, const double *dt,
                                                            int64_t n, int64_t slice, int nblocks,
                                                            nb_small *sm, int32_t *i_idx)
{
    __shared__ int ldi[WG / 64];
    __shared__ int wave_off[WG / 64];
    const double tn = sm->t_next;
    int before = 0;
    for (int k = threadIdx.x; k < (int)blockIdx.x; k += WG)
        before += sm->blockcnt[k];
    int base = wg_sum_int(before, ldi);
    const int64_t b0 = (int64_t)blockIdx.x * slice;
    const int64_t b1 = min(b0 + slice, n);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    for (int64_t r = b0; r < b1; r += WG) {
        const int64_t i = r + threadIdx.x;
        const bool due = (i < b1) && (t[i] + dt[i] == tn);
        const unsigned long long mask = __ballot(due);
        const int in_wave = __popcll(mask & ((1ull << l) - 1ull));
        __syncthreads();
        if (l == 0) wave_off[w] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int k = 0; k < w; ++k) off += wave_off[k];
        if (due)
            i_idx[off + in_wave] = (int32_t)i;
        int round = 0;
        for (int k = 0; k < WG / 64; ++k) round += wave_off[k];
        base += round;
    }
    if (blockIdx.x == nblocks - 1 && threadIdx.x == 0)
        sm->m = base;
}

hipError_t launch_select(const nb_system &s, nb_small *small, int32_t *i_idx, hipStream_t st)
{
    const SelShape sh = sel_shape(s.n);
    hipLaunchKernelGGL(select_min_kernel, dim3(sh.blocks), dim3(WG), 0, st, s.t, s.dt, s.n,
                       sh.slice, small);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_count_kernel, dim3(sh.blocks), dim3(WG), 0, st, s.t, s.dt, s.n,
                       sh.slice, sh.blocks, small);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_scatter_kernel, dim3(sh.blocks), dim3(WG), 0, st, s.t, s.dt, s.n,
                       sh.slice, sh.blocks, small, i_idx);
    return hipGetLastError();
}

// ---- predictor -----------------------------------------------------------------

__global__ __launch_bounds__(WG) void predict_kernel(nb_system s, double t_next)
{
    const int64_t stride = (int64_t)gridDim.x * WG;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < s.n; i += stride) {
        const double d = t_next - s.t[i];
        const double d2 = d * d * 0.5, d3 = d * d * d * (1.0 / 6.0);
        const double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
        const double ax = s.ax[i], ay = s.ay[i], az = s.az[i];
        const double jx = s.jx[i], jy = s.jy[i], jz = s.jz[i];
        s.xp[i] = s.x[i] + vx * d + ax * d2 + jx * d3;
        s.yp[i] = s.y[i] + vy * d + ay * d2 + jy * d3;
        s.zp[i] = s.z[i] + vz * d + az * d2 + jz * d3;
        const double px = vx + ax * d + jx * d2;
        const double py = vy + ay * d + jy * d2;
        const double pz = vz + az * d + jz * d2;
        s.vxp[i] = px; s.vyp[i] = py; s.vzp[i] = pz;
        if (s.vxp32) {
            s.vxp32[i] = (float)px; s.vyp32[i] = (float)py; s.vzp32[i] = (float)pz;
            s.m32[i] = (float)s.m[i];
        }
    }
}

hipError_t launch_predict(const nb_system &s, double t_next, hipStream_t st)
{
    int64_t blocks = (s.n + WG - 1) / WG;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(predict_kernel, dim3((unsigned)blocks), dim3(WG), 0, st, s, t_next);
    return hipGetLastError();
}

// ---- corrector and new step ------------------------------------------------------

__device__ __forceinline__ double norm3(double a, double b, double c)
{
    return sqrt(a * a + b * b + c * c);
}

__global__ __launch_bounds__(WG) void correct_kernel(nb_system s, const int32_t *i_idx, int32_t m,
                                                     const double *acc, const double *jerk,
                                                     double t_next, double eta, double dt_max,
                                                     double dt_min, int *status)
{
    const int64_t k = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (k >= m)
        return;
    const int64_t i = i_idx ? (int64_t)i_idx[k] : k;
    if (i < 0 || i >= s.n) {
        atomicOr(status, (int)NBK_EINDEX);
        return;
    }
    const double h = t_next - s.t[i];
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    double* xs[3] = {s.x, s.y, s.z};
    double* vs[3] = {s.vx, s.vy, s.vz};
    double* as[3] = {s.ax, s.ay, s.az};
    double* js[3] = {s.jx, s.jy, s.jz};
    const double* xps[3] = {s.xp, s.yp, s.zp};
    const double* vps[3] = {s.vxp, s.vyp, s.vzp};
    double a1v[3], j1v[3], a2e[3], a3v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a0 = as[c][i], j0 = js[c][i];
        const double a1 = acc[c * (int64_t)m + k], j1 = jerk[c * (int64_t)m + k];
        const double da = a0 - a1;
        const double a2 = (-6.0 * da - h * (4.0 * j0 + 2.0 * j1)) / h2;
        const double a3 = (12.0 * da + 6.0 * h * (j0 + j1)) / h3;
        xs[c][i] = xps[c][i] + a2 * h4 / 24.0 + a3 * h5 / 120.0;
        vs[c][i] = vps[c][i] + a2 * h3 / 6.0 + a3 * h4 / 24.0;
        as[c][i] = a1;
        js[c][i] = j1;
        a1v[c] = a1; j1v[c] = j1;
        a2e[c] = a2 + a3 * h;
        a3v[c] = a3;
    }
    const double an = norm3(a1v[0], a1v[1], a1v[2]);
    const double jn = norm3(j1v[0], j1v[1], j1v[2]);
    const double sn = norm3(a2e[0], a2e[1], a2e[2]);
    const double cn = norm3(a3v[0], a3v[1], a3v[2]);
    const double num = an * sn + jn * jn, den = jn * cn + sn * sn;
    const double dta = den > 0.0 ? sqrt(eta * num / den) : INFINITY;
    int err = 0;
    if (isnan(dta) || !isfinite(an) || !isfinite(jn))
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
        atomicOr(status, err);
}

hipError_t launch_correct(const nb_system &s, const int32_t *i_idx, int32_t m,
                          const double *acc, const double *jerk, double t_next, double eta,
                          double dt_max, double dt_min, int *status, hipStream_t st)
{
    const unsigned blocks = (unsigned)((m + WG - 1) / WG);
    hipLaunchKernelGGL(correct_kernel, dim3(blocks), dim3(WG), 0, st, s, i_idx, m, acc, jerk,
                       t_next, eta, dt_max, dt_min, status);
    return hipGetLastError();
}

// ---- startup ---------------------------------------------------------------------

__global__ __launch_bounds__(WG) void init_steps_kernel(nb_system s, const double *acc,
                                                        const double *jerk, double eta_s,
                                                        double dt_max, double dt_min, int *status)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i >= s.n)
        return;
    const int64_t n = s.n;
    const double ax = acc[i], ay = acc[n + i], az = acc[2 * n + i];
    const double jx = jerk[i], jy = jerk[n + i], jz = jerk[2 * n + i];
    s.ax[i] = ax; s.ay[i] = ay; s.az[i] = az;
    s.jx[i] = jx; s.jy[i] = jy; s.jz[i] = jz;
    const double an = norm3(ax, ay, az), jn = norm3(jx, jy, jz);
    int err = 0;
    if (!isfinite(an) || !isfinite(jn))
        err |= NBK_ENAN;
    double want = jn > 0.0 ? eta_s * an / jn : dt_max;
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
        atomicOr(status, err);
}

hipError_t launch_init_steps(const nb_system &s, const double *acc, const double *jerk,
                             double eta_s, double dt_max, double dt_min, int *status,
                             hipStream_t st)
{
    const unsigned blocks = (unsigned)((s.n + WG - 1) / WG);
    hipLaunchKernelGGL(init_steps_kernel, dim3(blocks), dim3(WG), 0, st, s, acc, jerk, eta_s,
                       dt_max, dt_min, status);
    return hipGetLastError();
}

}  // namespace nbk
