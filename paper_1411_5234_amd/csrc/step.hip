// Block-time-step kernels (Sec. 2 items 1-2 of the paper): active-block
// selection, Hermite-4 predictor for all bodies, corrector plus new
// power-of-two step for the active block, and the startup step.  All FP64.
// These are memory- or latency-bound one-pass kernels.  Every kernel serves a
// table of systems (items): a workgroup finds its item by binary search over
// the table's workgroup offsets and then works inside that one system.
#include "nb_internal.h"
#include "launch.h"

namespace nbk {

// Hermite-4 prediction of body i to t_next: position to the jerk term, velocity
// to the jerk term, FP64, plus the FP32 copies of the predicted velocity and mass.
__device__ __forceinline__ void predict_body(const nb_system &s, int64_t i, double t_next)
{
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

// ---- selection ---------------------------------------------------------------
// Per item, the bodies are cut into sel_blocks contiguous slices of sel_slice.
// Pass 1: each workgroup takes the minimum of t + dt over its slice and counts
//         the slice's bodies at that minimum.
// Pass 2: each workgroup reduces its item's slice minima to t_next (the same
//         arithmetic in every workgroup of the item), adds the counts of the
//         item's earlier slices whose minimum is t_next, and writes its due
//         bodies' indices in ascending order (ordered compaction with a wave
//         ballot and an LDS prefix over the four waves); the item's first
//         workgroup stores t_next, its last stores m.
// A slice whose minimum is above t_next holds no due body, and one whose minimum
// is t_next holds exactly its counted ones, so the offsets are those of the full
// ordered list.

// (minimum, count at the minimum) of two partial results.  A NaN never becomes
// the minimum and is never counted, as with fmin and ==.
__device__ __forceinline__ void min_count(double &v, int &c, double v2, int c2)
{
    if (v2 < v) {
        v = v2;
        c = c2;
    } else if (v2 == v) {
        c += c2;
    }
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

__global__ __launch_bounds__(WG) void select_min_kernel(const Item *items, const int64_t *starts,
                                                        int n_items, double *blockval,
                                                        int32_t *blockcnt)
{
    __shared__ double ldv[WG / 64];
    __shared__ int ldc[WG / 64];
    const int k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[k];
    const int64_t lb = (int64_t)blockIdx.x - starts[k];
    const int64_t b0 = lb * p.sel_slice;
    const int64_t b1 = min(b0 + p.sel_slice, p.s.n);
    double v = INFINITY;
    int c = 0;
    for (int64_t i = b0 + threadIdx.x; i < b1; i += WG)
        min_count(v, c, p.s.t[i] + p.s.dt[i], 1);
    for (int off = 32; off >= 1; off >>= 1) {
        const double v2 = __shfl_xor(v, off, 64);
        const int c2 = __shfl_xor(c, off, 64);
        min_count(v, c, v2, c2);
    }
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    if (l == 0) {
        ldv[w] = v;
        ldc[w] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        v = ldv[0];
        c = ldc[0];
        for (int q = 1; q < WG / 64; ++q) min_count(v, c, ldv[q], ldc[q]);
        blockval[p.sel_off + lb] = v;
        blockcnt[p.sel_off + lb] = c;
    }
}

__global__ __launch_bounds__(WG) void select_scatter_kernel(const Item *items,
                                                            const int64_t *starts, int n_items,
                                                            const double *blockval,
                                                            const int32_t *blockcnt,
                                                            SelResult *res)
{
    __shared__ double lds[WG / 64];
    __shared__ int ldi[WG / 64];
    __shared__ int wave_off[WG / 64];
    const int k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[k];
    const int64_t lb = (int64_t)blockIdx.x - starts[k];
    double v = INFINITY;
    for (int q = threadIdx.x; q < p.sel_blocks; q += WG)
        v = fmin(v, blockval[p.sel_off + q]);
    const double tn = wg_min(v, lds);
    int before = 0;
    for (int q = threadIdx.x; q < (int)lb; q += WG)
        before += blockval[p.sel_off + q] == tn ? blockcnt[p.sel_off + q] : 0;
    int base = wg_sum_int(before, ldi);
    if (lb == 0 && threadIdx.x == 0)
        res[k].t_next = tn;
    const int64_t b0 = lb * p.sel_slice;
    const int64_t b1 = min(b0 + p.sel_slice, p.s.n);
    const int w = threadIdx.x / 64, l = threadIdx.x % 64;
    int32_t *out = (int32_t *)p.i_idx;
    for (int64_t r = b0; r < b1; r += WG) {
        const int64_t i = r + threadIdx.x;
        const bool due = (i < b1) && (p.s.t[i] + p.s.dt[i] == tn);
        const unsigned long long mask = __ballot(due);
        const int in_wave = __popcll(mask & ((1ull << l) - 1ull));
        __syncthreads();
        if (l == 0) wave_off[w] = __popcll(mask);
        __syncthreads();
        int off = base;
        for (int q = 0; q < w; ++q) off += wave_off[q];
        if (due)
            out[off + in_wave] = (int32_t)i;
        int round = 0;
        for (int q = 0; q < WG / 64; ++q) round += wave_off[q];
        base += round;
    }
    if (lb == p.sel_blocks - 1 && threadIdx.x == 0)
        res[k].m = base;
}

hipError_t launch_select(const Table &t, double *blockval, int32_t *blockcnt, SelResult *res,
                         hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    const dim3 grid((unsigned)t.blocks);
    hipLaunchKernelGGL(select_min_kernel, grid, dim3(WG), 0, st, t.items, t.starts, t.n, blockval,
                       blockcnt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(select_scatter_kernel, grid, dim3(WG), 0, st, t.items, t.starts, t.n,
                       (const double *)blockval, (const int32_t *)blockcnt, res);
    return hipGetLastError();
}

// One workgroup: read every item's status word into res[k].status and, when
// `host` is set, write each item's whole result there (mapped pinned memory that
// the host reads once this kernel has completed, or once it sees `seq` in *flag);
// then clear the words (several items may share one word, so all reads finish
// before any clear).  Every lane's result stores reach host memory (system-scope
// fence) before the barrier, and the flag is stored after it with release order.
__global__ __launch_bounds__(WG) void collect_status_kernel(const Item *items, int n, SelResult *res,
                                                            SelResult *host, unsigned *flag,
                                                            unsigned seq)
{
    for (int k = threadIdx.x; k < n; k += WG) {
        SelResult r = res[k];
        r.status = *items[k].status;
        res[k].status = r.status;
        if (host) host[k] = r;
    }
    if (flag) __threadfence_system();
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += WG)
        *items[k].status = 0;
    if (flag && threadIdx.x == 0)
        __hip_atomic_store(flag, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(WG) void upload_kernel(const uint4 *src, uint4 *dst, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

hipError_t launch_upload(const char *src, char *dst, size_t bytes, hipStream_t st)
{
    const int64_t n = (int64_t)(bytes / sizeof(uint4));
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(upload_kernel, dim3((unsigned)((n + WG - 1) / WG)), dim3(WG), 0, st,
                       (const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

hipError_t launch_collect_status(const Item *items, int n, SelResult *res, SelResult *host,
                                 unsigned *flag, unsigned seq, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(collect_status_kernel, dim3(1), dim3(WG), 0, st, items, n, res, host, flag,
                       seq);
    return hipGetLastError();
}

// ---- predictor -----------------------------------------------------------------

// Each item's bodies to its t_next; or, with sel (the selection results of the
// same items, still on the device), to sel[k].t_next when that is not past the
// item's t_next field (then its horizon), so that the prediction can follow the
// selection on the stream while the host reads the results.
__global__ __launch_bounds__(WG) void predict_kernel(const Item *items, const int64_t *starts,
                                                     int n_items, const SelResult *sel)
{
    const int k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[k];
    const int64_t i = ((int64_t)blockIdx.x - starts[k]) * WG + threadIdx.x;
    double tn = p.t_next;
    if (sel) {
        tn = sel[k].t_next;
        if (!(tn <= p.t_next))
            return;
    }
    if (i < p.s.n)
        predict_body(p.s, i, tn);
}

hipError_t launch_predict(const Table &t, const SelResult *sel, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(predict_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items, t.starts,
                       t.n, sel);
    return hipGetLastError();
}

// ---- corrector and new step ------------------------------------------------------

__device__ __forceinline__ double norm3(double a, double b, double c)
{
    return sqrt(a * a + b * b + c * c);
}

__global__ __launch_bounds__(WG) void correct_kernel(const Item *items, const int64_t *starts,
                                                     int n_items, double eta, double dt_max,
                                                     double dt_min)
{
    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int64_t k = ((int64_t)blockIdx.x - starts[it_k]) * WG + threadIdx.x;
    const int32_t m = p.m;
    if (k >= m)
        return;
    const nb_system &s = p.s;
    const int64_t i = p.i_idx ? (int64_t)p.i_idx[k] : k;
    if (i < 0 || i >= s.n) {
        atomicOr(p.status, (int)NBK_EINDEX);
        return;
    }
    const double t_next = p.t_next;
    const double h = t_next - s.t[i];
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
    double *xs[3] = {s.x, s.y, s.z};
    double *vs[3] = {s.vx, s.vy, s.vz};
    double *as[3] = {s.ax, s.ay, s.az};
    double *js[3] = {s.jx, s.jy, s.jz};
    const double *xps[3] = {s.xp, s.yp, s.zp};
    const double *vps[3] = {s.vxp, s.vyp, s.vzp};
    double a1v[3], j1v[3], a2e[3], a3v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double a0 = as[c][i], j0 = js[c][i];
        const double a1 = p.acc[c * (int64_t)m + k], j1 = p.jerk[c * (int64_t)m + k];
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
        atomicOr(p.status, err);
}

hipError_t launch_correct(const Table &t, double eta, double dt_max, double dt_min,
                          hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(correct_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items, t.starts,
                       t.n, eta, dt_max, dt_min);
    return hipGetLastError();
}

// ---- startup ---------------------------------------------------------------------

__global__ __launch_bounds__(WG) void init_steps_kernel(const Item *items, const int64_t *starts,
                                                        int n_items, double eta_s, double dt_max,
                                                        double dt_min)
{
    const int k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[k];
    const int64_t q = ((int64_t)blockIdx.x - starts[k]) * WG + threadIdx.x;
    const nb_system &s = p.s;
    // every body (t = 0), or the listed bodies at the item's time t_next; the
    // acc/jerk rows hold one entry per body or per listed body
    const int64_t cnt = p.i_idx ? (int64_t)p.m : s.n;
    if (q >= cnt)
        return;
    int64_t i = p.i_idx ? (int64_t)p.i_idx[q] : q;
    if (i < 0 || i >= s.n) {
        atomicOr(p.status, (int)NBK_EINDEX);
        return;
    }
    const double ax = p.acc[q], ay = p.acc[cnt + q], az = p.acc[2 * cnt + q];
    const double jx = p.jerk[q], jy = p.jerk[cnt + q], jz = p.jerk[2 * cnt + q];
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
    s.t[i] = p.i_idx ? p.t_next : 0.0;
    s.dt[i] = step;
    if (err)
        atomicOr(p.status, err);
}

hipError_t launch_init_steps(const Table &t, double eta_s, double dt_max, double dt_min,
                             hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(init_steps_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items,
                       t.starts, t.n, eta_s, dt_max, dt_min);
    return hipGetLastError();
}

}  // namespace nbk
