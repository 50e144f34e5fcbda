// Tight pairs, carried in the block-step system as one body at their centre of
// mass (the HiGPUs-R scheme of Sec. 3 of the paper: tight groups are treated
// apart from the N-body integration, on CPU threads, while the GPU works).
//
//  - GPU: the tidal tensor d a / d x of the softened field at each listed body,
//    FP64, one workgroup per body.
//  - CPU: the relative orbit of each pair over a block step, in substeps of
//    kick (h/2) - exact two-body drift h - kick (h/2), the kicks from the tidal
//    tensor interpolated linearly over the step; OpenMP, one pair per thread
//    at a time; optionally queued on a thread of the context, so that it runs
//    while the host goes on enqueueing GPU work, as many block steps behind the
//    GPU as the CPU needs.
//  - The two-body drift uses universal variables (Stumpff functions), with the
//    universal anomaly found by Newton steps kept inside a bracket.
#include <math.h>
#include <omp.h>

#include <algorithm>
#include <vector>

#include "ctx.h"
#include "launch.h"

namespace nbk {

// T[(3a+b) nrows + row] = sum_{j != i} m_j (3 r_a r_b / s^(5/2) - delta_ab / s^(3/2)),
// r = xp_j - xp_i, s = |r|^2 + eps^2, for the k-th listed body i of an item, into
// the item's `tensor` (and the body's time t_i into its `t_out`, when set), at
// row k, or, with row0 >= 0, at row i - row0 (bodies below row0 write nothing:
// an active list whose centre-of-mass bodies start at row0).  With `pts` set the
// k-th workgroup takes the point k of `pts` instead of a body, leaves out the two
// rows excl[k] and excl[nrows + k] instead of i, and writes row k.  Each thread
// sums a strided slice of j in order; the 256 partial sums are combined in a
// fixed tree order.
__global__ __launch_bounds__(WG) void tidal_kernel(const Item *items, const int64_t *starts,
                                                   int n_items)
{
    __shared__ double part[9][WG];
    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int64_t k = (int64_t)blockIdx.x - starts[it_k];   // one workgroup per body or point
    const double *xp = p.s.xp, *yp = p.s.yp, *zp = p.s.zp, *mass = p.s.m;
    int64_t i = -1, skip0, skip1 = -1, row;
    double xi, yi, zi;
    if (p.pts) {
        row = k;
        xi = p.pts[k];
        yi = p.pts[p.nrows + k];
        zi = p.pts[2 * p.nrows + k];
        skip0 = p.excl ? p.excl[k] : -1;
        skip1 = p.excl ? p.excl[p.nrows + k] : -1;
    } else {
        i = p.i_idx ? (int64_t)p.i_idx[k] : k;
        if (i < 0 || i >= p.s.n) {
            if (threadIdx.x == 0)
                atomicOr(p.status, (int)NBK_EINDEX);
            i = 0;
        }
        row = p.row0 >= 0 ? i - p.row0 : k;
        if (row < 0 || row >= p.nrows)   // the same for every thread of the workgroup
            return;
        xi = xp[i];
        yi = yp[i];
        zi = zp[i];
        skip0 = i;
    }
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
        acc[q] = 0.0;
    for (int64_t j = p.j0 + threadIdx.x; j < p.j1; j += WG) {
        if (j == skip0 || j == skip1)
            continue;
        const double d[3] = {xp[j] - xi, yp[j] - yi, zp[j] - zi};
        const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + p.eps2;
        const double inv_s = 1.0 / s;
        const double w3 = mass[j] * inv_s / sqrt(s);     // m / s^(3/2)
        const double w5 = 3.0 * w3 * inv_s;              // 3 m / s^(5/2)
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b)
                acc[3 * a + b] += w5 * d[a] * d[b] - (a == b ? w3 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q)
        part[q][threadIdx.x] = acc[q];
    __syncthreads();
    for (int half = WG / 2; half >= 1; half >>= 1) {
        if ((int)threadIdx.x < half)
#pragma unroll
            for (int q = 0; q < 9; ++q)
                part[q][threadIdx.x] += part[q][threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x < 9)
        p.tensor[threadIdx.x * p.nrows + row] = part[threadIdx.x][0];
    if (threadIdx.x == 9 && p.t_out && i >= 0)
        p.t_out[row] = p.s.t[i];
}

// |r|^2 = (dx dx + dy dy) + dz dz in FP64, rounded after every operation (no fused
// multiply-add), so that equal inputs give equal distances everywhere.
__device__ __forceinline__ double dist2_rn(double dx, double dy, double dz)
{
#pragma clang fp contract(off)
    return dx * dx + dy * dy + dz * dz;
}

// Nearest other body of the k-th listed body i, over the whole predicted set:
// the least dist2_rn(xp_j - xp_i), the lowest j among equal distances.  Bodies at
// or above row_end, or with dt_i > dt_cap, are not searched (nn = -1, r2 = inf).
// Each thread scans a strided slice of j in order; the 256 (distance, index)
// candidates are then combined by a tree over LDS.
__global__ __launch_bounds__(WG) void nearest_kernel(const Item *items, const int64_t *starts,
                                                     int n_items)
{
    __shared__ double bd[WG];
    __shared__ int32_t bj[WG];
    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int64_t k = (int64_t)blockIdx.x - starts[it_k];   // one workgroup per listed body
    const int64_t n = p.s.n;
    const int64_t i = p.i_idx ? (int64_t)p.i_idx[k] : k;
    const bool bad = i < 0 || i >= n;
    if (bad || i >= p.row_end || !(p.s.dt[i] <= p.dt_cap)) {   // uniform over the workgroup
        if (threadIdx.x == 0) {
            if (bad)
                atomicOr(p.status, (int)NBK_EINDEX);
            p.nn[k] = -1;
            p.r2[k] = INFINITY;
        }
        return;
    }
    const double *xp = p.s.xp, *yp = p.s.yp, *zp = p.s.zp;
    const double xi = xp[i], yi = yp[i], zi = zp[i];
    double best = INFINITY;
    int32_t bestj = -1;
    for (int64_t j = threadIdx.x; j < n; j += WG) {
        if (j == i)
            continue;
        const double d = dist2_rn(xp[j] - xi, yp[j] - yi, zp[j] - zi);
        if (d < best) {          // j grows along the slice: the first of equals stays
            best = d;
            bestj = (int32_t)j;
        }
    }
    bd[threadIdx.x] = best;
    bj[threadIdx.x] = bestj;
    __syncthreads();
    for (int half = WG / 2; half >= 1; half >>= 1) {
        if ((int)threadIdx.x < half) {
            const double o = bd[threadIdx.x + half];
            const int32_t oj = bj[threadIdx.x + half];
            const int32_t mj = bj[threadIdx.x];
            // (distance, index) order; -1 marks an empty slice (distance inf)
            if (oj >= 0 && (mj < 0 || o < bd[threadIdx.x] || (o == bd[threadIdx.x] && oj < mj))) {
                bd[threadIdx.x] = o;
                bj[threadIdx.x] = oj;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        p.nn[k] = bj[0];
        p.r2[k] = bj[0] >= 0 ? bd[0] : INFINITY;
    }
}

hipError_t launch_tidal(const Table &t, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(tidal_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items, t.starts,
                       t.n);
    return hipGetLastError();
}

hipError_t launch_nearest(const Table &t, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(nearest_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items,
                       t.starts, t.n);
    return hipGetLastError();
}

}  // namespace nbk

// ---- host: two-body drift and the relative orbit of a pair -------------------------

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;

// Stumpff functions c2(z) = (1 - cos sqrt z) / z and c3(z) = (sqrt z - sin sqrt z) / z^1.5
// for z >= 0 (series below 1e-3).
void stumpff(double z, double &c2, double &c3)
{
    if (z > 1e-3) {
        const double sz = sqrt(z);
        c2 = (1.0 - cos(sz)) / z;
        c3 = (sz - sin(sz)) / (z * sz);
    } else {
        c2 = 0.5 - z / 24.0 + z * z / 720.0 - z * z * z / 40320.0;
        c3 = 1.0 / 6.0 - z / 120.0 + z * z / 5040.0 - z * z * z / 362880.0;
    }
}

// Bound two-body motion of the relative coordinate over dt (mu = total mass).
// Returns false for an unbound or degenerate pair.
bool drift(double mu, const double *r0, const double *v0, double dt, double *r1, double *v1)
{
    const double r0n = sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    const double v2 = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    if (!(mu > 0.0) || !(r0n > 0.0))
        return false;
    const double alpha = 2.0 / r0n - v2 / mu;                 // 1 / a
    if (!(alpha > 0.0))
        return false;
    const double smu = sqrt(mu);
    const double period = kTwoPi / (smu * alpha * sqrt(alpha));
    double t = fmod(dt, period);                              // Kepler motion is periodic
    if (t < 0.0)
        t += period;
    const double rv = (r0[0] * v0[0] + r0[1] * v0[1] + r0[2] * v0[2]) / smu;
    // F(chi) = rv chi^2 c2 + (1 - alpha r0) chi^3 c3 + r0 chi - sqrt(mu) t, with
    // F' = |r(chi)| > 0; over one period chi runs from 0 to 2 pi / sqrt(alpha)
    double lo = 0.0, hi = kTwoPi / sqrt(alpha);
    double chi = smu * alpha * t;
    if (!(chi > lo && chi < hi))
        chi = 0.5 * (lo + hi);
    double c2 = 0.5, c3 = 1.0 / 6.0, rn = r0n;
    for (int it = 0; it < 200; ++it) {
        const double z = alpha * chi * chi;
        stumpff(z, c2, c3);
        const double chi2 = chi * chi;
        const double F = rv * chi2 * c2 + (1.0 - alpha * r0n) * chi2 * chi * c3 + r0n * chi -
                         smu * t;
        rn = chi2 * c2 + rv * chi * (1.0 - z * c3) + r0n * (1.0 - z * c2);
        if (F > 0.0)
            hi = chi;
        else
            lo = chi;
        double next = chi - F / rn;
        if (!(next > lo && next < hi))
            next = 0.5 * (lo + hi);
        const double step = next - chi;
        chi = next;
        if (fabs(step) <= 4e-16 * (1.0 + chi) || hi - lo <= 4e-16 * (1.0 + hi))
            break;
    }
    const double z = alpha * chi * chi;
    stumpff(z, c2, c3);
    const double chi2 = chi * chi;
    const double f = 1.0 - chi2 / r0n * c2;
    const double g = t - chi2 * chi / smu * c3;
    double r[3];
    for (int c = 0; c < 3; ++c)
        r[c] = f * r0[c] + g * v0[c];
    const double r1n = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double fd = smu / (r1n * r0n) * chi * (z * c3 - 1.0);
    const double gd = 1.0 - chi2 / r1n * c2;
    for (int c = 0; c < 3; ++c) {
        v1[c] = fd * r0[c] + gd * v0[c];
        r1[c] = r[c];
    }
    return true;
}

// One pair over H: nsub substeps of kick - drift - kick, T linear from T0 to T1.
bool advance_pair(double mu, double *r, double *v, double H, const double *T0, const double *T1,
                  int per_period, int64_t max_sub)
{
    const double rn = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double alpha = 2.0 / rn - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) / mu;
    if (!(alpha > 0.0) || !(H >= 0.0))
        return false;
    const double period = kTwoPi / (sqrt(mu) * alpha * sqrt(alpha));
    int64_t nsub = (int64_t)ceil((double)per_period * H / period);
    if (nsub < 1) nsub = 1;
    if (nsub > max_sub) nsub = max_sub;
    const double h = H / (double)nsub;
    auto kick = [&](double w) {
        double tr[3];
        for (int a = 0; a < 3; ++a) {
            tr[a] = 0.0;
            for (int b = 0; b < 3; ++b)
                tr[a] += ((1.0 - w) * T0[3 * a + b] + w * T1[3 * a + b]) * r[b];
        }
        for (int a = 0; a < 3; ++a)
            v[a] += 0.5 * h * tr[a];
    };
    for (int64_t q = 0; q < nsub; ++q) {
        kick((double)q / (double)nsub);
        double r1[3], v1[3];
        if (!drift(mu, r, v, h, r1, v1))
            return false;
        for (int c = 0; c < 3; ++c) {
            r[c] = r1[c];
            v[c] = v1[c];
        }
        kick((double)(q + 1) / (double)nsub);
    }
    return true;
}

struct GroupJob {
    int32_t n;
    const int32_t *idx;   // row of pair k in M, r, v, status; NULL = k
    const double *M;
    double *r, *v;
    const double *H, *T0, *T1;
    int32_t per_period;
    int64_t max_sub;
    int32_t *status;
};

// threads: OpenMP team size (0 = the runtime's default).
nb_status run_groups(const GroupJob &j, int threads)
{
    int bad = 0;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : bad) num_threads(nt)
    for (int32_t k = 0; k < j.n; ++k) {
        const int64_t row = j.idx ? j.idx[k] : k;
        const bool ok = advance_pair(j.M[row], j.r + 3 * row, j.v + 3 * row, j.H[k],
                                     j.T0 + 9 * k, j.T1 + 9 * k, j.per_period, j.max_sub);
        if (j.status) j.status[row] = ok ? NB_OK : NB_EUNBOUND;
        bad += ok ? 0 : 1;
    }
    return bad ? NB_EUNBOUND : NB_OK;
}

nb_status check_group_args(int32_t n, const int32_t *idx, const double *M, const double *r,
                           const double *v, const double *H, const double *T0,
                           const double *T1, int32_t per_period, int64_t max_sub)
{
    if (n < 0 || per_period < 1 || max_sub < 1) return NB_EINVAL;
    if (n > 0 && (!M || !r || !v || !H || !T0 || !T1)) return NB_EINVAL;
    if (idx && n > 0) {
        // rows must be distinct: two threads must never advance one pair
        std::vector<int32_t> rows(idx, idx + n);
        std::sort(rows.begin(), rows.end());
        if (rows.front() < 0 || std::adjacent_find(rows.begin(), rows.end()) != rows.end())
            return NB_EINVAL;
    }
    return NB_OK;
}

}  // namespace

nb_status nb_groups_run(nb_ctx *ctx, int32_t n, const int32_t *idx, const double *M, double *r,
                        double *v, const double *H, const double *T0, const double *T1,
                        int32_t per_period, int64_t max_sub, int32_t *status, bool async)
{
    const nb_status e = check_group_args(n, idx, M, r, v, H, T0, T1, per_period, max_sub);
    if (e != NB_OK) {
        if (ctx) ctx->err = "nb_groups_advance: bad argument";
        return e;
    }
    const GroupJob job{n, idx, M, r, v, H, T0, T1, per_period, max_sub, status};
    if (!async)
        return run_groups(job, 0);
    // On the worker, leave one core to the thread that drives the GPU.
    const int threads = omp_get_max_threads() > 1 ? omp_get_max_threads() - 1 : 1;
    nb_ctx::Worker &w = ctx->worker;
    {
        std::lock_guard<std::mutex> lk(w.mu);
        w.queue.push_back([job, threads]() { return (int)run_groups(job, threads); });
    }
    if (!w.th.joinable()) {
        w.th = std::thread([&w]() {
            std::unique_lock<std::mutex> lk(w.mu);
            for (;;) {
                w.cv.wait(lk, [&w]() { return w.quit || !w.queue.empty(); });
                if (w.queue.empty()) return;   // quit, nothing left to run
                std::function<int()> f = std::move(w.queue.front());
                w.queue.pop_front();
                w.running = true;
                lk.unlock();
                const int r = f();
                lk.lock();
                if (w.result == NB_OK) w.result = r;
                w.running = false;
                w.cv.notify_all();
            }
        });
    }
    w.cv.notify_all();
    return NB_OK;
}

namespace {

// Pair indices valid: in [0, n), no index twice.  `seen` has n entries.
bool pairs_valid(int64_t n, int32_t n_pairs, const int64_t *pairs, std::vector<char> &seen)
{
    if (n < 0 || n_pairs < 0 || (n_pairs > 0 && !pairs) || 2 * (int64_t)n_pairs > n) return false;
    seen.assign((size_t)n, 0);
    for (int64_t q = 0; q < 2 * (int64_t)n_pairs; ++q) {
        const int64_t i = pairs[q];
        if (i < 0 || i >= n || seen[(size_t)i]) return false;
        seen[(size_t)i] = 1;
    }
    return true;
}

}  // namespace

extern "C" {

nb_status nb_pairs_reduce(int64_t n, const double *x, const double *v, const double *m,
                          int32_t n_pairs, const int64_t *pairs, double *xr, double *vr,
                          double *mr, double *M, double *r, double *w)
{
    std::vector<char> in_pair;
    if (!pairs_valid(n, n_pairs, pairs, in_pair)) return NB_EINVAL;
    if (n > 0 && (!x || !v || !m || !xr || !vr || !mr)) return NB_EINVAL;
    if (n_pairs > 0 && (!M || !r || !w)) return NB_EINVAL;
    int64_t q = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (in_pair[(size_t)i]) continue;
        for (int d = 0; d < 3; ++d) {
            xr[3 * q + d] = x[3 * i + d];
            vr[3 * q + d] = v[3 * i + d];
        }
        mr[q++] = m[i];
    }
    for (int32_t k = 0; k < n_pairs; ++k, ++q) {
        const int64_t a = pairs[2 * k], b = pairs[2 * k + 1];
        const double mt = m[a] + m[b];
        for (int d = 0; d < 3; ++d) {
            xr[3 * q + d] = (m[a] * x[3 * a + d] + m[b] * x[3 * b + d]) / mt;
            vr[3 * q + d] = (m[a] * v[3 * a + d] + m[b] * v[3 * b + d]) / mt;
            r[3 * k + d] = x[3 * b + d] - x[3 * a + d];
            w[3 * k + d] = v[3 * b + d] - v[3 * a + d];
        }
        mr[q] = mt;
        M[k] = mt;
    }
    return NB_OK;
}

nb_status nb_pairs_members(int64_t n, const double *xr, const double *vr, const double *m,
                           int32_t n_pairs, const int64_t *pairs, const double *r,
                           const double *w, double *x, double *v)
{
    std::vector<char> in_pair;
    if (!pairs_valid(n, n_pairs, pairs, in_pair)) return NB_EINVAL;
    if (n > 0 && (!x || !v || !m || !xr || !vr)) return NB_EINVAL;
    if (n_pairs > 0 && (!r || !w)) return NB_EINVAL;
    int64_t q = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (in_pair[(size_t)i]) continue;
        for (int d = 0; d < 3; ++d) {
            x[3 * i + d] = xr[3 * q + d];
            v[3 * i + d] = vr[3 * q + d];
        }
        ++q;
    }
    for (int32_t k = 0; k < n_pairs; ++k, ++q) {
        const int64_t a = pairs[2 * k], b = pairs[2 * k + 1];
        const double mt = m[a] + m[b], fa = m[b] / mt, fb = m[a] / mt;
        for (int d = 0; d < 3; ++d) {
            x[3 * a + d] = xr[3 * q + d] - fa * r[3 * k + d];
            x[3 * b + d] = xr[3 * q + d] + fb * r[3 * k + d];
            v[3 * a + d] = vr[3 * q + d] - fa * w[3 * k + d];
            v[3 * b + d] = vr[3 * q + d] + fb * w[3 * k + d];
        }
    }
    return NB_OK;
}

nb_status nb_pairs_energy(int32_t n_pairs, const double *m, const int64_t *pairs,
                          const double *r, const double *w, const double *T, double *out)
{
    if (!out || n_pairs < 0 || (n_pairs > 0 && (!m || !pairs || !r || !w || !T)))
        return NB_EINVAL;
    double s = 0.0, c = 0.0;     // Neumaier sum over the pairs in order
    for (int32_t k = 0; k < n_pairs; ++k) {
        const double ma = m[pairs[2 * k]], mb = m[pairs[2 * k + 1]];
        const double mt = ma + mb, mu = ma * mb / mt;
        const double *rk = r + 3 * k, *wk = w + 3 * k, *Tk = T + 9 * k;
        double w2 = 0.0, r2 = 0.0, rTr = 0.0;
        for (int a = 0; a < 3; ++a) {
            w2 += wk[a] * wk[a];
            r2 += rk[a] * rk[a];
            for (int b = 0; b < 3; ++b)
                rTr += rk[a] * Tk[3 * a + b] * rk[b];
        }
        if (!(r2 > 0.0)) return NB_EINVAL;
        const double e = mu * (0.5 * w2 - mt / sqrt(r2) - 0.5 * rTr);
        const double t = s + e;
        c += fabs(s) >= fabs(e) ? (s - t) + e : (e - t) + s;
        s = t;
    }
    *out = s + c;
    return NB_OK;
}

nb_status nb_pairs_perturbation(int32_t n_pairs, const double *M, const double *r,
                                const double *w, const double *T, double *a, double *gamma)
{
    if (n_pairs < 0 || (n_pairs > 0 && (!M || !a || !gamma || (r && !w)))) return NB_EINVAL;
    for (int32_t k = 0; k < n_pairs; ++k) {
        if (r) {
            const double *rk = r + 3 * k, *wk = w + 3 * k;
            const double rn = sqrt(rk[0] * rk[0] + rk[1] * rk[1] + rk[2] * rk[2]);
            const double w2 = wk[0] * wk[0] + wk[1] * wk[1] + wk[2] * wk[2];
            const double inv_a = 2.0 / rn - w2 / M[k];
            a[k] = inv_a > 0.0 ? 1.0 / inv_a : INFINITY;
        }
        double t2 = 0.0;
        if (T)
            for (int q = 0; q < 9; ++q)
                t2 += T[9 * k + q] * T[9 * k + q];
        const double d = 2.0 * a[k];
        gamma[k] = a[k] > 0.0 && isfinite(a[k]) ? sqrt(t2) * d * d * d / M[k] : INFINITY;
    }
    return NB_OK;
}

nb_status nb_pairs_split_energy(int32_t n_pairs, const double *m, const int64_t *pairs,
                                const double *r, double eps, double *out)
{
    if (!out || n_pairs < 0 || !(eps >= 0.0) || (n_pairs > 0 && (!m || !pairs || !r)))
        return NB_EINVAL;
    double s = 0.0;
    for (int32_t k = 0; k < n_pairs; ++k) {
        const double *rk = r + 3 * k;
        const double r2 = rk[0] * rk[0] + rk[1] * rk[1] + rk[2] * rk[2];
        if (!(r2 > 0.0)) return NB_EINVAL;
        s += m[pairs[2 * k]] * m[pairs[2 * k + 1]] * (1.0 / sqrt(r2) - 1.0 / sqrt(r2 + eps * eps));
    }
    *out = s;
    return NB_OK;
}

nb_status nb_kepler_drift(double M, const double *r0, const double *v0, double dt, double *r1,
                          double *v1)
{
    if (!r0 || !v0 || !r1 || !v1 || !isfinite(dt)) return NB_EINVAL;
    return drift(M, r0, v0, dt, r1, v1) ? NB_OK : NB_EUNBOUND;
}

nb_status nb_groups_advance(int32_t n, const int32_t *idx, const double *M, double *r,
                            double *v, const double *H, const double *T0, const double *T1,
                            int32_t per_period, int64_t max_sub, int32_t *status)
{
    return nb_groups_run(nullptr, n, idx, M, r, v, H, T0, T1, per_period, max_sub, status, false);
}

}  // extern "C"
