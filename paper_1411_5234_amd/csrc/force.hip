// Pair-force kernels: acceleration and jerk of the active block (Eq. 1 with the
// Plummer softening of Eq. 2, and its time derivative), plus the softened
// potential energy.  gfx950, wave64.
//
// Work decomposition (Sec. 2 items 3 and 5 of the paper, re-designed for CDNA4):
//  - a workgroup of 256 lanes holds IL i-bodies per lane-group in VGPRs;
//  - S consecutive lanes share the same i-bodies and take every S-th j of each
//    tile, so a small active block still gives every lane work; their partial
//    sums are combined at the end with cross-lane shuffles inside the wave;
//  - j-bodies are staged cooperatively through LDS in structure-of-arrays tiles
//    (coalesced global loads, broadcast LDS reads when S = 1);
//  - the j-range is split into B chunks (the paper's Bfactor); each chunk writes
//    FP64 partials that a second kernel sums in fixed order;
//  - a launch serves a table of systems (items); each workgroup finds its item
//    by binary search over the table's workgroup offsets, so systems of
//    different N and active-block size share one launch.
// Precision (Sec. 2 item 4): the FP64 kernel does all pair arithmetic in FP64;
// the mixed kernel forms r_j - r_i in FP64, rounds it to FP32, does the rest in
// FP32 with the hardware reciprocal square root, accumulates short runs of
// FP32 terms and folds them into FP64 totals.
#include "pair.h"
#include "launch.h"

namespace nbk {

// Acceleration and jerk terms of one j-body on one i-body, all FP32 once the
// position difference (dx, dy, dz) is formed, added to the FP32 run sums.
__device__ __forceinline__ void pair_f32(float dx, float dy, float dz, float dvx, float dvy,
                                         float dvz, float mj, float eps2, float (&a)[3],
                                         float (&jk)[3])
{
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float rv = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const float mr3 = mj * rinv * rinv2;
    const float al = -3.0f * rv * rinv2;
    a[0] = fmaf(mr3, dx, a[0]);
    a[1] = fmaf(mr3, dy, a[1]);
    a[2] = fmaf(mr3, dz, a[2]);
    jk[0] = fmaf(mr3, fmaf(al, dx, dvx), jk[0]);
    jk[1] = fmaf(mr3, fmaf(al, dy, dvy), jk[1]);
    jk[2] = fmaf(mr3, fmaf(al, dz, dvz), jk[2]);
}

template <int IL, int S, int F, bool DS>
__global__ __launch_bounds__(WG, NBK_MIXED_WAVES) void force_mixed_kernel(const Item *items,
                                                                          const int64_t *starts,
                                                                          int n_items)
{
    __shared__ Tile<DS> tile;

    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int64_t local = (int64_t)blockIdx.x - starts[it_k];
    const int64_t iblk = local / p.b, bidx = local % p.b;
    const int tid = threadIdx.x;
    const int g = tid / S, s = tid % S;
    constexpr int IWG = (WG / S) * IL;
    const int64_t kbase = iblk * IWG + (int64_t)g * IL;
    const int64_t jb = p.j0 + bidx * p.chunk;
    const int64_t je = min(jb + p.chunk, p.j1);
    const float eps2 = (float)p.eps2;
    const int64_t n = p.s.n;
    const double *xp = p.s.xp, *yp = p.s.yp, *zp = p.s.zp;
    const float *vx32 = p.s.vxp32, *vy32 = p.s.vyp32, *vz32 = p.s.vzp32, *m32 = p.s.m32;

    IPos<DS> pi[IL];
    float vxi[IL], vyi[IL], vzi[IL];
    Total A[IL][3], J[IL][3];
#pragma unroll
    for (int u = 0; u < IL; ++u) {
        const int64_t k = kbase + u;
        int64_t i = 0;
        if (k < p.m) {
            i = p.i_idx ? (int64_t)p.i_idx[k] : k;
            if (i < 0 || i >= n) {
                atomicOr(p.status, (int)NBK_EINDEX);
                i = 0;
            }
        }
        pi[u] = ipos(xp[i], yp[i], zp[i], (IPos<DS> *)nullptr);
        vxi[u] = vx32[i]; vyi[u] = vy32[i]; vzi[u] = vz32[i];
    }

    for (int64_t jt = jb; jt < je; jt += TILE) {
        __syncthreads();
        for (int q = tid; q < TILE; q += WG) {
            const int64_t j = jt + q;
            if (j < je)
                tile.put(q, xp[j], yp[j], zp[j], vx32[j], vy32[j], vz32[j], m32[j]);
            else  // padding: zero mass contributes exactly zero
                tile.put(q, 0.0, 0.0, 0.0, 0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
        const int lim = (int)min<int64_t>(TILE, je - jt);
        for (int kk = 0; kk < lim; kk += S * F) {
            float a32[IL][3], j32[IL][3];
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) { a32[u][c] = 0.f; j32[u][c] = 0.f; }
            JBody<DS> cur = tile.get(kk + s);
#pragma unroll NBK_UNROLL
            for (int f = 0; f < F; ++f) {
                // the next j-body is read ahead of this one's arithmetic
                const int qn = kk + (f + 1 < F ? f + 1 : f) * S + s;
                const JBody<DS> nxt = tile.get(qn);
#pragma unroll
                for (int u = 0; u < IL; ++u) {
                    float dx, dy, dz;
                    diff(cur, pi[u], dx, dy, dz);
                    pair_f32(dx, dy, dz, cur.vx - vxi[u], cur.vy - vyi[u], cur.vz - vzi[u], cur.m,
                             eps2, a32[u], j32[u]);
                }
                cur = nxt;
            }
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A[u][c].add(a32[u][c]);
                    J[u][c].add(j32[u][c]);
                }
        }
    }

#pragma unroll
    for (int u = 0; u < IL; ++u) {
        double At[3], Jt[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            At[c] = A[u][c].value();
            Jt[c] = J[u][c].value();
            if constexpr (S > 1) {
                At[c] = group_sum<S>(At[c]);
                Jt[c] = group_sum<S>(Jt[c]);
            }
        }
        const int64_t k = kbase + u;
        if (s == 0 && k < p.m) {
            const int64_t six_m = 6 * (int64_t)p.m;
            double *oa = p.b > 1 ? p.part + bidx * six_m : p.acc;
            double *oj = p.b > 1 ? p.part + bidx * six_m + 3 * (int64_t)p.m : p.jerk;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                oa[c * (int64_t)p.m + k] = At[c];
                oj[c * (int64_t)p.m + k] = Jt[c];
            }
        }
    }
}

template <int IL, int S, int F>
__global__ __launch_bounds__(WG) void force_fp64_kernel(const Item *items, const int64_t *starts,
                                                        int n_items)
{
    __shared__ double sx[TILE], sy[TILE], sz[TILE];
    __shared__ double svx[TILE], svy[TILE], svz[TILE], sm[TILE];

    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int64_t local = (int64_t)blockIdx.x - starts[it_k];
    const int64_t iblk = local / p.b, bidx = local % p.b;
    const int tid = threadIdx.x;
    const int g = tid / S, s = tid % S;
    constexpr int IWG = (WG / S) * IL;
    const int64_t kbase = iblk * IWG + (int64_t)g * IL;
    const int64_t jb = p.j0 + bidx * p.chunk;
    const int64_t je = min(jb + p.chunk, p.j1);
    const double eps2 = p.eps2;
    const int64_t n = p.s.n;
    const double *xp = p.s.xp, *yp = p.s.yp, *zp = p.s.zp;
    const double *vx64 = p.s.vxp, *vy64 = p.s.vyp, *vz64 = p.s.vzp, *m64 = p.s.m;

    double xi[IL], yi[IL], zi[IL], vxi[IL], vyi[IL], vzi[IL];
    double A[IL][3], J[IL][3];
#pragma unroll
    for (int u = 0; u < IL; ++u) {
        const int64_t k = kbase + u;
        int64_t i = 0;
        if (k < p.m) {
            i = p.i_idx ? (int64_t)p.i_idx[k] : k;
            if (i < 0 || i >= n) {
                atomicOr(p.status, (int)NBK_EINDEX);
                i = 0;
            }
        }
        xi[u] = xp[i]; yi[u] = yp[i]; zi[u] = zp[i];
        vxi[u] = vx64[i]; vyi[u] = vy64[i]; vzi[u] = vz64[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) { A[u][c] = 0.0; J[u][c] = 0.0; }
    }

    for (int64_t jt = jb; jt < je; jt += TILE) {
        __syncthreads();
        for (int q = tid; q < TILE; q += WG) {
            const int64_t j = jt + q;
            if (j < je) {
                sx[q] = xp[j]; sy[q] = yp[j]; sz[q] = zp[j];
                svx[q] = vx64[j]; svy[q] = vy64[j]; svz[q] = vz64[j];
                sm[q] = m64[j];
            } else {
                sx[q] = 0.0; sy[q] = 0.0; sz[q] = 0.0;
                svx[q] = 0.0; svy[q] = 0.0; svz[q] = 0.0; sm[q] = 0.0;
            }
        }
        __syncthreads();
        const int lim = (int)min<int64_t>(TILE, je - jt);
        for (int kk = 0; kk < lim; kk += S * F) {
            double at[IL][3], jt3[IL][3];
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) { at[u][c] = 0.0; jt3[u][c] = 0.0; }
#pragma unroll 2
            for (int f = 0; f < F; ++f) {
                const int q = kk + f * S + s;
                const double xj = sx[q], yj = sy[q], zj = sz[q];
                const double vxj = svx[q], vyj = svy[q], vzj = svz[q], mj = sm[q];
#pragma unroll
                for (int u = 0; u < IL; ++u) {
                    const double dx = xj - xi[u], dy = yj - yi[u], dz = zj - zi[u];
                    const double dvx = vxj - vxi[u], dvy = vyj - vyi[u], dvz = vzj - vzi[u];
                    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                    const double rv = fma(dx, dvx, fma(dy, dvy, dz * dvz));
                    const double rinv = rsqrt64(r2);
                    const double rinv2 = rinv * rinv;
                    const double mr3 = mj * rinv * rinv2;
                    const double al = -3.0 * rv * rinv2;
                    at[u][0] = fma(mr3, dx, at[u][0]);
                    at[u][1] = fma(mr3, dy, at[u][1]);
                    at[u][2] = fma(mr3, dz, at[u][2]);
                    jt3[u][0] = fma(mr3, fma(al, dx, dvx), jt3[u][0]);
                    jt3[u][1] = fma(mr3, fma(al, dy, dvy), jt3[u][1]);
                    jt3[u][2] = fma(mr3, fma(al, dz, dvz), jt3[u][2]);
                }
            }
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) { A[u][c] += at[u][c]; J[u][c] += jt3[u][c]; }
        }
    }

#pragma unroll
    for (int u = 0; u < IL; ++u) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if constexpr (S > 1) {
                A[u][c] = group_sum<S>(A[u][c]);
                J[u][c] = group_sum<S>(J[u][c]);
            }
        }
        const int64_t k = kbase + u;
        if (s == 0 && k < p.m) {
            const int64_t six_m = 6 * (int64_t)p.m;
            double *oa = p.b > 1 ? p.part + bidx * six_m : p.acc;
            double *oj = p.b > 1 ? p.part + bidx * six_m + 3 * (int64_t)p.m : p.jerk;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                oa[c * (int64_t)p.m + k] = A[u][c];
                oj[c * (int64_t)p.m + k] = J[u][c];
            }
        }
    }
}

// Fold interval: FP32 terms summed per lane before a fold into FP64 (mixed),
// bounded so that a tile holds a whole number of folds.
template <int S>
constexpr int fold_mixed() { return (TILE / S) < NBK_FOLD ? (TILE / S) : NBK_FOLD; }
template <int S>
constexpr int fold_fp64() { return TILE / S; }

template <int IL, int S>
static hipError_t launch_one(int precision, const Table &t, hipStream_t st)
{
    const dim3 grid((unsigned)t.blocks);
    if (precision == NB_MIXED)
        hipLaunchKernelGGL((force_mixed_kernel<IL, S, fold_mixed<S>(), false>), grid, dim3(WG), 0,
                           st, t.items, t.starts, t.n);
    else if (precision == NB_DS)
        hipLaunchKernelGGL((force_mixed_kernel<IL, S, fold_mixed<S>(), true>), grid, dim3(WG), 0,
                           st, t.items, t.starts, t.n);
    else
        hipLaunchKernelGGL((force_fp64_kernel<IL, S, fold_fp64<S>()>), grid, dim3(WG), 0, st,
                           t.items, t.starts, t.n);
    return hipGetLastError();
}

template <int IL>
static hipError_t launch_il(int precision, int s, const Table &t, hipStream_t st)
{
    switch (s) {
    case 1: return launch_one<IL, 1>(precision, t, st);
    case 4: return launch_one<IL, 4>(precision, t, st);
    case 16: return launch_one<IL, 16>(precision, t, st);
    case 64: return launch_one<IL, 64>(precision, t, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_force(int precision, int il, int s, const Table &t, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    switch (il) {
    case 1: return launch_il<1>(precision, s, t, st);
    case 2: return launch_il<2>(precision, s, t, st);
    case 4: return launch_il<4>(precision, s, t, st);
    default: return hipErrorInvalidValue;
    }
}

// Partial sums of every item with j_chunks B > 1, reduced to acc, jerk (and
// snap): 6 values per body, 9 for the 6th order.  L = red_lanes lanes (a power
// of two dividing WG) share an output value: lane l adds chunks l, l + L, l + 2L,
// ... in ascending order, then the L lane sums are added in ascending l.  The
// order depends on B and L only, so results are bitwise reproducible; with
// L = 1 it is the plain ascending sum.  Many lanes per value keep the loads of a
// large B (small active blocks) in flight together instead of in one chain.
__global__ __launch_bounds__(WG) void reduce_partials_kernel(const Item *items,
                                                             const int64_t *starts, int n_items)
{
    __shared__ double lane_sum[WG];
    const int it_k = find_item(starts, n_items, blockIdx.x);
    const Item &p = items[it_k];
    const int L = p.red_lanes;
    const int per = WG / L;                                  // values per workgroup
    const int ii = threadIdx.x % per, l = threadIdx.x / per;
    const int64_t idx = ((int64_t)blockIdx.x - starts[it_k]) * per + ii;   // < K m
    const int64_t three_m = 3 * (int64_t)p.m;
    const int64_t km = force_outputs(p) * three_m / 3;
    double v = 0.0;
    if (idx < km) {
#pragma unroll 8
        for (int b = l; b < p.b; b += L)
            v += p.part[(int64_t)b * km + idx];
    }
    lane_sum[threadIdx.x] = v;
    __syncthreads();
    if (l != 0 || idx >= km)
        return;
    for (int q = 1; q < L; ++q)
        v += lane_sum[q * per + ii];
    if (idx < three_m)
        p.acc[idx] = v;
    else if (idx < 2 * three_m)
        p.jerk[idx - three_m] = v;
    else
        p.snap[idx - 2 * three_m] = v;
}

hipError_t launch_reduce(const Table &t, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)t.blocks), dim3(WG), 0, st, t.items,
                       t.starts, t.n);
    return hipGetLastError();
}

// ---- energy -------------------------------------------------------------------

// rows[i] = m_i * sum_{j > i} m_j / sqrt(|x_j - x_i|^2 + eps^2): each unordered pair
// once, one i per lane.  Row i takes n - 1 - i pairs, so workgroup k takes two
// blocks of WG rows, block k and block nb - 1 - k (nb = blocks of WG rows), and
// every workgroup does about n pairs.  The first tile of a block holds its own
// rows' diagonal (pairs with j <= i masked out); the tiles after it are whole.
__global__ __launch_bounds__(WG) void potential_rows_kernel(const double *x, const double *y,
                                                            const double *z, const double *mass,
                                                            int64_t n, double eps2, double *rows)
{
    __shared__ double sx[TILE], sy[TILE], sz[TILE], sm[TILE];
    const int64_t nb = (n + WG - 1) / WG;
    const int64_t blk[2] = {(int64_t)blockIdx.x, nb - 1 - (int64_t)blockIdx.x};
    for (int h = 0; h < 2; ++h) {
        if (h == 1 && blk[1] == blk[0]) break;
        const int64_t i0 = blk[h] * WG;
        const int64_t i = i0 + threadIdx.x;
        const int64_t ii = i < n ? i : n - 1;
        const double xi = x[ii], yi = y[ii], zi = z[ii];
        double tot = 0.0;
        for (int64_t jt = i0; jt < n; jt += TILE) {
            __syncthreads();
            for (int q = threadIdx.x; q < TILE; q += WG) {
                const int64_t j = jt + q;
                if (j < n) { sx[q] = x[j]; sy[q] = y[j]; sz[q] = z[j]; sm[q] = mass[j]; }
            }
            __syncthreads();
            const int lim = (int)min<int64_t>(TILE, n - jt);
            double part = 0.0;
            if (jt == i0) {
                for (int q = 0; q < lim; ++q) {
                    const double dx = sx[q] - xi, dy = sy[q] - yi, dz = sz[q] - zi;
                    const bool upper = jt + q > i;
                    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                    part = fma(upper ? sm[q] : 0.0, rsqrt64(upper ? r2 : 1.0), part);
                }
            } else {
                for (int q = 0; q < lim; ++q) {
                    const double dx = sx[q] - xi, dy = sy[q] - yi, dz = sz[q] - zi;
                    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
                    part = fma(sm[q], rsqrt64(r2), part);
                }
            }
            tot += part;
        }
        if (i < n)
            rows[i] = mass[i] * tot;
    }
}

// Neumaier compensated accumulation.
struct CSum {
    double s = 0.0, c = 0.0;
    __device__ void add(double v)
    {
        const double t = s + v;
        if (fabs(s) >= fabs(v)) c += (s - t) + v;
        else c += (v - t) + s;
        s = t;
    }
};

// One workgroup: out[0] = sum_i m_i |v_i|^2 / 2, out[1] = -sum_i rows[i], each
// lane summing a strided slice in order, then lane 0 combining lanes in order.
__global__ __launch_bounds__(WG) void energy_total_kernel(const double *vx, const double *vy,
                                                          const double *vz, const double *mass,
                                                          const double *rows, int64_t n,
                                                          double *out)
{
    __shared__ double ks[WG], kc[WG], ps[WG], pc[WG];
    CSum kin, pot;
    for (int64_t i = threadIdx.x; i < n; i += WG) {
        kin.add(0.5 * mass[i] * (vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i]));
        pot.add(rows[i]);
    }
    ks[threadIdx.x] = kin.s; kc[threadIdx.x] = kin.c;
    ps[threadIdx.x] = pot.s; pc[threadIdx.x] = pot.c;
    __syncthreads();
    if (threadIdx.x == 0) {
        CSum k2, p2;
        for (int t = 0; t < WG; ++t) {
            k2.add(ks[t]); k2.add(kc[t]);
            p2.add(ps[t]); p2.add(pc[t]);
        }
        out[0] = k2.s + k2.c;
        out[1] = -(p2.s + p2.c);
    }
}

hipError_t launch_energy(const nb_system &s, double eps2, double *rows, double *out,
                         hipStream_t st)
{
    const int64_t n = s.n;
    const unsigned blocks = (unsigned)(((n + WG - 1) / WG + 1) / 2);
    hipLaunchKernelGGL(potential_rows_kernel, dim3(blocks), dim3(WG), 0, st, s.x, s.y, s.z, s.m,
                       n, eps2, rows);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(energy_total_kernel, dim3(1), dim3(WG), 0, st, s.vx, s.vy, s.vz, s.m, rows,
                       n, out);
    return hipGetLastError();
}

}  // namespace nbk
