// Pair-force kernels of the 6th-order Hermite scheme: acceleration, jerk and
// snap of the active block (Eq. 1 with the softening of Eq. 2 and its first two
// time derivatives along the predicted motion; the paper's HiGPUs integrates
// with this scheme, Sec. 2 item 1).  gfx950, wave64.
//
// Same work decomposition as the 4th-order kernels: IL i-bodies per lane group
// in VGPRs, S lanes per group splitting each tile's j-bodies, LDS tiles of
// j-bodies in structure-of-arrays form, B chunks of the j-range per i-block
// with FP64 partials summed in a fixed order, and a table of items per launch.
// Each j-body additionally brings its predicted acceleration (12 bytes in FP32,
// 24 in FP64), and each i-body keeps nine sums instead of six.
//
// Pair terms, with r, w, b the relative predicted position, velocity and
// acceleration, s = |r|^2 + eps^2, mu = m_j s^(-3/2), alpha = (r.w)/s and
// beta = (|w|^2 + r.b)/s + alpha^2:
//   A = mu r,   J = mu u with u = w - 3 alpha r,
//   S = mu (b - 6 alpha u - 3 beta r).
#include "pair.h"
#include "launch.h"

namespace nbk {

// The three terms of one j-body on one i-body in FP32, added to the run sums.
__device__ __forceinline__ void pair6_f32(float dx, float dy, float dz, float dvx, float dvy,
                                          float dvz, float dax, float day, float daz, float mj,
                                          float eps2, float (&a)[3], float (&jk)[3],
                                          float (&sn)[3])
{
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps2)));
    const float rw = fmaf(dx, dvx, fmaf(dy, dvy, dz * dvz));
    const float ww = fmaf(dvx, dvx, fmaf(dvy, dvy, dvz * dvz));
    const float rb = fmaf(dx, dax, fmaf(dy, day, dz * daz));
    const float rinv = __builtin_amdgcn_rsqf(r2);
    const float rinv2 = rinv * rinv;
    const float mu = mj * rinv * rinv2;
    const float al = rw * rinv2;
    const float be = fmaf(al, al, (ww + rb) * rinv2);
    const float c3a = -3.0f * al, c6a = -6.0f * al, c3b = -3.0f * be;
    const float ux = fmaf(c3a, dx, dvx), uy = fmaf(c3a, dy, dvy), uz = fmaf(c3a, dz, dvz);
    const float sx = fmaf(c6a, ux, fmaf(c3b, dx, dax));
    const float sy = fmaf(c6a, uy, fmaf(c3b, dy, day));
    const float sz = fmaf(c6a, uz, fmaf(c3b, dz, daz));
    a[0] = fmaf(mu, dx, a[0]);
    a[1] = fmaf(mu, dy, a[1]);
    a[2] = fmaf(mu, dz, a[2]);
    jk[0] = fmaf(mu, ux, jk[0]);
    jk[1] = fmaf(mu, uy, jk[1]);
    jk[2] = fmaf(mu, uz, jk[2]);
    sn[0] = fmaf(mu, sx, sn[0]);
    sn[1] = fmaf(mu, sy, sn[1]);
    sn[2] = fmaf(mu, sz, sn[2]);
}

// The same in FP64 (the NB_FP64 kernel), with the refined reciprocal square root.
__device__ __forceinline__ void pair6_f64(double dx, double dy, double dz, double dvx,
                                          double dvy, double dvz, double dax, double day,
                                          double daz, double mj, double eps2, double (&a)[3],
                                          double (&jk)[3], double (&sn)[3])
{
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, eps2)));
    const double rw = fma(dx, dvx, fma(dy, dvy, dz * dvz));
    const double ww = fma(dvx, dvx, fma(dvy, dvy, dvz * dvz));
    const double rb = fma(dx, dax, fma(dy, day, dz * daz));
    const double rinv = rsqrt64(r2);
    const double rinv2 = rinv * rinv;
    const double mu = mj * rinv * rinv2;
    const double al = rw * rinv2;
    const double be = fma(al, al, (ww + rb) * rinv2);
    const double c3a = -3.0 * al, c6a = -6.0 * al, c3b = -3.0 * be;
    const double ux = fma(c3a, dx, dvx), uy = fma(c3a, dy, dvy), uz = fma(c3a, dz, dvz);
    const double sx = fma(c6a, ux, fma(c3b, dx, dax));
    const double sy = fma(c6a, uy, fma(c3b, dy, day));
    const double sz = fma(c6a, uz, fma(c3b, dz, daz));
    a[0] = fma(mu, dx, a[0]);
    a[1] = fma(mu, dy, a[1]);
    a[2] = fma(mu, dz, a[2]);
    jk[0] = fma(mu, ux, jk[0]);
    jk[1] = fma(mu, uy, jk[1]);
    jk[2] = fma(mu, uz, jk[2]);
    sn[0] = fma(mu, sx, sn[0]);
    sn[1] = fma(mu, sy, sn[1]);
    sn[2] = fma(mu, sz, sn[2]);
}

// Active index k of an item, checked against n (an out-of-range index latches
// NBK_EINDEX and is replaced by body 0; its output is still written).
__device__ __forceinline__ int64_t active_body(const Item &p, int64_t k)
{
    if (k >= p.m)
        return 0;
    const int64_t i = p.i_idx ? (int64_t)p.i_idx[k] : k;
    if (i < 0 || i >= p.s.n) {
        atomicOr(p.status, (int)NBK_EINDEX);
        return 0;
    }
    return i;
}

// Write the nine sums of active body k: to the outputs, or to this chunk's
// partials when the j-range is split.
__device__ __forceinline__ void store9(const Item &p, int64_t bidx, int64_t k, const double (&A)[3],
                                       const double (&J)[3], const double (&Sn)[3])
{
    const int64_t m = p.m;
    double *oa, *oj, *os;
    if (p.b > 1) {
        double *base = p.part + bidx * 9 * m;
        oa = base;
        oj = base + 3 * m;
        os = base + 6 * m;
    } else {
        oa = p.acc;
        oj = p.jerk;
        os = p.snap;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        oa[c * m + k] = A[c];
        oj[c * m + k] = J[c];
        os[c * m + k] = Sn[c];
    }
}

// LDS tile of the 6th-order mixed and DS kernels: one 64-byte record per j-body
// (position as FP64 or as double-single hi/lo parts, then FP32 velocity, mass
// and predicted acceleration), read with 16-byte LDS loads at immediate offsets
// from one byte offset b = 64 q that the kernel keeps in a VGPR.  This takes
// the address arithmetic of the structure-of-arrays tile (one SGPR-to-VGPR move
// per array and j pair) out of the pair loop.  TILE6_PAD leaves room for the
// read one run past the tile.
constexpr int TILE6_PAD = TILE + 64;
template <bool DS>
struct Rec6;
template <>
struct Rec6<false> {
    double x, y, z;
    float vx, vy, vz, m, ax, ay, az, pad;
};
template <>
struct Rec6<true> {
    float xh, yh, zh, xl, yl, zl, vx, vy, vz, m, ax, ay, az, pad0, pad1, pad2;
};

template <bool DS>
struct Tile6 {
    static constexpr int REC = 64;
    struct alignas(16) Slot {
        Rec6<DS> e;
    };
    static_assert(sizeof(Slot) == 64, "64-byte j records");
    Slot r[TILE6_PAD];
    __device__ __forceinline__ void put(int q, double px, double py, double pz, float pvx,
                                        float pvy, float pvz, float pm, float pax, float pay,
                                        float paz)
    {
        Rec6<DS> e;
        if constexpr (DS) {
            split_ds(px, e.xh, e.xl);
            split_ds(py, e.yh, e.yl);
            split_ds(pz, e.zh, e.zl);
            e.pad0 = 0.f; e.pad1 = 0.f; e.pad2 = 0.f;
        } else {
            e.x = px; e.y = py; e.z = pz;
            e.pad = 0.f;
        }
        e.vx = pvx; e.vy = pvy; e.vz = pvz; e.m = pm;
        e.ax = pax; e.ay = pay; e.az = paz;
        r[q].e = e;
    }
    // j-body and its predicted acceleration at byte offset b (four 16-byte loads)
    __device__ __forceinline__ JBody<DS> at(int b, float &ax, float &ay, float &az) const
    {
        const char *p = reinterpret_cast<const char *>(r) + b;
        const float4 c = *reinterpret_cast<const float4 *>(p + 16);
        const float4 d = *reinterpret_cast<const float4 *>(p + 32);
        const float4 e = *reinterpret_cast<const float4 *>(p + 48);
        // both layouts end in (vz, m, ax, ay), (az, pad...)
        ax = d.z; ay = d.w; az = e.x;
        if constexpr (DS) {
            const float4 a = *reinterpret_cast<const float4 *>(p);
            return JBody<true>{a.x, a.y, a.z, a.w, c.x, c.y, c.z, c.w, d.x, d.y};
        } else {
            const double2 xy = *reinterpret_cast<const double2 *>(p);
            const double z = __hiloint2double(__float_as_int(c.y), __float_as_int(c.x));
            return JBody<false>{xy.x, xy.y, z, c.z, c.w, d.x, d.y};
        }
    }
};

// The value v in a VGPR, so that offsets derived from it stay in VGPRs.
__device__ __forceinline__ int in_vgpr(int v)
{
    int r;
    asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
}

template <int IL, int S, int F, bool DS>
__global__ __launch_bounds__(WG, NBK_MIXED_WAVES) void force6_mixed_kernel(const Item *items,
                                                                           const int64_t *starts,
                                                                           int n_items)
{
    __shared__ Tile6<DS> tile;

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
    const double *xp = p.s.xp, *yp = p.s.yp, *zp = p.s.zp;
    const float *vx32 = p.s.vxp32, *vy32 = p.s.vyp32, *vz32 = p.s.vzp32, *m32 = p.s.m32;
    const float *ax32 = p.h6.axp32, *ay32 = p.h6.ayp32, *az32 = p.h6.azp32;

    IPos<DS> pi[IL];
    float vxi[IL], vyi[IL], vzi[IL], axi[IL], ayi[IL], azi[IL];
    Total A[IL][3], J[IL][3], Sn[IL][3];
#pragma unroll
    for (int u = 0; u < IL; ++u) {
        const int64_t i = active_body(p, kbase + u);
        pi[u] = ipos(xp[i], yp[i], zp[i], (IPos<DS> *)nullptr);
        vxi[u] = vx32[i]; vyi[u] = vy32[i]; vzi[u] = vz32[i];
        axi[u] = ax32[i]; ayi[u] = ay32[i]; azi[u] = az32[i];
    }

    for (int64_t jt = jb; jt < je; jt += TILE) {
        __syncthreads();
        for (int q = tid; q < TILE; q += WG) {
            const int64_t j = jt + q;
            if (j < je)
                tile.put(q, xp[j], yp[j], zp[j], vx32[j], vy32[j], vz32[j], m32[j], ax32[j],
                         ay32[j], az32[j]);
            else   // padding: zero mass contributes exactly zero
                tile.put(q, 0.0, 0.0, 0.0, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f);
        }
        __syncthreads();
        const int lim = (int)min<int64_t>(TILE, je - jt);
        for (int kk = 0; kk < lim; kk += S * F) {
            float a32[IL][3], j32[IL][3], s32[IL][3];
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) { a32[u][c] = 0.f; j32[u][c] = 0.f; s32[u][c] = 0.f; }
            // byte offset of this lane's j; the next j is read ahead of this one's
            // arithmetic (one run past the tile at the last step, into the padding)
            int b = in_vgpr(Tile6<DS>::REC * (kk + s));
            float cax, cay, caz;
            JBody<DS> cur = tile.at(b, cax, cay, caz);
#pragma unroll NBK_UNROLL
            for (int f = 0; f < F; ++f) {
                b += Tile6<DS>::REC * S;
                float nax, nay, naz;
                const JBody<DS> nxt = tile.at(b, nax, nay, naz);
#pragma unroll
                for (int u = 0; u < IL; ++u) {
                    float dx, dy, dz;
                    diff(cur, pi[u], dx, dy, dz);
                    pair6_f32(dx, dy, dz, cur.vx - vxi[u], cur.vy - vyi[u], cur.vz - vzi[u],
                              cax - axi[u], cay - ayi[u], caz - azi[u], cur.m, eps2, a32[u],
                              j32[u], s32[u]);
                }
                cur = nxt;
                cax = nax; cay = nay; caz = naz;
            }
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A[u][c].add(a32[u][c]);
                    J[u][c].add(j32[u][c]);
                    Sn[u][c].add(s32[u][c]);
                }
        }
    }

#pragma unroll
    for (int u = 0; u < IL; ++u) {
        double At[3], Jt[3], St[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            At[c] = A[u][c].value();
            Jt[c] = J[u][c].value();
            St[c] = Sn[u][c].value();
            if constexpr (S > 1) {
                At[c] = group_sum<S>(At[c]);
                Jt[c] = group_sum<S>(Jt[c]);
                St[c] = group_sum<S>(St[c]);
            }
        }
        const int64_t k = kbase + u;
        if (s == 0 && k < p.m)
            store9(p, bidx, k, At, Jt, St);
    }
}

template <int IL, int S, int F>
__global__ __launch_bounds__(WG) void force6_fp64_kernel(const Item *items, const int64_t *starts,
                                                         int n_items)
{
    __shared__ double sx[TILE], sy[TILE], sz[TILE];
    __shared__ double svx[TILE], svy[TILE], svz[TILE];
    __shared__ double sax[TILE], say[TILE], saz[TILE], sm[TILE];

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
    const double *xp = p.s.xp, *yp = p.s.yp, *zp = p.s.zp;
    const double *vxp = p.s.vxp, *vyp = p.s.vyp, *vzp = p.s.vzp, *mass = p.s.m;
    const double *axp = p.h6.axp, *ayp = p.h6.ayp, *azp = p.h6.azp;

    double xi[IL], yi[IL], zi[IL], vxi[IL], vyi[IL], vzi[IL], axi[IL], ayi[IL], azi[IL];
    double A[IL][3], J[IL][3], Sn[IL][3];
#pragma unroll
    for (int u = 0; u < IL; ++u) {
        const int64_t i = active_body(p, kbase + u);
        xi[u] = xp[i]; yi[u] = yp[i]; zi[u] = zp[i];
        vxi[u] = vxp[i]; vyi[u] = vyp[i]; vzi[u] = vzp[i];
        axi[u] = axp[i]; ayi[u] = ayp[i]; azi[u] = azp[i];
#pragma unroll
        for (int c = 0; c < 3; ++c) { A[u][c] = 0.0; J[u][c] = 0.0; Sn[u][c] = 0.0; }
    }

    for (int64_t jt = jb; jt < je; jt += TILE) {
        __syncthreads();
        for (int q = tid; q < TILE; q += WG) {
            const int64_t j = jt + q;
            const bool in = j < je;
            sx[q] = in ? xp[j] : 0.0; sy[q] = in ? yp[j] : 0.0; sz[q] = in ? zp[j] : 0.0;
            svx[q] = in ? vxp[j] : 0.0; svy[q] = in ? vyp[j] : 0.0; svz[q] = in ? vzp[j] : 0.0;
            sax[q] = in ? axp[j] : 0.0; say[q] = in ? ayp[j] : 0.0; saz[q] = in ? azp[j] : 0.0;
            sm[q] = in ? mass[j] : 0.0;
        }
        __syncthreads();
        const int lim = (int)min<int64_t>(TILE, je - jt);
        for (int kk = 0; kk < lim; kk += S * F) {
            double at[IL][3], jt3[IL][3], st3[IL][3];
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) { at[u][c] = 0.0; jt3[u][c] = 0.0; st3[u][c] = 0.0; }
#pragma unroll 2
            for (int f = 0; f < F; ++f) {
                const int q = kk + f * S + s;
                const double xj = sx[q], yj = sy[q], zj = sz[q];
                const double vxj = svx[q], vyj = svy[q], vzj = svz[q];
                const double axj = sax[q], ayj = say[q], azj = saz[q], mj = sm[q];
#pragma unroll
                for (int u = 0; u < IL; ++u)
                    pair6_f64(xj - xi[u], yj - yi[u], zj - zi[u], vxj - vxi[u], vyj - vyi[u],
                              vzj - vzi[u], axj - axi[u], ayj - ayi[u], azj - azi[u], mj, eps2,
                              at[u], jt3[u], st3[u]);
            }
#pragma unroll
            for (int u = 0; u < IL; ++u)
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    A[u][c] += at[u][c];
                    J[u][c] += jt3[u][c];
                    Sn[u][c] += st3[u][c];
                }
        }
    }

#pragma unroll
    for (int u = 0; u < IL; ++u) {
        if constexpr (S > 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                A[u][c] = group_sum<S>(A[u][c]);
                J[u][c] = group_sum<S>(J[u][c]);
                Sn[u][c] = group_sum<S>(Sn[u][c]);
            }
        }
        const int64_t k = kbase + u;
        if (s == 0 && k < p.m)
            store9(p, bidx, k, A[u], J[u], Sn[u]);
    }
}

template <int S>
constexpr int fold6_mixed() { return (TILE / S) < NBK_FOLD ? (TILE / S) : NBK_FOLD; }
template <int S>
constexpr int fold6_fp64() { return TILE / S; }

template <int IL, int S>
static hipError_t launch6_one(int precision, const Table &t, hipStream_t st)
{
    const dim3 grid((unsigned)t.blocks);
    if (precision == NB_MIXED)
        hipLaunchKernelGGL((force6_mixed_kernel<IL, S, fold6_mixed<S>(), false>), grid, dim3(WG),
                           0, st, t.items, t.starts, t.n);
    else if (precision == NB_DS)
        hipLaunchKernelGGL((force6_mixed_kernel<IL, S, fold6_mixed<S>(), true>), grid, dim3(WG),
                           0, st, t.items, t.starts, t.n);
    else
        hipLaunchKernelGGL((force6_fp64_kernel<IL, S, fold6_fp64<S>()>), grid, dim3(WG), 0, st,
                           t.items, t.starts, t.n);
    return hipGetLastError();
}

template <int IL>
static hipError_t launch6_il(int precision, int s, const Table &t, hipStream_t st)
{
    switch (s) {
    case 1: return launch6_one<IL, 1>(precision, t, st);
    case 4: return launch6_one<IL, 4>(precision, t, st);
    case 16: return launch6_one<IL, 16>(precision, t, st);
    case 64: return launch6_one<IL, 64>(precision, t, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_force6(int precision, int il, int s, const Table &t, hipStream_t st)
{
    if (t.blocks <= 0) return hipSuccess;
    switch (il) {
    case 1: return launch6_il<1>(precision, s, t, st);
    case 2: return launch6_il<2>(precision, s, t, st);
    case 4: return launch6_il<4>(precision, s, t, st);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nbk
