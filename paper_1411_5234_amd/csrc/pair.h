// Device helpers shared by the pair-force kernels of both Hermite orders:
// FP64 reciprocal square root, lane-group sums, the i-body position forms
// (FP64 or double-single), the position difference, the FP32 run-sum totals
// and the LDS j-tile of the mixed and double-single kernels.
#pragma once

#include "nb_internal.h"

namespace nbk {

// FP64 reciprocal square root: hardware estimate refined by two Newton steps
// y <- y (3 - s y^2) / 2 written as y + y (1/2 - (s/2) y^2).
__device__ __forceinline__ double rsqrt64(double s)
{
    double y = __builtin_amdgcn_rsq(s);
    const double hs = 0.5 * s;
    double e = fma(-hs, y * y, 0.5);
    y = fma(y, e, y);
    e = fma(-hs, y * y, 0.5);
    y = fma(y, e, y);
    return y;
}

template <int S>
__device__ __forceinline__ double group_sum(double v)
{
    // butterfly over the S consecutive lanes of a group (S divides 64)
#pragma unroll
    for (int off = S / 2; off >= 1; off >>= 1)
        v += __shfl_xor(v, off, S);
    return v;
}

// i-body position: FP64 (mixed) or a double-single pair (DS).
template <bool DS>
struct IPos;
template <>
struct IPos<false> {
    double x, y, z;
};
template <>
struct IPos<true> {
    float xh, yh, zh, xl, yl, zl;
};

// One j-body of a tile, read from LDS.
template <bool DS>
struct JBody;
template <>
struct JBody<false> {
    double x, y, z;
    float vx, vy, vz, m;
};
template <>
struct JBody<true> {
    float xh, yh, zh, xl, yl, zl, vx, vy, vz, m;
};

// Split a double into hi = its FP32 rounding and lo = the FP32 rounding of the rest.
__device__ __forceinline__ void split_ds(double v, float &hi, float &lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

// Position difference x_j - x_i rounded to FP32.  Mixed: formed in FP64 and
// converted.  DS (the double-single alternative of Sec. 2 item 4): formed from
// the hi and lo parts as (xj_hi - xi_hi) + (xj_lo - xi_lo) in FP32; the hi
// difference is exact when the bodies are close (Sterbenz) and otherwise
// rounded relative to the result, so dx carries about one FP32 rounding.
__device__ __forceinline__ void diff(const JBody<false> &j, const IPos<false> &i, float &dx,
                                     float &dy, float &dz)
{
    dx = (float)(j.x - i.x);
    dy = (float)(j.y - i.y);
    dz = (float)(j.z - i.z);
}
__device__ __forceinline__ void diff(const JBody<true> &j, const IPos<true> &i, float &dx,
                                     float &dy, float &dz)
{
    dx = (j.xh - i.xh) + (j.xl - i.xl);
    dy = (j.yh - i.yh) + (j.yl - i.yl);
    dz = (j.zh - i.zh) + (j.zl - i.zl);
}

#ifndef NBK_KAHAN
#define NBK_KAHAN 0
#endif
#ifndef NBK_MIXED_WAVES
#define NBK_MIXED_WAVES 1
#endif

// Running total of the FP32 run sums: FP64, or (NBK_KAHAN) an FP32 Kahan pair.
struct Total {
#if NBK_KAHAN
    float s = 0.f, c = 0.f;
    __device__ __forceinline__ void add(float v)
    {
        const float y = v - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
#else
    double s = 0.0;
    __device__ __forceinline__ void add(float v) { s += (double)v; }
    __device__ __forceinline__ double value() const { return s; }
#endif
};

// LDS tile of a mixed or DS kernel: 40 bytes per j-body either way.
template <bool DS>
struct Tile;
template <>
struct Tile<false> {
    double x[TILE], y[TILE], z[TILE];
    float vx[TILE], vy[TILE], vz[TILE], m[TILE];
    __device__ __forceinline__ void put(int q, double px, double py, double pz, float pvx,
                                        float pvy, float pvz, float pm)
    {
        x[q] = px; y[q] = py; z[q] = pz;
        vx[q] = pvx; vy[q] = pvy; vz[q] = pvz; m[q] = pm;
    }
    __device__ __forceinline__ JBody<false> get(int q) const
    {
        return JBody<false>{x[q], y[q], z[q], vx[q], vy[q], vz[q], m[q]};
    }
};
template <>
struct Tile<true> {
    float xh[TILE], yh[TILE], zh[TILE], xl[TILE], yl[TILE], zl[TILE];
    float vx[TILE], vy[TILE], vz[TILE], m[TILE];
    __device__ __forceinline__ void put(int q, double px, double py, double pz, float pvx,
                                        float pvy, float pvz, float pm)
    {
        split_ds(px, xh[q], xl[q]);
        split_ds(py, yh[q], yl[q]);
        split_ds(pz, zh[q], zl[q]);
        vx[q] = pvx; vy[q] = pvy; vz[q] = pvz; m[q] = pm;
    }
    __device__ __forceinline__ JBody<true> get(int q) const
    {
        return JBody<true>{xh[q], yh[q], zh[q], xl[q], yl[q], zl[q], vx[q], vy[q], vz[q], m[q]};
    }
};

__device__ __forceinline__ IPos<false> ipos(double x, double y, double z, IPos<false> *)
{
    return IPos<false>{x, y, z};
}
__device__ __forceinline__ IPos<true> ipos(double x, double y, double z, IPos<true> *)
{
    IPos<true> r;
    split_ds(x, r.xh, r.xl);
    split_ds(y, r.yh, r.yl);
    split_ds(z, r.zh, r.zl);
    return r;
}

}  // namespace nbk
