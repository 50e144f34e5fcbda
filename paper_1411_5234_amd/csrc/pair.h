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

// v plus the value that DPP control CTRL moves into this lane (within a row of 16
// lanes; every lane of the wave must be active).  Both 32-bit halves move alike.
template <int CTRL>
__device__ __forceinline__ double dpp_add(double v)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
    const unsigned long long q = ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
    return v + __longlong_as_double((long long)q);
}

// Sum over the S consecutive lanes of a group (S = 1, 4, 16 or 64), the same value
// in every lane of the group.  Inside a row the partners come from DPP lane moves
// (register to register): lanes 2 apart and 1 apart within a quad, then the
// half-row mirror (the other quad of each 8 lanes) and the row mirror (the other
// half of each 16); rows are then combined with cross-row shuffles.
template <int S>
__device__ __forceinline__ double group_sum(double v)
{
    static_assert(S == 1 || S == 4 || S == 16 || S == 64, "group size");
    if constexpr (S >= 4) {
        v = dpp_add<0x4E>(v);    // quad_perm [2,3,0,1]
        v = dpp_add<0xB1>(v);    // quad_perm [1,0,3,2]
    }
    if constexpr (S >= 16) {
        v = dpp_add<0x141>(v);   // row_half_mirror
        v = dpp_add<0x140>(v);   // row_mirror
    }
    if constexpr (S == 64) {
        v += __shfl_xor(v, 16, 64);
        v += __shfl_xor(v, 32, 64);
    }
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

#ifndef NBK_MIXED_WAVES
#define NBK_MIXED_WAVES 1
#endif

// Running FP64 total of a lane's FP32 run sums.
struct Total {
    double s = 0.0;
    __device__ __forceinline__ void add(float v) { s += (double)v; }
    __device__ __forceinline__ double value() const { return s; }
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
