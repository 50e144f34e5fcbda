// C ABI of libnbody.so: argument checking, context and scratch management, the
// force launch plan, and dispatch to the kernels.  See include/nbody.h for the
// contract of every entry point.
#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include "nb_internal.h"

#define NB_VERSION "0.1.0"

namespace {

nb_status fail(nb_ctx *ctx, nb_status code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

nb_status hip_fail(nb_ctx *ctx, hipError_t e, const char *what)
{
    return fail(ctx, NB_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define NB_HIP(ctx, call)                                     \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

nb_status check_system(nb_ctx *ctx, const nb_system *s, bool need_pred)
{
    if (!ctx) return NB_EINVAL;
    if (!s) return fail(ctx, NB_EINVAL, "system is NULL");
    if (s->n < 0 || s->n > (int64_t)INT32_MAX) return fail(ctx, NB_EINVAL, "n out of range");
    if (s->n == 0) return NB_OK;
    const double *need[] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->ax, s->ay, s->az,
                            s->jx, s->jy, s->jz, s->m, s->t, s->dt};
    for (const double *p : need)
        if (!p) return fail(ctx, NB_EINVAL, "a state array is NULL");
    if (need_pred && (!s->xp || !s->yp || !s->zp || !s->vxp || !s->vyp || !s->vzp))
        return fail(ctx, NB_EINVAL, "a predicted array is NULL");
    const bool any32 = s->vxp32 || s->vyp32 || s->vzp32 || s->m32;
    const bool all32 = s->vxp32 && s->vyp32 && s->vzp32 && s->m32;
    if (any32 && !all32) return fail(ctx, NB_EINVAL, "FP32 copies must be all set or all NULL");
    return NB_OK;
}

nb_status ensure_scratch(nb_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->scratch_bytes) return NB_OK;
    NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->scratch) {
        NB_HIP(ctx, hipFree(ctx->scratch));
        ctx->scratch = nullptr;
        ctx->scratch_bytes = 0;
    }
    size_t want = bytes + bytes / 4;
    if (hipMalloc(&ctx->scratch, want) != hipSuccess) {
        ctx->scratch = nullptr;
        (void)hipGetLastError();
        return fail(ctx, NB_ENOMEM, "scratch allocation of %zu bytes failed", want);
    }
    ctx->scratch_bytes = want;
    return NB_OK;
}

// Convert and clear the latched status word (the caller has synchronised and
// copied the word to the pinned mirror).
nb_status take_status(nb_ctx *ctx, int word)
{
    if (word == 0) return NB_OK;
    if (word & NBK_EINDEX) return fail(ctx, NB_EINDEX, "an active index was outside [0, n)");
    if (word & NBK_ENAN) return fail(ctx, NB_ENAN, "non-finite acceleration, jerk or step");
    return fail(ctx, NB_ERANGE, "a time step fell below dt_min");
}

// Copy the first `bytes` of the small device area to the pinned mirror, clear the
// status word, wait, and convert the status.
nb_status sync_small(nb_ctx *ctx, size_t bytes)
{
    NB_HIP(ctx, hipMemcpyAsync(ctx->small_host, ctx->small, bytes, hipMemcpyDeviceToHost,
                               ctx->stream));
    NB_HIP(ctx, hipMemsetAsync(&ctx->small->status, 0, sizeof(int), ctx->stream));
    NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return take_status(ctx, ctx->small_host->status);
}

struct Plan {
    int il, s, b;
};

// Launch plan: enough lanes to fill 256 CUs (about 2^18 lane slots: 4 waves of
// 64 lanes on each of 4 SIMDs per CU) while every lane still walks at least
// 128 j-bodies, so the fixed cost of the final reduction stays small.  Large
// mixed-precision blocks hold two i-bodies per lane to halve LDS traffic per
// interaction.  Pure function of (nj, m, precision).
Plan make_plan(int64_t nj, int32_t m, int precision)
{
    const int64_t target_lanes = (int64_t)1 << 18;
    const int64_t min_j = 128;
    Plan p{(precision == NB_MIXED && m >= (1 << 16)) ? 2 : 1, 1, 1};
    if (m <= 0 || nj <= 0) return p;
    int64_t lanes = (m + p.il - 1) / p.il;
    while (p.s < 64 && lanes * p.s < target_lanes && nj / (p.s * 4) >= min_j)
        p.s *= 4;
    lanes *= p.s;
    int64_t b = 1;
    while (lanes * b < target_lanes && nj / (p.s * b * 2) >= min_j && b < 1024)
        b *= 2;
    p.b = (int)b;
    return p;
}

bool valid_plan(int il, int s, int b)
{
    return (il == 1 || il == 2 || il == 4) && (s == 1 || s == 4 || s == 16 || s == 64) &&
           b >= 1 && b <= 65535;
}

nb_status force_impl(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                     int64_t j0, int64_t j1, double eps, nb_precision prec, Plan plan,
                     double *acc, double *jerk)
{
    nb_status st = check_system(ctx, sys, true);
    if (st != NB_OK) return st;
    if (!(eps > 0.0) || !isfinite(eps)) return fail(ctx, NB_EINVAL, "eps must be > 0 and finite");
    if (prec != NB_FP64 && prec != NB_MIXED) return fail(ctx, NB_EINVAL, "unknown precision");
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    if (j0 < 0 || j1 > sys->n || j0 > j1) return fail(ctx, NB_EINVAL, "bad j-range");
    if (m == 0) return NB_OK;
    if (!acc || !jerk) return fail(ctx, NB_EINVAL, "acc/jerk is NULL");
    if (prec == NB_MIXED && !sys->vxp32)
        return fail(ctx, NB_EINVAL, "mixed precision needs the FP32 copies");
    if (!valid_plan(plan.il, plan.s, plan.b)) return fail(ctx, NB_EINVAL, "invalid plan");

    constexpr int TILE = 512;
    const int64_t nj = j1 - j0;
    int64_t chunk = (nj + plan.b - 1) / plan.b;
    chunk = (chunk + TILE - 1) / TILE * TILE;
    if (chunk < TILE) chunk = TILE;
    const int iwg = (nbk::WG / plan.s) * plan.il;
    dim3 grid((unsigned)((m + iwg - 1) / iwg), (unsigned)plan.b);

    nbk::ForceArgs a{};
    a.xp = sys->xp; a.yp = sys->yp; a.zp = sys->zp;
    a.vx64 = sys->vxp; a.vy64 = sys->vyp; a.vz64 = sys->vzp; a.m64 = sys->m;
    a.vx32 = sys->vxp32; a.vy32 = sys->vyp32; a.vz32 = sys->vzp32; a.m32 = sys->m32;
    a.i_idx = i_idx;
    a.m = m;
    a.n = sys->n;
    a.j0 = j0; a.j1 = j1; a.chunk = chunk;
    a.eps2 = eps * eps;
    a.status = &ctx->small->status;
    double *part = nullptr;
    if (plan.b > 1) {
        st = ensure_scratch(ctx, sizeof(double) * 6 * (size_t)m * (size_t)plan.b);
        if (st != NB_OK) return st;
        part = (double *)ctx->scratch;
        a.out_acc = part;
        a.out_jerk = part + 3 * (int64_t)m;
        a.stride_b = 6 * (int64_t)m;
    } else {
        a.out_acc = acc;
        a.out_jerk = jerk;
        a.stride_b = 0;
    }
    hipError_t e = nbk::launch_force(prec, plan.il, plan.s, grid, a, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "force kernel launch");
    if (plan.b > 1) {
        e = nbk::launch_reduce_partials(part, m, plan.b, acc, jerk, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "partial reduction launch");
    }
    return NB_OK;
}

}  // namespace

extern "C" {

const char *nb_version(void) { return NB_VERSION; }

nb_status nb_ctx_create(nb_ctx **out, int device, void *hip_stream)
{
    if (!out) return NB_EINVAL;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return NB_EINVAL;
    }
    nb_ctx *ctx = new nb_ctx();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    if (hipSetDevice(device) != hipSuccess ||
        hipMalloc((void **)&ctx->small, sizeof(nb_small)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->small_host, sizeof(nb_small), hipHostMallocDefault) != hipSuccess ||
        hipMemset(ctx->small, 0, sizeof(nb_small)) != hipSuccess) {
        (void)hipGetLastError();
        if (ctx->small) (void)hipFree(ctx->small);
        if (ctx->small_host) (void)hipHostFree(ctx->small_host);
        delete ctx;
        return NB_ENOMEM;
    }
    memset(ctx->small_host, 0, sizeof(nb_small));
    *out = ctx;
    return NB_OK;
}

nb_status nb_ctx_destroy(nb_ctx *ctx)
{
    if (!ctx) return NB_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->small) (void)hipFree(ctx->small);
    if (ctx->small_host) (void)hipHostFree(ctx->small_host);
    delete ctx;
    return NB_OK;
}

const char *nb_last_error(const nb_ctx *ctx)
{
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

nb_status nb_sync(nb_ctx *ctx)
{
    if (!ctx) return NB_EINVAL;
    return sync_small(ctx, sizeof(int));
}

nb_status nb_select_active(nb_ctx *ctx, const nb_system *sys, double *t_next_host,
                           int32_t *i_idx, int32_t *m_host)
{
    nb_status st = check_system(ctx, sys, false);
    if (st != NB_OK) return st;
    if (!t_next_host || !m_host) return fail(ctx, NB_EINVAL, "host outputs are NULL");
    if (sys->n == 0) {
        *m_host = 0;
        *t_next_host = INFINITY;
        return NB_OK;
    }
    if (!i_idx) return fail(ctx, NB_EINVAL, "i_idx is NULL");
    hipError_t e = nbk::launch_select(*sys, ctx->small, i_idx, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "selection launch");
    st = sync_small(ctx, offsetof(nb_small, energy));
    *t_next_host = ctx->small_host->t_next;
    *m_host = ctx->small_host->m;
    return st;
}

nb_status nb_predict(nb_ctx *ctx, const nb_system *sys, double t_next)
{
    nb_status st = check_system(ctx, sys, true);
    if (st != NB_OK) return st;
    if (!isfinite(t_next)) return fail(ctx, NB_EINVAL, "t_next must be finite");
    if (sys->n == 0) return NB_OK;
    hipError_t e = nbk::launch_predict(*sys, t_next, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "predict launch");
}

nb_status nb_force_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                          int64_t j0, int64_t j1, double eps, nb_precision precision,
                          double *acc, double *jerk)
{
    Plan p = make_plan(j1 - j0, m, precision);
    return force_impl(ctx, sys, i_idx, m, j0, j1, eps, precision, p, acc, jerk);
}

nb_status nb_force_active_plan(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                               int32_t m, int64_t j0, int64_t j1, double eps,
                               nb_precision precision, int32_t i_per_lane, int32_t lanes_per_i,
                               int32_t j_chunks, double *acc, double *jerk)
{
    Plan p{i_per_lane, lanes_per_i, j_chunks};
    return force_impl(ctx, sys, i_idx, m, j0, j1, eps, precision, p, acc, jerk);
}

void nb_force_plan(int64_t nj, int32_t m, nb_precision precision, int32_t *i_per_lane,
                   int32_t *lanes_per_i, int32_t *j_chunks)
{
    Plan p = make_plan(nj, m, precision);
    if (i_per_lane) *i_per_lane = p.il;
    if (lanes_per_i) *lanes_per_i = p.s;
    if (j_chunks) *j_chunks = p.b;
}

nb_status nb_init_steps(nb_ctx *ctx, const nb_system *sys, const double *acc,
                        const double *jerk, double eta_s, double dt_max, double dt_min)
{
    nb_status st = check_system(ctx, sys, false);
    if (st != NB_OK) return st;
    if (!(eta_s > 0.0) || !(dt_max > 0.0) || !(dt_min > 0.0) || dt_min > dt_max)
        return fail(ctx, NB_EINVAL, "need eta_s > 0 and 0 < dt_min <= dt_max");
    if (sys->n == 0) return NB_OK;
    if (!acc || !jerk) return fail(ctx, NB_EINVAL, "acc/jerk is NULL");
    hipError_t e = nbk::launch_init_steps(*sys, acc, jerk, eta_s, dt_max, dt_min,
                                          &ctx->small->status, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps launch");
}

nb_status nb_correct(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                     const double *acc, const double *jerk, double t_next, double eta,
                     double dt_max, double dt_min)
{
    nb_status st = check_system(ctx, sys, true);
    if (st != NB_OK) return st;
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    if (!(eta > 0.0) || !(dt_max > 0.0) || !(dt_min > 0.0) || dt_min > dt_max)
        return fail(ctx, NB_EINVAL, "need eta > 0 and 0 < dt_min <= dt_max");
    if (!isfinite(t_next)) return fail(ctx, NB_EINVAL, "t_next must be finite");
    if (m == 0) return NB_OK;
    if (!acc || !jerk) return fail(ctx, NB_EINVAL, "acc/jerk is NULL");
    hipError_t e = nbk::launch_correct(*sys, i_idx, m, acc, jerk, t_next, eta, dt_max, dt_min,
                                       &ctx->small->status, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "correct launch");
}

nb_status nb_energy(nb_ctx *ctx, const nb_system *sys, double eps, double *kinetic_host,
                    double *potential_host)
{
    nb_status st = check_system(ctx, sys, false);
    if (st != NB_OK) return st;
    if (!(eps >= 0.0) || !isfinite(eps)) return fail(ctx, NB_EINVAL, "eps must be >= 0");
    if (!kinetic_host || !potential_host) return fail(ctx, NB_EINVAL, "host outputs are NULL");
    if (sys->n == 0) {
        *kinetic_host = 0.0;
        *potential_host = 0.0;
        return NB_OK;
    }
    st = ensure_scratch(ctx, sizeof(double) * (size_t)sys->n);
    if (st != NB_OK) return st;
    hipError_t e = nbk::launch_energy(*sys, eps * eps, (double *)ctx->scratch, ctx->small->energy,
                                      ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "energy launch");
    st = sync_small(ctx, offsetof(nb_small, blockval));
    *kinetic_host = ctx->small_host->energy[0];
    *potential_host = ctx->small_host->energy[1];
    return st;
}

}  // extern "C"
