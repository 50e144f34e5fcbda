// C ABI of libnbody.so: argument checking, context and scratch management, the
// force launch plan, item tables, and dispatch to the kernels.  See
// include/nbody.h for the contract of every entry point.
#include <math.h>
#include <stdarg.h>
#include <stddef.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "ctx.h"
#include "launch.h"

#define NB_VERSION "0.5.0"

using nbk::Item;
using nbk::SelResult;
using nbk::Table;

// Longest host spin on the selection flag before a stream synchronization, in
// microseconds.
constexpr long SEL_SPIN_US = 5000;

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

#define NB_HIP(ctx, call)                                      \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #call); \
    } while (0)

#define NB_TRY(call)                    \
    do {                                \
        nb_status s_ = (call);          \
        if (s_ != NB_OK) return s_;     \
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

nb_status check_h6(nb_ctx *ctx, const nb_system *s, const nb_hermite6 *h)
{
    if (!h) return fail(ctx, NB_EINVAL, "6th-order arrays are NULL");
    if (s->n == 0) return NB_OK;
    const double *need[] = {h->sx, h->sy, h->sz, h->cx, h->cy, h->cz, h->axp, h->ayp, h->azp};
    for (const double *p : need)
        if (!p) return fail(ctx, NB_EINVAL, "a 6th-order array is NULL");
    const bool any32 = h->axp32 || h->ayp32 || h->azp32;
    const bool all32 = h->axp32 && h->ayp32 && h->azp32;
    if (any32 && !all32) return fail(ctx, NB_EINVAL, "FP32 copies must be all set or all NULL");
    if (all32 && !s->vxp32)
        return fail(ctx, NB_EINVAL, "FP32 predicted accelerations need the system's FP32 copies");
    return NB_OK;
}

// Grow a device buffer to at least `bytes` (waits for the stream before freeing).
nb_status grow(nb_ctx *ctx, void **buf, size_t *have, size_t bytes, const char *what)
{
    if (bytes <= *have) return NB_OK;
    NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    if (*buf) {
        NB_HIP(ctx, hipFree(*buf));
        *buf = nullptr;
        *have = 0;
    }
    const size_t want = bytes + bytes / 4 + 256;
    if (hipMalloc(buf, want) != hipSuccess) {
        *buf = nullptr;
        (void)hipGetLastError();
        return fail(ctx, NB_ENOMEM, "%s: allocation of %zu bytes failed", what, want);
    }
    *have = want;
    return NB_OK;
}

// The flag word that follows the selection results in the mapped ring, as the
// host and the device address it.
unsigned *sel_flag_host(nb_ctx *ctx) { return (unsigned *)((char *)ctx->res_host + ctx->res_bytes); }
unsigned *sel_flag_dev(nb_ctx *ctx) { return (unsigned *)((char *)ctx->res_host_dev + ctx->res_bytes); }

nb_status ensure_res(nb_ctx *ctx, size_t bytes)
{
    if (bytes <= ctx->res_bytes) return NB_OK;
    size_t have = ctx->res_bytes;
    NB_TRY(grow(ctx, &ctx->res, &have, bytes, "selection results"));
    if (ctx->res_host) (void)hipHostFree(ctx->res_host);
    ctx->res_host = nullptr;
    ctx->res_host_dev = nullptr;
    ctx->res_bytes = 0;
    // Coherent and mapped: the status kernel writes the results here directly,
    // then a flag word after them (at offset `have`), and the host reads them once
    // it sees the flag or that kernel has completed (no copy).
    if (hipHostMalloc(&ctx->res_host, have + 64, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess) {
        (void)hipGetLastError();
        ctx->res_host = nullptr;
        return fail(ctx, NB_ENOMEM, "pinned selection results");
    }
    if (hipHostGetDevicePointer(&ctx->res_host_dev, ctx->res_host, 0) != hipSuccess ||
        !ctx->res_host_dev) {
        (void)hipGetLastError();
        (void)hipHostFree(ctx->res_host);
        ctx->res_host = nullptr;
        ctx->res_host_dev = nullptr;
        return fail(ctx, NB_EDEVICE, "device address of the pinned selection results");
    }
    ctx->res_bytes = have;
    __atomic_store_n(sel_flag_host(ctx), 0u, __ATOMIC_RELAXED);
    return NB_OK;
}

// Copy `bytes` of host data into the pinned ring and enqueue its upload to the
// device ring; returns the device address.  The upload is a small kernel on
// `stream` that reads the mapped ring (no copy engine, so no wait between
// queues).  Regions are reused only after the stream has drained (a wrap waits
// for the stream), so an upload is never overwritten before the copy and the
// kernels that read it have run.
nb_status upload(nb_ctx *ctx, const void *src, size_t bytes, const void **dev)
{
    const size_t need = (bytes + 255) / 256 * 256;
    if (need > ctx->stage_bytes) {
        NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
        if (ctx->stage_dev) (void)hipFree(ctx->stage_dev);
        ctx->stage_host = nullptr;
        ctx->stage_host_dev = nullptr;
        ctx->stage_dev = nullptr;
        ctx->stage_bytes = 0;
        const size_t want = std::max(need * 2, (size_t)8 << 20);
        void *hd = nullptr;
        if (hipHostMalloc((void **)&ctx->stage_host, want,
                          hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer(&hd, ctx->stage_host, 0) != hipSuccess || !hd ||
            hipMalloc((void **)&ctx->stage_dev, want) != hipSuccess) {
            (void)hipGetLastError();
            if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
            ctx->stage_host = nullptr;
            ctx->stage_dev = nullptr;
            return fail(ctx, NB_ENOMEM, "item table staging");
        }
        ctx->stage_host_dev = (const char *)hd;
        ctx->stage_bytes = want;
        ctx->stage_off = 0;
    }
    if (ctx->stage_off + need > ctx->stage_bytes) {
        NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
        ctx->stage_off = 0;
    }
    memcpy(ctx->stage_host + ctx->stage_off, src, bytes);
    hipError_t e = nbk::launch_upload(ctx->stage_host_dev + ctx->stage_off,
                                      ctx->stage_dev + ctx->stage_off, need, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "table upload launch");
    *dev = ctx->stage_dev + ctx->stage_off;
    ctx->stage_off += need;
    return NB_OK;
}

// Tables of one call that are uploaded together: make_table appends each to
// `buf` and records where its pointers go; flush uploads the buffer in one copy
// and sets them.  The Tables must stay in place until the flush.
struct Staging {
    std::vector<char> buf;
    struct Fix {
        Table *t;
        size_t items_off, starts_off;
    };
    std::vector<Fix> fix;
};

nb_status flush(nb_ctx *ctx, Staging *st)
{
    if (st->fix.empty()) return NB_OK;
    const void *d = nullptr;
    NB_TRY(upload(ctx, st->buf.data(), st->buf.size(), &d));
    for (const Staging::Fix &f : st->fix) {
        f.t->items = (const Item *)((const char *)d + f.items_off);
        f.t->starts = (const int64_t *)((const char *)d + f.starts_off);
    }
    st->buf.clear();
    st->fix.clear();
    return NB_OK;
}

// The table of the items with a positive workgroup count: items, then their
// workgroup offsets.  Uploaded at once (st == nullptr) or at st's flush.
nb_status make_table(nb_ctx *ctx, const std::vector<Item> &items,
                     const std::vector<int64_t> &blocks, Table *t, Staging *st = nullptr)
{
    std::vector<Item> keep;
    std::vector<int64_t> starts;
    int64_t total = 0;
    for (size_t k = 0; k < items.size(); ++k) {
        if (blocks[k] <= 0) continue;
        keep.push_back(items[k]);
        starts.push_back(total);
        total += blocks[k];
    }
    starts.push_back(total);
    t->n = (int)keep.size();
    t->blocks = total;
    t->items = nullptr;
    t->starts = nullptr;
    if (total == 0) return NB_OK;
    if (total > (int64_t)INT32_MAX) return fail(ctx, NB_EINVAL, "launch too large");
    static_assert(sizeof(Item) % 8 == 0, "Item size");
    const size_t ib = keep.size() * sizeof(Item), sb = starts.size() * sizeof(int64_t);
    Staging local;
    Staging *s = st ? st : &local;
    const size_t off = (s->buf.size() + 255) / 256 * 256;
    s->buf.resize(off + ib + sb);
    memcpy(s->buf.data() + off, keep.data(), ib);
    memcpy(s->buf.data() + off + ib, starts.data(), sb);
    s->fix.push_back({t, off, off + ib});
    return st ? NB_OK : flush(ctx, &local);
}

nb_status take_status(nb_ctx *ctx, int word)
{
    if (word == 0) return NB_OK;
    if (word & NBK_EINDEX) return fail(ctx, NB_EINDEX, "an active index was outside [0, n)");
    if (word & NBK_ENAN) return fail(ctx, NB_ENAN, "non-finite acceleration, jerk or step");
    return fail(ctx, NB_ERANGE, "a time step fell below dt_min");
}

nb_status status_code(int word)
{
    if (word == 0) return NB_OK;
    if (word & NBK_EINDEX) return NB_EINDEX;
    if (word & NBK_ENAN) return NB_ENAN;
    return NB_ERANGE;
}

Item base_item(nb_ctx *ctx, const nb_system &s)
{
    Item it;
    memset(&it, 0, sizeof it);
    it.s = s;
    it.status = &ctx->small->status;
    it.b = 1;
    return it;
}

// ---- force -------------------------------------------------------------------

struct Plan {
    int il, s, b;
};

// Launch plan.  A wave64 lane holds IL i-bodies; S lanes share them; the j-range
// is split into B chunks (the paper's Bfactor).  The plan
//  - uses S > 1 only as far as needed to fill a workgroup's lanes when the
//    active block is small (S = 1 keeps the LDS reads broadcasts);
//  - splits j into B chunks while the grid has fewer than about 2^21 lanes --
//    eight times the lanes the force kernels keep resident on 256 CUs, so the
//    last round of workgroups is a small part of the run -- keeping at least
//    1024 j-bodies per chunk, so the FP64 partial sums (48 B per body and
//    chunk) stay a small part of the pair work;
//  - then raises S while the grid has fewer than about 2^20 lanes and every
//    lane keeps at least 32 j-bodies (S > 1 turns LDS broadcasts into per-lane
//    reads, so it is used less eagerly than the j-split).
// The two floors were chosen on measured times over N = 2048 ... 2^20 and active
// blocks of 16 ... N: against floors of 2048 and 128 they cut small blocks of
// systems up to N = 2^18 by 10-25% and cost nowhere more than about 1%.
// Large mixed-precision blocks hold two i-bodies per lane (half the LDS reads
// per interaction).  Pure function of (nj, m, precision, lane target): a
// system's results never depend on what else runs.  The default target lets
// one system fill the GPU; a batch of many systems fills it together and may
// give each a smaller target (fewer, longer lanes).
Plan make_plan(int64_t nj, int32_t m, int precision, int64_t lanes = 0)
{
    const int64_t target_lanes = lanes > 0 ? lanes : NB_PLAN_LANES;
    const int64_t min_j_lane = 32, min_j_chunk = 1024;
    Plan p{(precision != NB_FP64 && m >= (1 << 16)) ? 2 : 1, 1, 1};
    if (m <= 0 || nj <= 0) return p;
    const int64_t groups = (m + p.il - 1) / p.il;   // lane groups holding distinct i-bodies
    while (p.s < 64 && groups * p.s < nbk::WG && nj / (p.s * 4) >= min_j_lane)
        p.s *= 4;
    int64_t b = 1;
    while (groups * p.s * b < target_lanes && nj / (b * 2) >= min_j_chunk &&
           nj / (p.s * b * 2) >= min_j_lane && b < 1024)
        b *= 2;
    p.b = (int)b;
    while (p.s < 64 && groups * p.s * b < target_lanes / 2 && nj / (p.s * 4 * b) >= min_j_lane)
        p.s *= 4;
    return p;
}

bool valid_plan(const Plan &p)
{
    return (p.il == 1 || p.il == 2 || p.il == 4) &&
           (p.s == 1 || p.s == 4 || p.s == 16 || p.s == 64) && p.b >= 1 && p.b <= 65535;
}

struct ForceJob {
    Item it;
    Plan plan;
};

nb_status ensure_side_streams(nb_ctx *ctx)
{
    if (ctx->side_ready) return NB_OK;
    NB_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
    for (int q = 0; q < nb_ctx::NSIDE; ++q) {
        NB_HIP(ctx, hipStreamCreateWithFlags(&ctx->side[q], hipStreamNonBlocking));
        NB_HIP(ctx, hipEventCreateWithFlags(&ctx->join[q], hipEventDisableTiming));
    }
    ctx->side_ready = true;
    return NB_OK;
}

// The force launches of a set of jobs: one per plan shape, then the partial
// reduction.  prepare_force fixes each job's chunks and partials and stages the
// tables; launch_force enqueues them once the tables are uploaded.
struct ForceLaunch {
    int il, s;
    bool h6;
    Table t;
    double work;   // pair interactions of the launch
};
struct ForcePlan {
    std::vector<ForceLaunch> launches;   // reserved up front: staged Tables stay in place
    Table red{};
};

// The j-chunks of an item under its plan: ceil(nj / B) bodies rounded up to the
// kernel's work granule -- the j-bodies a lane group passes over between two
// FP32 run folds (S x fold, at most one LDS tile) in the mixed and double-single
// kernels, the whole tile in the FP64 ones -- then as many chunks as that takes
// (at most B; the last one shorter).  A chunk ends on a granule, so no chunk
// does work past its share, and no chunk is empty.
void set_chunks(Item &it, const Plan &plan, int prec)
{
    const int64_t nj = it.j1 - it.j0;
    const int64_t g = prec == NB_FP64 ? nbk::TILE
                                      : (int64_t)plan.s * std::min(nbk::TILE / plan.s, NBK_FOLD);
    int64_t chunk = (nj + plan.b - 1) / plan.b;
    chunk = std::max<int64_t>(g, (chunk + g - 1) / g * g);
    it.chunk = chunk;
    it.b = nj > 0 ? (int)((nj + chunk - 1) / chunk) : 1;
}

// FP64 partial sums an item with more than one j-chunk writes (0 otherwise).
size_t part_doubles(const Item &it)
{
    return it.b > 1 ? nbk::force_outputs(it) * (size_t)it.m * (size_t)it.b : 0;
}

// Lanes per output value of the partial reduction: about 16 chunks per lane, 1 to 64.
void set_red_lanes(Item &it)
{
    int lanes = 1;
    while (lanes < 64 && lanes * 16 <= it.b) lanes *= 2;
    it.red_lanes = lanes;
}

// Workgroups of an item's force launch and of its partial reduction.
int64_t force_blocks(const Item &it, const Plan &plan)
{
    const int iwg = (nbk::WG / plan.s) * plan.il;
    return (int64_t)((it.m + iwg - 1) / iwg) * it.b;
}
int64_t reduce_blocks(const Item &it)
{
    const int64_t per = nbk::WG / it.red_lanes;
    return (nbk::force_outputs(it) * (int64_t)it.m + per - 1) / per;
}

nb_status prepare_force(nb_ctx *ctx, std::vector<ForceJob> &jobs, int prec, ForcePlan *fp,
                        Staging *st)
{
    size_t total = 0;
    for (ForceJob &j : jobs) {
        set_chunks(j.it, j.plan, prec);
        total += part_doubles(j.it);
    }
    if (total) {
        size_t have = ctx->scratch_bytes;
        NB_TRY(grow(ctx, &ctx->scratch, &have, total * sizeof(double), "force partials"));
        ctx->scratch_bytes = have;
    }
    size_t off = 0;
    for (ForceJob &j : jobs) {
        if (j.it.b > 1) {
            j.it.part = (double *)ctx->scratch + off;
            off += part_doubles(j.it);
            set_red_lanes(j.it);
        }
    }
    std::map<std::tuple<int, int, bool>, std::vector<size_t>> shapes;
    for (size_t k = 0; k < jobs.size(); ++k)
        if (jobs[k].it.m > 0)
            shapes[{jobs[k].plan.il, jobs[k].plan.s, jobs[k].it.snap != nullptr}].push_back(k);
    fp->launches.clear();
    fp->launches.reserve(shapes.size());
    for (auto &kv : shapes) {
        const int il = std::get<0>(kv.first), s = std::get<1>(kv.first);
        std::vector<Item> items;
        std::vector<int64_t> blocks;
        double work = 0.0;
        for (size_t k : kv.second) {
            items.push_back(jobs[k].it);
            blocks.push_back(force_blocks(jobs[k].it, jobs[k].plan));
            work += (double)jobs[k].it.m * (double)(jobs[k].it.j1 - jobs[k].it.j0);
        }
        fp->launches.push_back(ForceLaunch{il, s, std::get<2>(kv.first), Table{}, work});
        NB_TRY(make_table(ctx, items, blocks, &fp->launches.back().t, st));
    }
    std::vector<Item> red;
    std::vector<int64_t> rblocks;
    for (ForceJob &j : jobs) {
        if (j.it.b > 1 && j.it.m > 0) {
            red.push_back(j.it);
            rblocks.push_back(reduce_blocks(j.it));
        }
    }
    return make_table(ctx, red, rblocks, &fp->red, st);
}

// One launch per plan shape.  Several shapes (ragged batches) run side by side:
// the one with the most pair interactions on the context's stream, the others on
// side streams forked after the table uploads and joined back before the partial
// reduction (the longest launch on the joining stream: the join then seldom
// waits).  Every item writes only its own outputs and partials, so the results do
// not depend on how the launches overlap.
nb_status launch_force(nb_ctx *ctx, const ForcePlan &fp, int prec)
{
    const int nl = (int)fp.launches.size();
    int heavy = 0;
    for (int k = 1; k < nl; ++k)
        if (fp.launches[k].work > fp.launches[heavy].work) heavy = k;
    auto launch = [&](const ForceLaunch &l, hipStream_t st) {
        return l.h6 ? nbk::launch_force6(prec, l.il, l.s, l.t, st)
                    : nbk::launch_force(prec, l.il, l.s, l.t, st);
    };
    if (nl > 1) {
        NB_TRY(ensure_side_streams(ctx));
        NB_HIP(ctx, hipEventRecord(ctx->fork, ctx->stream));
    }
    // the largest launch first: it does not wait behind the side streams' set-up
    // (each cross-stream wait costs the host several microseconds)
    hipError_t e = nl > 0 ? launch(fp.launches[heavy], ctx->stream) : hipSuccess;
    if (nl > 1)
        for (int q = 0; q < std::min(nl - 1, nb_ctx::NSIDE); ++q)
            NB_HIP(ctx, hipStreamWaitEvent(ctx->side[q], ctx->fork, 0));
    for (int k = 0, q = 0; k < nl && e == hipSuccess; ++k)
        if (k != heavy) e = launch(fp.launches[k], ctx->side[q++ % nb_ctx::NSIDE]);
    // Joined even after a failed launch: the staging ring's reuse waits on
    // `stream` alone, so every side stream's work must sit behind it.
    for (int q = 0; q < std::min(nl - 1, nb_ctx::NSIDE); ++q) {
        NB_HIP(ctx, hipEventRecord(ctx->join[q], ctx->side[q]));
        NB_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->join[q], 0));
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "force kernel launch");
    e = nbk::launch_reduce(fp.red, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "partial reduction launch");
}

// Force for a set of jobs; every job's item already has its system, i_idx, m,
// j-range, eps2, acc/jerk and status set.
nb_status run_force(nb_ctx *ctx, std::vector<ForceJob> &jobs, int prec)
{
    Staging st;
    ForcePlan fp;
    NB_TRY(prepare_force(ctx, jobs, prec, &fp, &st));
    NB_TRY(flush(ctx, &st));
    return launch_force(ctx, fp, prec);
}

nb_status check_force_args(nb_ctx *ctx, const nb_system *sys, int32_t m, int64_t j0, int64_t j1,
                           double eps, int prec, const double *acc, const double *jerk)
{
    NB_TRY(check_system(ctx, sys, true));
    if (!(eps > 0.0) || !isfinite(eps)) return fail(ctx, NB_EINVAL, "eps must be > 0 and finite");
    if (prec != NB_FP64 && prec != NB_MIXED && prec != NB_DS)
        return fail(ctx, NB_EINVAL, "unknown precision");
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    if (j0 < 0 || j1 > sys->n || j0 > j1) return fail(ctx, NB_EINVAL, "bad j-range");
    if (m > 0 && (!acc || !jerk)) return fail(ctx, NB_EINVAL, "acc/jerk is NULL");
    if (m > 0 && prec != NB_FP64 && !sys->vxp32)
        return fail(ctx, NB_EINVAL, "mixed and DS precision need the FP32 copies");
    return NB_OK;
}

nb_status force_one(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                    int64_t j0, int64_t j1, double eps, nb_precision prec, Plan plan,
                    double *acc, double *jerk)
{
    NB_TRY(check_force_args(ctx, sys, m, j0, j1, eps, prec, acc, jerk));
    if (!valid_plan(plan)) return fail(ctx, NB_EINVAL, "invalid plan");
    if (m == 0) return NB_OK;
    ForceJob job;
    job.it = base_item(ctx, *sys);
    job.it.i_idx = i_idx;
    job.it.m = m;
    job.it.j0 = j0;
    job.it.j1 = j1;
    job.it.eps2 = eps * eps;
    job.it.acc = acc;
    job.it.jerk = jerk;
    job.plan = plan;
    std::vector<ForceJob> jobs{job};
    return run_force(ctx, jobs, prec);
}

nb_status force6_one(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                     const int32_t *i_idx, int32_t m, int64_t j0, int64_t j1, double eps,
                     nb_precision prec, Plan plan, double *acc, double *jerk, double *snap)
{
    NB_TRY(check_force_args(ctx, sys, m, j0, j1, eps, prec, acc, jerk));
    NB_TRY(check_h6(ctx, sys, h6));
    if (m > 0 && !snap) return fail(ctx, NB_EINVAL, "snap is NULL");
    if (m > 0 && prec != NB_FP64 && !h6->axp32)
        return fail(ctx, NB_EINVAL, "mixed and DS precision need the FP32 accelerations");
    if (!valid_plan(plan)) return fail(ctx, NB_EINVAL, "invalid plan");
    if (m == 0) return NB_OK;
    ForceJob job;
    job.it = base_item(ctx, *sys);
    job.it.h6 = *h6;
    job.it.i_idx = i_idx;
    job.it.m = m;
    job.it.j0 = j0;
    job.it.j1 = j1;
    job.it.eps2 = eps * eps;
    job.it.acc = acc;
    job.it.jerk = jerk;
    job.it.snap = snap;
    job.plan = plan;
    std::vector<ForceJob> jobs{job};
    return run_force(ctx, jobs, prec);
}

// ---- selection -------------------------------------------------------------------

void sel_shape(int64_t n, int32_t *blocks_out, int64_t *slice_out)
{
    int64_t blocks = (n + 4095) / 4096;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    int64_t slice = (n + blocks - 1) / blocks;
    slice = (slice + nbk::WG - 1) / nbk::WG * nbk::WG;
    blocks = (n + slice - 1) / slice;
    if (blocks < 1) blocks = 1;
    *blocks_out = (int32_t)blocks;
    *slice_out = slice;
}

// Device selection for `items` (each with s, i_idx and status set; every item
// has n >= 1); fills res (one SelResult per item, which the status kernel writes
// into the mapped pinned buffer).  Waits for the stream.
// predict (4 or 6, 0 for none): after the status kernel, every item is also
// predicted (by that order's predictor; 6 needs the items' h6) to its t_next
// unless that is past the item's t_next field (its horizon); the host waits only
// for the status kernel, so the prediction runs while it reads the results and
// prepares the next launches.
nb_status run_select(nb_ctx *ctx, std::vector<Item> &items, std::vector<SelResult> &res,
                     int predict = 0)
{
    res.assign(items.size(), SelResult{INFINITY, 0, 0});
    if (items.empty()) return NB_OK;
    int64_t total = 0;
    std::vector<int64_t> blocks, pblocks;
    for (Item &it : items) {
        sel_shape(it.s.n, &it.sel_blocks, &it.sel_slice);
        it.sel_off = total;
        total += it.sel_blocks;
        blocks.push_back(it.sel_blocks);
        pblocks.push_back((it.s.n + nbk::WG - 1) / nbk::WG);
    }
    size_t have = ctx->selbuf_bytes;
    NB_TRY(grow(ctx, &ctx->selbuf, &have, (size_t)total * (sizeof(double) + sizeof(int32_t)),
                "selection temporaries"));
    ctx->selbuf_bytes = have;
    NB_TRY(ensure_res(ctx, items.size() * sizeof(SelResult)));
    double *blockval = (double *)ctx->selbuf;
    int32_t *blockcnt = (int32_t *)(blockval + total);
    SelResult *dres = (SelResult *)ctx->res;
    Staging st;
    Table t, tp;
    NB_TRY(make_table(ctx, items, blocks, &t, &st));
    if (predict) NB_TRY(make_table(ctx, items, pblocks, &tp, &st));
    NB_TRY(flush(ctx, &st));
    if (t.n != (int)items.size()) return fail(ctx, NB_EINVAL, "selection of an empty system");
    hipError_t e = nbk::launch_select(t, blockval, blockcnt, dres, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "selection launch");
    const unsigned seq = ++ctx->sel_seq ? ctx->sel_seq : ++ctx->sel_seq;   // never 0
    e = nbk::launch_collect_status(t.items, t.n, dres, (SelResult *)ctx->res_host_dev,
                                   predict ? sel_flag_dev(ctx) : nullptr, seq, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "status collection launch");
    if (predict) {
        e = predict == 6 ? nbk::launch_predict6(tp, dres, ctx->stream)
                         : nbk::launch_predict(tp, dres, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "predict launch");
        // The results are complete once the status kernel has written the flag:
        // spinning on it reacts within about a microsecond, where an event wait
        // woke the thread tens of microseconds late (and the event's record in
        // the stream held the prediction back by about 6 us).  The spin is
        // bounded: a long wait, or a device error, falls through to a stream
        // synchronization (which also waits for the prediction).
        const unsigned *flag = sel_flag_host(ctx);
        const auto t0 = std::chrono::steady_clock::now();
        bool seen = false;
        for (int k = 0; !seen; ++k) {
            seen = __atomic_load_n(flag, __ATOMIC_ACQUIRE) == seq;
            if (!seen && (k & 1023) == 1023 &&
                std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(SEL_SPIN_US))
                break;
        }
        if (!seen) NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    } else {
        NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    }
    memcpy(res.data(), ctx->res_host, items.size() * sizeof(SelResult));
    return NB_OK;
}

// ---- batches -----------------------------------------------------------------------

nb_status check_item(nb_ctx *ctx, const nb_batch_item &b, bool need_m)
{
    NB_TRY(check_system(ctx, &b.sys, true));
    if (b.sys.n == 0) return NB_OK;
    if (!(b.eps > 0.0) || !isfinite(b.eps)) return fail(ctx, NB_EINVAL, "item eps must be > 0");
    if (!b.i_idx || !b.acc || !b.jerk) return fail(ctx, NB_EINVAL, "item buffers are NULL");
    if (need_m && !b.startup && (b.m < 0 || (int64_t)b.m > b.sys.n))
        return fail(ctx, NB_EINVAL, "item m out of range");
    if (need_m && !b.startup && !isfinite(b.t_next))
        return fail(ctx, NB_EINVAL, "item t_next must be finite");
    if (b.lanes != 0 && (b.lanes < NB_PLAN_LANES_MIN || b.lanes > NB_PLAN_LANES_MAX))
        return fail(ctx, NB_EINVAL, "item lane target out of range");
    return NB_OK;
}

Item batch_item(nb_ctx *ctx, const nb_batch_item &b)
{
    Item it = base_item(ctx, b.sys);
    if (b.status) it.status = b.status;
    it.eps2 = b.eps * b.eps;
    it.t_next = b.t_next;
    it.acc = b.acc;
    it.jerk = b.jerk;
    if (b.startup) {
        it.i_idx = nullptr;
        it.m = (int32_t)b.sys.n;
    } else {
        it.i_idx = b.i_idx;
        it.m = b.m;
    }
    it.j0 = 0;
    it.j1 = b.sys.n;
    return it;
}

// a1 for every item (see nb_select_active_batch).
// predict (4 or 6, 0 for none): non-startup items are also predicted to their
// t_next unless it is past their t_end (see run_select); 6 takes item k's
// 6th-order arrays from h6s[k].
nb_status select_items(nb_ctx *ctx, nb_batch_item *items, int32_t n_items, int predict = 0,
                       const nb_hermite6 *h6s = nullptr)
{
    std::vector<Item> dev;
    std::vector<int32_t> which;
    for (int32_t k = 0; k < n_items; ++k) {
        NB_TRY(check_item(ctx, items[k], false));
        items[k].error = NB_OK;
        if (items[k].sys.n == 0) {
            items[k].m = 0;
            items[k].t_next = INFINITY;
            continue;
        }
        if (items[k].startup) {
            items[k].m = (int32_t)items[k].sys.n;
            items[k].t_next = 0.0;
        }
        // a startup item runs the selection too (its result is ignored), so that
        // every item's status word is collected by the same launch
        Item it = base_item(ctx, items[k].sys);
        if (items[k].status) it.status = items[k].status;
        it.i_idx = items[k].i_idx;
        it.t_next = items[k].startup ? -INFINITY : items[k].t_end;   // prediction horizon
        if (h6s) it.h6 = h6s[k];
        dev.push_back(it);
        which.push_back(k);
    }
    std::vector<SelResult> res;
    NB_TRY(run_select(ctx, dev, res, predict));
    for (size_t q = 0; q < which.size(); ++q) {
        nb_batch_item &b = items[which[q]];
        if (!b.startup) {
            b.t_next = res[q].t_next;
            b.m = res[q].m;
        }
        b.error = status_code(res[q].status);
    }
    return NB_OK;
}

// a2 .. a5 for the items flagged in `run` (see the batch entry points).
// predicted: the selection already predicted the non-startup items.
nb_status advance_items(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items,
                        const std::vector<char> &run, nb_precision precision, double eta,
                        double eta_s, double dt_max, double dt_min, bool predicted = false)
{
    std::vector<Item> pred, cor, ini;
    std::vector<int64_t> pblocks, cblocks, iblocks;
    std::vector<ForceJob> jobs;
    for (int32_t k = 0; k < n_items; ++k) {
        if (!run[k] || items[k].sys.n == 0) continue;
        if (precision != NB_FP64 && !items[k].sys.vxp32)
            return fail(ctx, NB_EINVAL, "mixed and DS precision need the FP32 copies");
        const Item it = batch_item(ctx, items[k]);
        const int64_t nb = (items[k].sys.n + nbk::WG - 1) / nbk::WG;
        if (items[k].startup) {
            ini.push_back(it);
            iblocks.push_back(nb);
        } else {
            if (!predicted) {
                pred.push_back(it);
                pblocks.push_back(nb);
            }
            if (it.m > 0) {
                cor.push_back(it);
                cblocks.push_back((it.m + nbk::WG - 1) / nbk::WG);
            }
        }
        ForceJob job;
        job.it = it;
        job.plan = make_plan(items[k].sys.n, it.m, precision, items[k].lanes);
        jobs.push_back(job);
    }
    // every table of the iteration in one upload
    Staging st;
    Table tp, tc, ti;
    ForcePlan fp;
    NB_TRY(make_table(ctx, pred, pblocks, &tp, &st));
    NB_TRY(prepare_force(ctx, jobs, precision, &fp, &st));
    NB_TRY(make_table(ctx, cor, cblocks, &tc, &st));
    NB_TRY(make_table(ctx, ini, iblocks, &ti, &st));
    NB_TRY(flush(ctx, &st));
    hipError_t e = nbk::launch_predict(tp, nullptr, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "predict launch");
    NB_TRY(launch_force(ctx, fp, precision));
    e = nbk::launch_correct(tc, eta, dt_max, dt_min, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "correct launch");
    e = nbk::launch_init_steps(ti, eta_s, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps launch");
}

// The 6th-order step of the items flagged in `run` (see nb_step6_batch).  Startup
// items take the two passes of the 6th-order startup: the 4th-order force and
// startup steps, then prediction to t = 0 (which stores the accelerations as the
// predicted ones), acceleration + jerk + snap and the 6th-order startup steps.
// The other items: predict6 to t_next, force6, correct6.  The startup's first
// pass is its own group of launches, so that the force partials of the two
// passes never share a scratch allocation.
nb_status advance_items6(nb_ctx *ctx, const nb_batch_item *items, const nb_hermite6 *h6s,
                         double *const *snaps, int32_t n_items, const std::vector<char> &run,
                         nb_precision precision, double eta, double eta_s, double dt_max,
                         double dt_min, bool predicted = false)
{
    std::vector<Item> ini4, pred6, cor6, ini6;
    std::vector<int64_t> bi4, bp6, bc6, bi6;
    std::vector<ForceJob> jobs4, jobs6;
    for (int32_t k = 0; k < n_items; ++k) {
        if (!run[k] || items[k].sys.n == 0) continue;
        const int64_t n = items[k].sys.n;
        const int64_t nb = (n + nbk::WG - 1) / nbk::WG;
        Item it = batch_item(ctx, items[k]);
        it.h6 = h6s[k];
        if (items[k].startup) {
            ini4.push_back(it);
            bi4.push_back(nb);
            jobs4.push_back(ForceJob{it, make_plan(n, (int32_t)n, precision, items[k].lanes)});
            it.t_next = 0.0;
        }
        it.snap = snaps[k];
        if (items[k].startup || !predicted) {
            pred6.push_back(it);
            bp6.push_back(nb);
        }
        jobs6.push_back(ForceJob{it, make_plan(n, it.m, precision, items[k].lanes)});
        if (items[k].startup) {
            ini6.push_back(it);
            bi6.push_back(nb);
        } else if (it.m > 0) {
            cor6.push_back(it);
            bc6.push_back((it.m + nbk::WG - 1) / nbk::WG);
        }
    }
    if (!jobs4.empty()) {
        Staging st;
        Table t4;
        ForcePlan fp4;
        NB_TRY(prepare_force(ctx, jobs4, precision, &fp4, &st));
        NB_TRY(make_table(ctx, ini4, bi4, &t4, &st));
        NB_TRY(flush(ctx, &st));
        NB_TRY(launch_force(ctx, fp4, precision));
        hipError_t e = nbk::launch_init_steps(t4, eta_s, dt_max, dt_min, ctx->stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "init_steps launch");
    }
    Staging st;
    Table tp, tc, ti;
    ForcePlan fp;
    NB_TRY(make_table(ctx, pred6, bp6, &tp, &st));
    NB_TRY(prepare_force(ctx, jobs6, precision, &fp, &st));
    NB_TRY(make_table(ctx, cor6, bc6, &tc, &st));
    NB_TRY(make_table(ctx, ini6, bi6, &ti, &st));
    NB_TRY(flush(ctx, &st));
    hipError_t e = nbk::launch_predict6(tp, nullptr, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "predict6 launch");
    NB_TRY(launch_force(ctx, fp, precision));
    e = nbk::launch_correct6(tc, eta, dt_max, dt_min, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "correct6 launch");
    e = nbk::launch_init_steps6(ti, eta_s, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps6 launch");
}

nb_status check_step_params(nb_ctx *ctx, double eta, double dt_max, double dt_min)
{
    if (!(eta > 0.0) || !(dt_max > 0.0) || !(dt_min > 0.0) || dt_min > dt_max)
        return fail(ctx, NB_EINVAL, "need eta > 0 and 0 < dt_min <= dt_max");
    return NB_OK;
}

}  // namespace

// ---- allocation-free force ---------------------------------------------------------

// Static device area of nb_force_active_noalloc: its launch table (one item and
// the workgroup offsets of the force launch and of the partial reduction) and
// its j-chunk partial sums.  Every GPU the library runs on holds one copy until
// the process ends.  Host code never uses this name as an address: it uses the
// device address hipGetSymbolAddress gives for it on each device
// (locate_noalloc_area, called by nb_ctx_create with that device current).
static __device__ __align__(256) unsigned char scratch[NB_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t NOALLOC_TABLE_BYTES = 1024;   // item + 4 offsets, rounded up
static_assert(sizeof(Item) + 4 * sizeof(int64_t) <= NOALLOC_TABLE_BYTES, "table area");

std::mutex g_noalloc_mu;
std::map<int, void *> g_noalloc_area;   // device -> address of `scratch` there

nb_status locate_noalloc_area(int device, void **out)
{
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto f = g_noalloc_area.find(device);
    if (f != g_noalloc_area.end()) {
        *out = f->second;
        return NB_OK;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        return NB_EDEVICE;
    }
    g_noalloc_area[device] = p;
    *out = p;
    return NB_OK;
}

// Writes the launch table of one item into the static area: items[0] = it,
// starts[0..1] = {0, force_blocks}, starts[2..3] = {0, reduce_blocks}.  The item
// travels as a kernel argument, so nothing is staged in host memory.
__global__ void put_noalloc_table_kernel(Item it, int64_t fblocks, int64_t rblocks, Item *items,
                                         int64_t *starts)
{
    if (threadIdx.x == 0) {
        items[0] = it;
        starts[0] = 0;
        starts[1] = fblocks;
        starts[2] = 0;
        starts[3] = rblocks;
    }
}

nb_status force_noalloc(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                        int64_t j0, int64_t j1, double eps, nb_precision prec, double *acc,
                        double *jerk)
{
    NB_TRY(check_force_args(ctx, sys, m, j0, j1, eps, prec, acc, jerk));
    if (!ctx->noalloc_area)
        return fail(ctx, NB_EDEVICE, "the static scratch area was not located on device %d",
                    ctx->device);
    if (m == 0) return NB_OK;
    // The item and plan of nb_force_active, so the kernels and the results are the same.
    const Plan plan = make_plan(j1 - j0, m, prec);
    Item it = base_item(ctx, *sys);
    it.i_idx = i_idx;
    it.m = m;
    it.j0 = j0;
    it.j1 = j1;
    it.eps2 = eps * eps;
    it.acc = acc;
    it.jerk = jerk;
    set_chunks(it, plan, prec);
    char *area = (char *)ctx->noalloc_area;
    const size_t need = NOALLOC_TABLE_BYTES + part_doubles(it) * sizeof(double);
    if (need > (size_t)NB_NOALLOC_SCRATCH_BYTES)
        return fail(ctx, NB_ESCRATCH,
                    "m = %d with %d j-chunks needs %zu bytes of static scratch; it holds %lld",
                    (int)m, it.b, need, (long long)NB_NOALLOC_SCRATCH_BYTES);
    if (it.b > 1) {
        it.part = (double *)(area + NOALLOC_TABLE_BYTES);
        set_red_lanes(it);
    }
    const int64_t fb = force_blocks(it, plan), rb = it.b > 1 ? reduce_blocks(it) : 0;
    if (fb > (int64_t)INT32_MAX) return fail(ctx, NB_EINVAL, "launch too large");
    Item *items = (Item *)area;
    int64_t *starts = (int64_t *)(area + sizeof(Item));
    hipLaunchKernelGGL(put_noalloc_table_kernel, dim3(1), dim3(64), 0, ctx->stream, it, fb, rb,
                       items, starts);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(ctx, e, "table launch");
    e = nbk::launch_force(prec, plan.il, plan.s, Table{items, starts, 1, fb}, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "force kernel launch");
    if (rb > 0) {
        e = nbk::launch_reduce(Table{items, starts + 2, 1, rb}, ctx->stream);
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
    if (locate_noalloc_area(device, &ctx->noalloc_area) != NB_OK) {
        (void)hipFree(ctx->small);
        (void)hipHostFree(ctx->small_host);
        delete ctx;
        return NB_EDEVICE;
    }
    *out = ctx;
    return NB_OK;
}

nb_status nb_ctx_destroy(nb_ctx *ctx)
{
    if (!ctx) return NB_EINVAL;
    if (ctx->worker.th.joinable()) {
        {
            std::lock_guard<std::mutex> lk(ctx->worker.mu);
            ctx->worker.quit = true;
        }
        ctx->worker.cv.notify_all();
        ctx->worker.th.join();   // queued pair advances finish first
    }
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (int q = 0; q < nb_ctx::NSIDE; ++q) {
        if (ctx->side[q]) (void)hipStreamDestroy(ctx->side[q]);
        if (ctx->join[q]) (void)hipEventDestroy(ctx->join[q]);
    }
    if (ctx->fork) (void)hipEventDestroy(ctx->fork);
    if (ctx->scratch) (void)hipFree(ctx->scratch);
    if (ctx->selbuf) (void)hipFree(ctx->selbuf);
    if (ctx->res) (void)hipFree(ctx->res);
    if (ctx->res_host) (void)hipHostFree(ctx->res_host);
    if (ctx->stage_dev) (void)hipFree(ctx->stage_dev);
    if (ctx->stage_host) (void)hipHostFree(ctx->stage_host);
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
    NB_HIP(ctx, hipMemcpyAsync(ctx->small_host, ctx->small, sizeof(int), hipMemcpyDeviceToHost,
                               ctx->stream));
    NB_HIP(ctx, hipMemsetAsync(&ctx->small->status, 0, sizeof(int), ctx->stream));
    NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    return take_status(ctx, ctx->small_host->status);
}

nb_status nb_select_active(nb_ctx *ctx, const nb_system *sys, double *t_next_host,
                           int32_t *i_idx, int32_t *m_host)
{
    NB_TRY(check_system(ctx, sys, false));
    if (!t_next_host || !m_host) return fail(ctx, NB_EINVAL, "host outputs are NULL");
    if (sys->n == 0) {
        *m_host = 0;
        *t_next_host = INFINITY;
        return NB_OK;
    }
    if (!i_idx) return fail(ctx, NB_EINVAL, "i_idx is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].i_idx = i_idx;
    std::vector<SelResult> res;
    NB_TRY(run_select(ctx, items, res));
    *t_next_host = res[0].t_next;
    *m_host = res[0].m;
    return take_status(ctx, res[0].status);
}

nb_status nb_predict(nb_ctx *ctx, const nb_system *sys, double t_next)
{
    NB_TRY(check_system(ctx, sys, true));
    if (!isfinite(t_next)) return fail(ctx, NB_EINVAL, "t_next must be finite");
    if (sys->n == 0) return NB_OK;
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].t_next = t_next;
    std::vector<int64_t> blocks{(sys->n + nbk::WG - 1) / nbk::WG};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_predict(t, nullptr, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "predict launch");
}

nb_status nb_force_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                          int64_t j0, int64_t j1, double eps, nb_precision precision,
                          double *acc, double *jerk)
{
    return force_one(ctx, sys, i_idx, m, j0, j1, eps, precision, make_plan(j1 - j0, m, precision),
                     acc, jerk);
}

nb_status nb_force_active_plan(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                               int32_t m, int64_t j0, int64_t j1, double eps,
                               nb_precision precision, int32_t i_per_lane, int32_t lanes_per_i,
                               int32_t j_chunks, double *acc, double *jerk)
{
    return force_one(ctx, sys, i_idx, m, j0, j1, eps, precision,
                     Plan{i_per_lane, lanes_per_i, j_chunks}, acc, jerk);
}

nb_status nb_force_active_noalloc(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                                  int32_t m, int64_t j0, int64_t j1, double eps,
                                  nb_precision precision, double *acc, double *jerk)
{
    return force_noalloc(ctx, sys, i_idx, m, j0, j1, eps, precision, acc, jerk);
}

void nb_force_plan(int64_t nj, int32_t m, nb_precision precision, int32_t *i_per_lane,
                   int32_t *lanes_per_i, int32_t *j_chunks)
{
    Plan p = make_plan(nj, m, precision);
    if (i_per_lane) *i_per_lane = p.il;
    if (lanes_per_i) *lanes_per_i = p.s;
    if (j_chunks) *j_chunks = p.b;
}

nb_status nb_force_plan_lanes(int64_t nj, int32_t m, nb_precision precision, int64_t lanes,
                              int32_t *i_per_lane, int32_t *lanes_per_i, int32_t *j_chunks)
{
    if (lanes != 0 && (lanes < NB_PLAN_LANES_MIN || lanes > NB_PLAN_LANES_MAX)) return NB_EINVAL;
    Plan p = make_plan(nj, m, precision, lanes);
    if (i_per_lane) *i_per_lane = p.il;
    if (lanes_per_i) *lanes_per_i = p.s;
    if (j_chunks) *j_chunks = p.b;
    return NB_OK;
}

nb_status nb_init_steps(nb_ctx *ctx, const nb_system *sys, const double *acc,
                        const double *jerk, double eta_s, double dt_max, double dt_min)
{
    NB_TRY(check_system(ctx, sys, false));
    NB_TRY(check_step_params(ctx, eta_s, dt_max, dt_min));
    if (sys->n == 0) return NB_OK;
    if (!acc || !jerk) return fail(ctx, NB_EINVAL, "acc/jerk is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].acc = (double *)acc;
    items[0].jerk = (double *)jerk;
    std::vector<int64_t> blocks{(sys->n + nbk::WG - 1) / nbk::WG};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_init_steps(t, eta_s, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps launch");
}

nb_status nb_init_steps_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                               int32_t m, const double *acc, const double *jerk, double t,
                               double eta_s, double dt_max, double dt_min)
{
    NB_TRY(check_system(ctx, sys, false));
    NB_TRY(check_step_params(ctx, eta_s, dt_max, dt_min));
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    if (!(t >= 0.0) || !isfinite(t)) return fail(ctx, NB_EINVAL, "t must be finite and >= 0");
    if (fmod(t, dt_max) != 0.0) return fail(ctx, NB_EINVAL, "t must be a multiple of dt_max");
    if (m == 0) return NB_OK;
    if (!i_idx || !acc || !jerk) return fail(ctx, NB_EINVAL, "i_idx/acc/jerk is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].i_idx = i_idx;
    items[0].m = m;
    items[0].t_next = t;
    items[0].acc = (double *)acc;
    items[0].jerk = (double *)jerk;
    std::vector<int64_t> blocks{(m + nbk::WG - 1) / nbk::WG};
    Table tb;
    NB_TRY(make_table(ctx, items, blocks, &tb));
    hipError_t e = nbk::launch_init_steps(tb, eta_s, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps launch");
}

nb_status nb_correct(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                     const double *acc, const double *jerk, double t_next, double eta,
                     double dt_max, double dt_min)
{
    NB_TRY(check_system(ctx, sys, true));
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    NB_TRY(check_step_params(ctx, eta, dt_max, dt_min));
    if (!isfinite(t_next)) return fail(ctx, NB_EINVAL, "t_next must be finite");
    if (m == 0) return NB_OK;
    if (!acc || !jerk) return fail(ctx, NB_EINVAL, "acc/jerk is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].i_idx = i_idx;
    items[0].m = m;
    items[0].acc = (double *)acc;
    items[0].jerk = (double *)jerk;
    items[0].t_next = t_next;
    std::vector<int64_t> blocks{(m + nbk::WG - 1) / nbk::WG};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_correct(t, eta, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "correct launch");
}

nb_status nb_energy(nb_ctx *ctx, const nb_system *sys, double eps, double *kinetic_host,
                    double *potential_host)
{
    NB_TRY(check_system(ctx, sys, false));
    if (!(eps >= 0.0) || !isfinite(eps)) return fail(ctx, NB_EINVAL, "eps must be >= 0");
    if (!kinetic_host || !potential_host) return fail(ctx, NB_EINVAL, "host outputs are NULL");
    if (sys->n == 0) {
        *kinetic_host = 0.0;
        *potential_host = 0.0;
        return NB_OK;
    }
    size_t have = ctx->scratch_bytes;
    NB_TRY(grow(ctx, &ctx->scratch, &have, sizeof(double) * (size_t)sys->n, "energy rows"));
    ctx->scratch_bytes = have;
    hipError_t e = nbk::launch_energy(*sys, eps * eps, (double *)ctx->scratch, ctx->small->energy,
                                      ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "energy launch");
    NB_HIP(ctx, hipMemcpyAsync(ctx->small_host, ctx->small, sizeof(nb_small), hipMemcpyDeviceToHost,
                               ctx->stream));
    NB_HIP(ctx, hipMemsetAsync(&ctx->small->status, 0, sizeof(int), ctx->stream));
    NB_HIP(ctx, hipStreamSynchronize(ctx->stream));
    *kinetic_host = ctx->small_host->energy[0];
    *potential_host = ctx->small_host->energy[1];
    return take_status(ctx, ctx->small_host->status);
}

nb_status nb_select_active_batch(nb_ctx *ctx, nb_batch_item *items, int32_t n_items)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    return select_items(ctx, items, n_items);
}

nb_status nb_predict_batch(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    std::vector<Item> dev;
    std::vector<int64_t> blocks;
    for (int32_t k = 0; k < n_items; ++k) {
        NB_TRY(check_item(ctx, items[k], true));
        if (items[k].startup || items[k].sys.n == 0) continue;
        dev.push_back(batch_item(ctx, items[k]));
        blocks.push_back((items[k].sys.n + nbk::WG - 1) / nbk::WG);
    }
    Table t;
    NB_TRY(make_table(ctx, dev, blocks, &t));
    hipError_t e = nbk::launch_predict(t, nullptr, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "predict launch");
}

nb_status nb_force_active_batch(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items,
                                nb_precision precision)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    if (precision != NB_FP64 && precision != NB_MIXED && precision != NB_DS)
        return fail(ctx, NB_EINVAL, "unknown precision");
    std::vector<ForceJob> jobs;
    for (int32_t k = 0; k < n_items; ++k) {
        NB_TRY(check_item(ctx, items[k], true));
        if (items[k].sys.n == 0) continue;
        if (precision != NB_FP64 && !items[k].sys.vxp32)
            return fail(ctx, NB_EINVAL, "mixed and DS precision need the FP32 copies");
        ForceJob job;
        job.it = batch_item(ctx, items[k]);
        job.plan = make_plan(items[k].sys.n, job.it.m, precision, items[k].lanes);
        jobs.push_back(job);
    }
    return run_force(ctx, jobs, precision);
}

nb_status nb_correct_batch(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items, double eta,
                           double eta_s, double dt_max, double dt_min)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    NB_TRY(check_step_params(ctx, eta, dt_max, dt_min));
    if (!(eta_s > 0.0)) return fail(ctx, NB_EINVAL, "eta_s must be > 0");
    std::vector<Item> cor, ini;
    std::vector<int64_t> cblocks, iblocks;
    for (int32_t k = 0; k < n_items; ++k) {
        NB_TRY(check_item(ctx, items[k], true));
        if (items[k].sys.n == 0) continue;
        Item it = batch_item(ctx, items[k]);
        if (items[k].startup) {
            ini.push_back(it);
            iblocks.push_back((items[k].sys.n + nbk::WG - 1) / nbk::WG);
        } else if (it.m > 0) {
            cor.push_back(it);
            cblocks.push_back((it.m + nbk::WG - 1) / nbk::WG);
        }
    }
    Table t;
    NB_TRY(make_table(ctx, cor, cblocks, &t));
    hipError_t e = nbk::launch_correct(t, eta, dt_max, dt_min, ctx->stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "correct launch");
    NB_TRY(make_table(ctx, ini, iblocks, &t));
    e = nbk::launch_init_steps(t, eta_s, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps launch");
}

nb_status nb_step_batch(nb_ctx *ctx, nb_batch_item *items, int32_t n_items,
                        nb_precision precision, double eta, double eta_s, double dt_max,
                        double dt_min)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    if (precision != NB_FP64 && precision != NB_MIXED && precision != NB_DS)
        return fail(ctx, NB_EINVAL, "unknown precision");
    NB_TRY(check_step_params(ctx, eta, dt_max, dt_min));
    if (!(eta_s > 0.0)) return fail(ctx, NB_EINVAL, "eta_s must be > 0");
    NB_TRY(select_items(ctx, items, n_items, 4));
    std::vector<char> run(n_items, 0);
    for (int32_t k = 0; k < n_items; ++k) {
        nb_batch_item &b = items[k];
        b.done = 0;
        if (b.error != NB_OK || b.sys.n == 0) continue;
        if (!b.startup && b.t_next > b.t_end) {
            b.done = 1;
            continue;
        }
        NB_TRY(check_item(ctx, b, true));
        run[k] = 1;
    }
    NB_TRY(advance_items(ctx, items, n_items, run, precision, eta, eta_s, dt_max, dt_min, true));
    for (int32_t k = 0; k < n_items; ++k)
        if (run[k]) items[k].startup = 0;
    return NB_OK;
}

// ---- 6th order ---------------------------------------------------------------------

nb_status nb_predict6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6, double t_next)
{
    NB_TRY(check_system(ctx, sys, true));
    NB_TRY(check_h6(ctx, sys, h6));
    if (!isfinite(t_next)) return fail(ctx, NB_EINVAL, "t_next must be finite");
    if (sys->n == 0) return NB_OK;
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].h6 = *h6;
    items[0].t_next = t_next;
    std::vector<int64_t> blocks{(sys->n + nbk::WG - 1) / nbk::WG};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_predict6(t, nullptr, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "predict6 launch");
}

nb_status nb_force6_active(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                           const int32_t *i_idx, int32_t m, int64_t j0, int64_t j1, double eps,
                           nb_precision precision, double *acc, double *jerk, double *snap)
{
    return force6_one(ctx, sys, h6, i_idx, m, j0, j1, eps, precision,
                      make_plan(j1 - j0, m, precision), acc, jerk, snap);
}

nb_status nb_force6_active_plan(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                                const int32_t *i_idx, int32_t m, int64_t j0, int64_t j1,
                                double eps, nb_precision precision, int32_t i_per_lane,
                                int32_t lanes_per_i, int32_t j_chunks, double *acc,
                                double *jerk, double *snap)
{
    return force6_one(ctx, sys, h6, i_idx, m, j0, j1, eps, precision,
                      Plan{i_per_lane, lanes_per_i, j_chunks}, acc, jerk, snap);
}

nb_status nb_init_steps6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                         const double *acc, const double *jerk, const double *snap,
                         double eta_s, double dt_max, double dt_min)
{
    NB_TRY(check_system(ctx, sys, false));
    NB_TRY(check_h6(ctx, sys, h6));
    NB_TRY(check_step_params(ctx, eta_s, dt_max, dt_min));
    if (sys->n == 0) return NB_OK;
    if (!acc || !jerk || !snap) return fail(ctx, NB_EINVAL, "acc/jerk/snap is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].h6 = *h6;
    items[0].acc = (double *)acc;
    items[0].jerk = (double *)jerk;
    items[0].snap = (double *)snap;
    std::vector<int64_t> blocks{(sys->n + nbk::WG - 1) / nbk::WG};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_init_steps6(t, eta_s, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "init_steps6 launch");
}

nb_status nb_correct6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                      const int32_t *i_idx, int32_t m, const double *acc, const double *jerk,
                      const double *snap, double t_next, double eta, double dt_max,
                      double dt_min)
{
    NB_TRY(check_system(ctx, sys, false));
    NB_TRY(check_h6(ctx, sys, h6));
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    NB_TRY(check_step_params(ctx, eta, dt_max, dt_min));
    if (!isfinite(t_next)) return fail(ctx, NB_EINVAL, "t_next must be finite");
    if (m == 0) return NB_OK;
    if (!acc || !jerk || !snap) return fail(ctx, NB_EINVAL, "acc/jerk/snap is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].h6 = *h6;
    items[0].i_idx = i_idx;
    items[0].m = m;
    items[0].acc = (double *)acc;
    items[0].jerk = (double *)jerk;
    items[0].snap = (double *)snap;
    items[0].t_next = t_next;
    std::vector<int64_t> blocks{(m + nbk::WG - 1) / nbk::WG};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_correct6(t, eta, dt_max, dt_min, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "correct6 launch");
}

// ---- tight pairs -------------------------------------------------------------------

nb_status nb_step6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6, int32_t *i_idx,
                   double *acc, double *jerk, double *snap, double eps, nb_precision precision,
                   double eta, double dt_max, double dt_min, double t_end, double *t_next_host,
                   int32_t *m_host, int32_t *done_host)
{
    if (!ctx) return NB_EINVAL;
    if (!done_host) return fail(ctx, NB_EINVAL, "done is NULL");
    *done_host = 0;
    NB_TRY(check_system(ctx, sys, true));
    NB_TRY(check_h6(ctx, sys, h6));
    NB_TRY(check_step_params(ctx, eta, dt_max, dt_min));
    if (!t_next_host || !m_host) return fail(ctx, NB_EINVAL, "host outputs are NULL");
    if (sys->n == 0) {
        *t_next_host = INFINITY;
        *m_host = 0;
        *done_host = 1;
        return NB_OK;
    }
    if (!i_idx) return fail(ctx, NB_EINVAL, "i_idx is NULL");
    // the selection, with the 6th-order prediction enqueued behind its results
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].i_idx = i_idx;
    items[0].h6 = *h6;
    items[0].t_next = t_end;
    std::vector<SelResult> res;
    NB_TRY(run_select(ctx, items, res, 6));
    *t_next_host = res[0].t_next;
    *m_host = res[0].m;
    NB_TRY(take_status(ctx, res[0].status));
    if (!(*t_next_host <= t_end)) {
        *done_host = 1;
        return NB_OK;
    }
    NB_TRY(nb_force6_active(ctx, sys, h6, i_idx, *m_host, 0, sys->n, eps, precision, acc, jerk,
                            snap));
    return nb_correct6(ctx, sys, h6, i_idx, *m_host, acc, jerk, snap, *t_next_host, eta, dt_max,
                       dt_min);
}

nb_status nb_step6_batch(nb_ctx *ctx, nb_batch_item *items, const nb_hermite6 *h6s,
                         double *const *snaps, int32_t n_items, nb_precision precision,
                         double eta, double eta_s, double dt_max, double dt_min)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && (!items || !h6s || !snaps)))
        return fail(ctx, NB_EINVAL, "bad item arrays");
    if (precision != NB_FP64 && precision != NB_MIXED && precision != NB_DS)
        return fail(ctx, NB_EINVAL, "unknown precision");
    NB_TRY(check_step_params(ctx, eta, dt_max, dt_min));
    if (!(eta_s > 0.0)) return fail(ctx, NB_EINVAL, "eta_s must be > 0");
    for (int32_t k = 0; k < n_items; ++k) {
        if (items[k].sys.n == 0) continue;
        NB_TRY(check_h6(ctx, &items[k].sys, &h6s[k]));
        if (!snaps[k]) return fail(ctx, NB_EINVAL, "an item's snap array is NULL");
        if (precision != NB_FP64 && !h6s[k].axp32)
            return fail(ctx, NB_EINVAL, "mixed and DS precision need the FP32 accelerations");
    }
    NB_TRY(select_items(ctx, items, n_items, 6, h6s));
    std::vector<char> run(n_items, 0);
    for (int32_t k = 0; k < n_items; ++k) {
        nb_batch_item &b = items[k];
        b.done = 0;
        if (b.error != NB_OK || b.sys.n == 0) continue;
        if (!b.startup && b.t_next > b.t_end) {
            b.done = 1;
            continue;
        }
        NB_TRY(check_item(ctx, b, true));
        if (precision != NB_FP64 && !b.sys.vxp32)
            return fail(ctx, NB_EINVAL, "mixed and DS precision need the FP32 copies");
        run[k] = 1;
    }
    NB_TRY(advance_items6(ctx, items, h6s, snaps, n_items, run, precision, eta, eta_s, dt_max,
                          dt_min, true));
    for (int32_t k = 0; k < n_items; ++k)
        if (run[k]) items[k].startup = 0;
    return NB_OK;
}

nb_status nb_tidal_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                          int64_t j0, int64_t j1, double eps, double *tensor)
{
    NB_TRY(check_system(ctx, sys, true));
    if (!(eps >= 0.0) || !isfinite(eps)) return fail(ctx, NB_EINVAL, "eps must be >= 0 and finite");
    if (m < 0 || (int64_t)m > sys->n) return fail(ctx, NB_EINVAL, "m out of range");
    if (j0 < 0 || j1 > sys->n || j0 > j1) return fail(ctx, NB_EINVAL, "bad j-range");
    if (m == 0) return NB_OK;
    if (!tensor) return fail(ctx, NB_EINVAL, "tensor is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].i_idx = i_idx;
    items[0].m = m;
    items[0].j0 = j0;
    items[0].j1 = j1;
    items[0].eps2 = eps * eps;
    items[0].tensor = tensor;
    items[0].row0 = -1;
    items[0].nrows = m;
    std::vector<int64_t> blocks{m};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_tidal(t, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "tidal launch");
}

nb_status nb_tidal_active_batch(nb_ctx *ctx, const nb_tidal_item *items, int32_t n_items)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    std::vector<Item> dev;
    std::vector<int64_t> blocks;
    for (int32_t k = 0; k < n_items; ++k) {
        const nb_tidal_item &b = items[k];
        NB_TRY(check_system(ctx, &b.sys, true));
        if (!(b.eps >= 0.0) || !isfinite(b.eps))
            return fail(ctx, NB_EINVAL, "item %d: eps must be >= 0 and finite", (int)k);
        if (b.m < 0 || (int64_t)b.m > b.sys.n)
            return fail(ctx, NB_EINVAL, "item %d: m out of range", (int)k);
        if (b.m == 0) continue;
        if (!b.i_idx || !b.tensor)
            return fail(ctx, NB_EINVAL, "item %d: i_idx or tensor is NULL", (int)k);
        if (b.row0 >= 0 && (b.row0 > b.sys.n || b.nrows < 0 || b.row0 + b.nrows > b.sys.n))
            return fail(ctx, NB_EINVAL, "item %d: bad row0 / nrows", (int)k);
        Item it = base_item(ctx, b.sys);
        if (b.status) it.status = b.status;
        it.i_idx = b.i_idx;
        it.m = b.m;
        it.j0 = 0;
        it.j1 = b.sys.n;
        it.eps2 = b.eps * b.eps;
        it.tensor = b.tensor;
        it.t_out = b.t_out;
        it.row0 = b.row0 >= 0 ? b.row0 : -1;
        it.nrows = b.row0 >= 0 ? b.nrows : b.m;
        dev.push_back(it);
        blocks.push_back(b.m);
    }
    Table t;
    NB_TRY(make_table(ctx, dev, blocks, &t));
    hipError_t e = nbk::launch_tidal(t, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "tidal launch");
}

nb_status nb_tidal_points(nb_ctx *ctx, const nb_system *sys, int32_t k, const double *pts,
                          const int32_t *excl, double eps, double *tensor)
{
    NB_TRY(check_system(ctx, sys, true));
    if (!(eps >= 0.0) || !isfinite(eps)) return fail(ctx, NB_EINVAL, "eps must be >= 0 and finite");
    if (k < 0) return fail(ctx, NB_EINVAL, "k < 0");
    if (k == 0) return NB_OK;
    if (!pts || !tensor) return fail(ctx, NB_EINVAL, "pts or tensor is NULL");
    std::vector<Item> items{base_item(ctx, *sys)};
    items[0].m = k;
    items[0].j0 = 0;
    items[0].j1 = sys->n;
    items[0].eps2 = eps * eps;
    items[0].tensor = tensor;
    items[0].row0 = -1;
    items[0].nrows = k;
    items[0].pts = pts;
    items[0].excl = excl;
    std::vector<int64_t> blocks{k};
    Table t;
    NB_TRY(make_table(ctx, items, blocks, &t));
    hipError_t e = nbk::launch_tidal(t, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "tidal launch");
}

nb_status nb_nearest_active_batch(nb_ctx *ctx, const nb_nearest_item *items, int32_t n_items)
{
    if (!ctx) return NB_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, NB_EINVAL, "bad item array");
    std::vector<Item> dev;
    std::vector<int64_t> blocks;
    for (int32_t k = 0; k < n_items; ++k) {
        const nb_nearest_item &b = items[k];
        NB_TRY(check_system(ctx, &b.sys, true));
        if (b.m < 0 || (int64_t)b.m > b.sys.n)
            return fail(ctx, NB_EINVAL, "item %d: m out of range", (int)k);
        if (b.dt_cap != b.dt_cap)
            return fail(ctx, NB_EINVAL, "item %d: dt_cap is NaN", (int)k);
        if (b.m == 0) continue;
        if (!b.i_idx || !b.nn || !b.r2)
            return fail(ctx, NB_EINVAL, "item %d: i_idx, nn or r2 is NULL", (int)k);
        Item it = base_item(ctx, b.sys);
        if (b.status) it.status = b.status;
        it.i_idx = b.i_idx;
        it.m = b.m;
        it.nn = b.nn;
        it.r2 = b.r2;
        it.row_end = b.row_end;
        it.dt_cap = b.dt_cap;
        dev.push_back(it);
        blocks.push_back(b.m);
    }
    Table t;
    NB_TRY(make_table(ctx, dev, blocks, &t));
    hipError_t e = nbk::launch_nearest(t, ctx->stream);
    return e == hipSuccess ? NB_OK : hip_fail(ctx, e, "nearest launch");
}

nb_status nb_groups_advance_async(nb_ctx *ctx, int32_t n, const int32_t *idx, const double *M,
                                  double *r, double *v, const double *H, const double *T0,
                                  const double *T1, int32_t per_period, int64_t max_sub,
                                  int32_t *status)
{
    if (!ctx) return NB_EINVAL;
    return nb_groups_run(ctx, n, idx, M, r, v, H, T0, T1, per_period, max_sub, status, true);
}

nb_status nb_groups_wait(nb_ctx *ctx)
{
    if (!ctx) return NB_EINVAL;
    nb_ctx::Worker &w = ctx->worker;
    std::unique_lock<std::mutex> lk(w.mu);
    w.cv.wait(lk, [&w]() { return w.queue.empty() && !w.running; });
    const nb_status r = (nb_status)w.result;
    w.result = NB_OK;
    lk.unlock();
    if (r != NB_OK) fail(ctx, r, "a pair handed to the two-body drift is not bound");
    return r;
}

}  // extern "C"
