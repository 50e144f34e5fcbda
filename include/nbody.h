/*
 * nbody.h -- C ABI of libnbody.so, the MI355X (gfx950) hot path of a direct
 * N-body code with 4th- and 6th-order Hermite integrators and power-of-two
 * block time steps (Spera 2014, "Using GPUs to solve the classical N-body
 * problem", GPUHEP2014: Eq. 1-2 and Sec. 2 items 1-5).
 *
 * General conventions
 *  - Units: G = 1.  Every floating-point state array is FP64.
 *  - Layout: structure of arrays.  A body's x, y, z (and so on) live in separate
 *    arrays of length n; "3*m SoA" below means three consecutive arrays of m
 *    values each (x-components, then y, then z).
 *  - Ownership: every array pointer is DEVICE memory owned by the caller (the
 *    Python layer passes torch tensors).  The library owns only the context's
 *    scratch memory.  Host pointers are named *_host.
 *  - Streams: every call is enqueued on the context's HIP stream and returns
 *    without waiting, except nb_select_active, nb_energy and nb_sync, which
 *    wait for the stream.
 *  - Errors: a call returns NB_OK or a negative nb_status.  Argument errors are
 *    detected on the host before anything is enqueued.  Errors that kernels
 *    find (a non-finite acceleration, jerk or step; a step below dt_min; an
 *    index out of range) are latched in a device status word and reported by
 *    the next waiting call (nb_select_active, nb_energy, nb_sync), which also
 *    clears the word.  nb_last_error() gives a message for the last failure.
 *  - Indices are int32 (n < 2^31); sizes are int64.
 *  - A context is bound to one device and one stream and is not thread-safe.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nb_ctx nb_ctx;

typedef enum {
    NB_OK = 0,
    NB_EINVAL = -1,   /* bad argument (null pointer, eps <= 0, bad range ...)  */
    NB_ENOMEM = -2,   /* device or pinned allocation failed                    */
    NB_EDEVICE = -3,  /* a HIP runtime call failed                             */
    NB_ERANGE = -4,   /* a new time step fell below dt_min                      */
    NB_ENAN = -5,     /* non-finite acceleration, jerk or time step            */
    NB_EINDEX = -6,   /* an active index was outside [0, n)                     */
    NB_EUNBOUND = -7, /* a pair handed to the two-body drift is not bound        */
    NB_ESCRATCH = -8  /* nb_force_active_noalloc: the call needs more scratch than
                         the static area holds                                  */
} nb_status;

typedef enum {
    NB_FP64 = 0,      /* all pair arithmetic in FP64                            */
    NB_MIXED = 1,     /* FP64 pair differences, FP32 pair arithmetic, FP64 sums */
    NB_DS = 2         /* double-single pair differences (each FP64 position as
                         FP32 hi + lo, difference (hi_j - hi_i) + (lo_j - lo_i)),
                         then as NB_MIXED: the DS alternative of Sec. 2 item 4 */
} nb_precision;

/* One system of n bodies.  Every pointer is a device array of length n.
 *  state at each body's own time t_i:  x..z, vx..vz, ax..az (acceleration),
 *      jx..jz (jerk), m (mass), t (time), dt (power-of-two step);
 *  predicted j-set at the current block time:  xp..zp, vxp..vzp;
 *  FP32 copies used by NB_MIXED:  vxp32..vzp32, m32 (may be NULL when only
 *      NB_FP64 is used).                                                      */
typedef struct {
    int64_t n;
    double *x, *y, *z;
    double *vx, *vy, *vz;
    double *ax, *ay, *az;
    double *jx, *jy, *jz;
    double *m, *t, *dt;
    double *xp, *yp, *zp;
    double *vxp, *vyp, *vzp;
    float *vxp32, *vyp32, *vzp32, *m32;
} nb_system;

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL means the null stream).  The context allocates its scratch memory here
 * (force partial sums, selection temporaries, the status word, pinned host
 * words); a later call that needs more scratch grows it once, after waiting
 * for the stream.  Returns NB_OK, NB_EINVAL or NB_ENOMEM. */
nb_status nb_ctx_create(nb_ctx **ctx, int device, void *hip_stream);
nb_status nb_ctx_destroy(nb_ctx *ctx);
/* Message for the last failing call on this context (never NULL). */
const char *nb_last_error(const nb_ctx *ctx);
/* Wait for the context's stream; return and clear any latched kernel error. */
nb_status nb_sync(nb_ctx *ctx);

/* Active block (Sec. 2 item 2: bodies share power-of-two steps and only the
 * block due next is advanced).  Computes t_next = min_i (t_i + dt_i) and writes
 * to i_idx (device, capacity n) every i with t_i + dt_i == t_next, in ascending
 * order.  The comparison is exact: all times are dyadic.  Waits for the stream
 * and returns t_next and the block size m on the host.  n == 0 gives m = 0. */
nb_status nb_select_active(nb_ctx *ctx, const nb_system *sys, double *t_next_host,
                           int32_t *i_idx, int32_t *m_host);

/* Predictor (Sec. 2 item 2: bodies outside the active block are only advanced
 * by Taylor expansion).  For every body, with d = t_next - t_i:
 *   xp = x + v d + a d^2/2 + j d^3/6,   vp = v + a d + j d^2/2   (FP64),
 * and, when the FP32 pointers are non-NULL, vp32 = (float)vp and m32 = (float)m. */
nb_status nb_predict(nb_ctx *ctx, const nb_system *sys, double t_next);

/* Acceleration and jerk of the active block from the predicted j-set (Eq. 1
 * with G = 1 and the Plummer softening of Eq. 2; the jerk is its time
 * derivative).  For k < m, with i = i_idx[k] (or i = k when i_idx is NULL) and
 * every j in [j0, j1):
 *   r = xp_j - xp_i, w = vp_j - vp_i, s = |r|^2 + eps^2,
 *   acc_k  += m_j r s^(-3/2),
 *   jerk_k += m_j (w s^(-3/2) - 3 (r.w) r s^(-5/2)).
 * The pair j = i contributes exactly 0 because eps > 0 is required.
 * acc and jerk are device arrays of 3*m doubles (SoA, stride m) and are
 * overwritten.  NB_FP64 does all pair arithmetic in FP64; NB_MIXED forms r in
 * FP64, rounds it to FP32, does the rest of the pair arithmetic in FP32 (with
 * the hardware reciprocal square root) and accumulates in FP64 (the precision
 * split of Sec. 2 item 4); NB_DS forms r from double-single (FP32 hi + lo)
 * positions in FP32 and continues as NB_MIXED.  NB_MIXED and NB_DS need the
 * FP32 velocity and mass copies.  The j-range is split across workgroups when m is
 * small (Sec. 2 item 3) and the partial sums are combined in a fixed order,
 * so results are bitwise reproducible.  m == 0 is a no-op.
 * Returns NB_EINVAL for eps <= 0, j0 < 0, j1 > n, j0 > j1, m < 0 or m > n. */
nb_status nb_force_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                          int32_t m, int64_t j0, int64_t j1, double eps,
                          nb_precision precision, double *acc, double *jerk);

/* Startup (t = 0, every body active): copy acc/jerk (3*n SoA, from
 * nb_force_active with i_idx = NULL, m = n) into the state, set t = 0 and
 * dt = the largest power of two not above min(eta_s |a| / |j|, dt_max).
 * A step below dt_min latches NB_ERANGE; a non-finite value latches NB_ENAN. */
nb_status nb_init_steps(nb_ctx *ctx, const nb_system *sys, const double *acc,
                        const double *jerk, double eta_s, double dt_max, double dt_min);

/* Bodies joining a running block-step system at block time t (the two members
 * of a pair returned to the N-body system): copy acc/jerk of the m listed bodies
 * (3*m SoA, from nb_force_active on the predicted set at t) into their state,
 * set their time to t and their step by the startup rule, the largest power of
 * two not above min(eta_s |a| / |j|, dt_max).  dt_max must be a power of two
 * that divides t (for instance the step of the body they replace), so the new
 * steps keep the block times commensurate (Sec. 2 item 2).  A step below dt_min
 * latches NB_ERANGE; a non-finite value NB_ENAN; an index outside [0, n)
 * NB_EINDEX.  Returns NB_EINVAL for bad arguments or t not a multiple of dt_max. */
nb_status nb_init_steps_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                               int32_t m, const double *acc, const double *jerk, double t,
                               double eta_s, double dt_max, double dt_min);

/* Corrector and new step for the active block (Sec. 2 items 1-2; the standard
 * 4th-order Hermite form of Aarseth's book, cited there).  With h = t_next - t_i,
 * (a0, j0) the stored and (a1, j1) the new acc/jerk (3*m SoA, order of i_idx):
 *   a2 = [-6 (a0 - a1) - h (4 j0 + 2 j1)] / h^2,  a3 = [12 (a0 - a1) + 6 h (j0 + j1)] / h^3,
 *   x = xp + a2 h^4/24 + a3 h^5/120,  v = vp + a2 h^3/6 + a3 h^4/24,
 * then a = a1, j = j1, t = t_next, and the new step from Aarseth's criterion
 *   dtA = sqrt(eta (|a1||a2'| + |j1|^2) / (|j1||a3| + |a2'|^2)),  a2' = a2 + a3 h,
 * kept a power of two: halve while above dtA; if no halving was needed, double
 * once when dtA >= 2h, t_next is a multiple of 2h and 2h <= dt_max.
 * A step below dt_min latches NB_ERANGE; non-finite values latch NB_ENAN. */
nb_status nb_correct(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx, int32_t m,
                     const double *acc, const double *jerk, double t_next,
                     double eta, double dt_max, double dt_min);

/* Total energy of the current state (x, v at the bodies' own times, so call it
 * when every body is synchronised):  kinetic = sum_i m_i |v_i|^2 / 2 and
 * potential = -sum_{i<j} m_i m_j / sqrt(|x_j - x_i|^2 + eps^2), self term
 * excluded, all in FP64 with compensated final sums.  This is the conservation
 * diagnostic of Sec. 3 (Fig. 3).  Waits for the stream.  eps >= 0. */
nb_status nb_energy(nb_ctx *ctx, const nb_system *sys, double eps,
                    double *kinetic_host, double *potential_host);

/* Launch plan of nb_force_active for a j-range of nj bodies and an active
 * block of m (a pure function of (nj, m, precision), so a system's results do
 * not depend on anything else running): i-bodies per lane, lanes sharing one
 * i-body, and the number of j-chunks (the paper's Bfactor).  Out-pointers may
 * be NULL. */
void nb_force_plan(int64_t nj, int32_t m, nb_precision precision,
                   int32_t *i_per_lane, int32_t *lanes_per_i, int32_t *j_chunks);

/* The same plan for a given lane target: the plan splits the work until about
 * `lanes` lanes are busy (0 = the default, NB_PLAN_LANES, which lets one system
 * fill the GPU).  Batch items carry their own target (nb_batch_item.lanes).
 * Returns NB_EINVAL (and leaves the outputs alone) unless lanes is 0 or in
 * [NB_PLAN_LANES_MIN, NB_PLAN_LANES_MAX]. */
#define NB_PLAN_LANES ((int64_t)1 << 21)
#define NB_PLAN_LANES_MIN ((int64_t)1 << 10)
#define NB_PLAN_LANES_MAX ((int64_t)1 << 24)
nb_status nb_force_plan_lanes(int64_t nj, int32_t m, nb_precision precision, int64_t lanes,
                              int32_t *i_per_lane, int32_t *lanes_per_i, int32_t *j_chunks);

/* Same as nb_force_active but with an explicit plan (for tests and tuning);
 * i_per_lane in {1, 2, 4}, lanes_per_i in {1, 4, 16, 64}, j_chunks >= 1. */
nb_status nb_force_active_plan(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                               int32_t m, int64_t j0, int64_t j1, double eps,
                               nb_precision precision, int32_t i_per_lane,
                               int32_t lanes_per_i, int32_t j_chunks,
                               double *acc, double *jerk);

/* Allocation-free form of nb_force_active, for callers that cannot allocate
 * memory during the call: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, launch plan, kernels and
 * results (bitwise) as nb_force_active; it allocates nothing, device or host.
 * Its launch table and j-chunk partial sums live in a static device area of
 * NB_NOALLOC_SCRATCH_BYTES, one per GPU, held until the process ends and
 * located by nb_ctx_create.  A call whose partial sums (6 doubles per active
 * body and j-chunk when the plan has more than one chunk) would not fit returns
 * NB_ESCRATCH before anything is enqueued.  Every call on one GPU uses that
 * GPU's single area, which keeps the last call's contents: calls that overlap
 * on one GPU (several streams or contexts) race, so serialise them. */
#define NB_NOALLOC_SCRATCH_BYTES ((int64_t)64 << 20)
nb_status nb_force_active_noalloc(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                                  int32_t m, int64_t j0, int64_t j1, double eps,
                                  nb_precision precision, double *acc, double *jerk);

/* ---- ragged batches: many independent systems in one launch per phase -------
 * Ensemble serving advances many systems of different n together.  Each batch
 * call runs ONE launch per phase (per plan shape for the force) over all items,
 * with every workgroup working for exactly one item.  Each item is computed
 * with the same kernels, the same launch plan (a pure function of its own n, m
 * and lane target) and the same arithmetic as the single-system calls above,
 * which are themselves batches of one, so a system's results are bitwise the
 * same alone and in any mix.  The block-step parameters (eta, eta_s, dt_max, dt_min) are
 * shared by the items of a call.  An item whose status word is non-NULL gets its
 * own kernel error bits there (device int, owned by the caller); otherwise the
 * context's word is used. */
typedef struct {
    nb_system sys;       /* the system's device arrays                              */
    int32_t *i_idx;      /* device, capacity sys.n: the active list                  */
    double *acc, *jerk;  /* device, capacity 3*sys.n each (SoA with stride m)        */
    int32_t *status;     /* device word for this item's kernel errors, or NULL       */
    double eps;          /* Plummer softening, > 0                                   */
    double t_next;       /* block time: set by nb_select_active_batch                */
    double t_end;        /* nb_step_batch: the item is done once t_next > t_end       */
    int32_t m;           /* active block size: set by nb_select_active_batch         */
    int32_t startup;     /* 1: the t = 0 step (all bodies active, no selection)      */
    int32_t error;       /* host: nb_status of this item's latched errors, set by
                            nb_select_active_batch (the item's word is then cleared) */
    int32_t done;        /* host: set to 1 by nb_step_batch when t_next > t_end      */
    int64_t lanes;       /* force plan lane target (see nb_force_plan_lanes); 0 = the
                            default.  A server whose systems fill the GPU together can
                            give each fewer lanes than one system alone would take. */
} nb_batch_item;

/* a1 for every item (Sec. 2 item 2).  Startup items get m = n, t_next = 0 and no
 * device work.  Waits for the stream; fills t_next, m and error of every item. */
nb_status nb_select_active_batch(nb_ctx *ctx, nb_batch_item *items, int32_t n_items);
/* a2 for every non-startup item, each to its own t_next (Sec. 2 item 2). */
nb_status nb_predict_batch(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items);
/* a3 + a4 for every item: acc/jerk of its m active bodies (all n for startup
 * items, i = k) from its whole predicted j-set (Eq. 1-2, Sec. 2 items 3-5). */
nb_status nb_force_active_batch(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items,
                                nb_precision precision);
/* a5 for every non-startup item (Sec. 2 items 1-2); the startup step of
 * nb_init_steps for startup items. */
nb_status nb_correct_batch(nb_ctx *ctx, const nb_batch_item *items, int32_t n_items,
                           double eta, double eta_s, double dt_max, double dt_min);

/* One iteration of an ensemble loop in one call: a1 for every item (waits until
 * the selection's results have reached the host, by a bounded spin on a flag the
 * device writes after them, else a stream synchronization), then, for every item
 * without an error whose next block time is
 * not past its t_end, a2 + a3 + a4 + a5 as in the four calls above (startup
 * items: force + startup steps, after which their startup flag is cleared).
 * Here a2 is enqueued right after the selection and runs while the host reads
 * its results, with the same arithmetic as nb_predict_batch.
 * Items past t_end get done = 1 and no work; items with an error get no work.
 * Host fields t_next, m, error, done and startup are updated in place. */
nb_status nb_step_batch(nb_ctx *ctx, nb_batch_item *items, int32_t n_items,
                        nb_precision precision, double eta, double eta_s, double dt_max,
                        double dt_min);

/* ---- 6th-order Hermite ----------------------------------------------------------
 * The scheme of the paper's HiGPUs code (Sec. 2 item 1: Hermite integrators of
 * order 4, 6 and 8 need one force evaluation per step).  The pair sum adds the
 * snap (second time derivative of the acceleration), which needs the predicted
 * accelerations of the j-bodies; the predictor reaches the crackle (third
 * derivative); the corrector is the two-point Hermite quadrature exact for a
 * quartic acceleration, and the crackle at the step's end comes from the
 * degree-5 interpolant of (a, j, s) at both ends.
 * These calls take an nb_system (whose a and j are the state's acceleration and
 * jerk, and whose xp, vp, vp32, m32 are the predicted j-set as for the 4th
 * order) plus the extra arrays below, all device arrays of length n owned by
 * the caller.  Snap and crackle must hold finite values before the first
 * nb_predict6 (zeros are fine: the startup sets them).                         */
typedef struct {
    double *sx, *sy, *sz;          /* snap at t_i                                  */
    double *cx, *cy, *cz;          /* crackle at t_i                               */
    double *axp, *ayp, *azp;       /* predicted acceleration at the block time     */
    float *axp32, *ayp32, *azp32;  /* FP32 copies for NB_MIXED / NB_DS (or NULL)   */
} nb_hermite6;

/* Predictor to the crackle for every body, with d = t_next - t_i:
 *   xp = x + v d + a d^2/2 + j d^3/6 + s d^4/24 + c d^5/120,
 *   vp = v + a d + j d^2/2 + s d^3/6 + c d^4/24,
 *   ap = a + j d + s d^2/2 + c d^3/6                       (FP64),
 * and, when the FP32 pointers are non-NULL, vp32, ap32 and m32 as FP32 copies. */
nb_status nb_predict6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                      double t_next);

/* Acceleration, jerk and snap of the active block from the predicted j-set.
 * As nb_force_active, plus, with b = ap_j - ap_i, alpha = (r.w)/s and
 * beta = (|w|^2 + r.b)/s + alpha^2:
 *   jerk_k += m_j s^(-3/2) (w - 3 alpha r),
 *   snap_k += m_j s^(-3/2) (b - 6 alpha (w - 3 alpha r) - 3 beta r),
 * the second time derivative of the pair acceleration along the predicted
 * motion.  acc, jerk and snap are device arrays of 3*m doubles (SoA, stride m)
 * and are overwritten.  Precisions as nb_force_active; NB_MIXED and NB_DS need
 * the FP32 copies of sys and h6.  Bitwise reproducible; m == 0 is a no-op.
 * Returns NB_EINVAL for eps <= 0, j0 < 0, j1 > n, j0 > j1, m < 0 or m > n. */
nb_status nb_force6_active(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                           const int32_t *i_idx, int32_t m, int64_t j0, int64_t j1,
                           double eps, nb_precision precision, double *acc, double *jerk,
                           double *snap);

/* Same as nb_force6_active with an explicit plan (as nb_force_active_plan). */
nb_status nb_force6_active_plan(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                                const int32_t *i_idx, int32_t m, int64_t j0, int64_t j1,
                                double eps, nb_precision precision, int32_t i_per_lane,
                                int32_t lanes_per_i, int32_t j_chunks, double *acc,
                                double *jerk, double *snap);

/* Startup of the 6th-order scheme (t = 0, every body active): copy acc, jerk
 * and snap (3*n SoA each, from nb_force6_active over all bodies with the
 * accelerations of a first nb_force_active pass as predicted accelerations)
 * into the state, set the crackle to 0, t = 0 and dt = the largest power of
 * two not above min(eta_s (sqrt(|a||s|) + |j|) / (|s| + |j|^2/|a|), dt_max).
 * Errors latched as nb_init_steps. */
nb_status nb_init_steps6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                         const double *acc, const double *jerk, const double *snap,
                         double eta_s, double dt_max, double dt_min);

/* 6th-order corrector and new step for the active block.  With h = t_next - t_i,
 * (a0, j0, s0) stored and (a1, j1, s1) new (3*m SoA, order of i_idx):
 *   v = v + h/2 (a0 + a1) - h^2/10 (j1 - j0) + h^3/120 (s0 + s1),
 *   x = x + h/2 (v_old + v) - h^2/10 (a1 - a0) + h^3/120 (j0 + j1),
 *   crackle = -3 (20 (a0 - a1) + h^2 (s0 - 3 s1) + h (8 j0 + 12 j1)) / h^3
 * (the third derivative at t_next of the degree-5 interpolant of (a, j, s) at
 * both ends), a, j, s = a1, j1, s1, t = t_next, and the new step
 *   dtC = eta (sqrt(|a1||s1|) + |j1|) / (sqrt(|j1||crackle|) + |s1|),
 *   dtD = eta (sqrt(|a1||s1|) + |j1|) / (|s1| + |j1|^2 / |a1|),
 *   dtA = max(dtC, dtD / 8)
 * (both eta/omega on a circular orbit), kept a power of two by the rule of
 * nb_correct.  The crackle announces approaching close encounters; the floor
 * dtD/8 (computed derivatives only) keeps FP32 rounding noise in the
 * interpolated crackle, which grows as h^-3, from driving small steps to dt_min.
 * Errors latched as nb_correct. */
nb_status nb_correct6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6,
                      const int32_t *i_idx, int32_t m, const double *acc, const double *jerk,
                      const double *snap, double t_next, double eta, double dt_max,
                      double dt_min);

/* One whole 6th-order block step of one system in one call (Sec. 2 items 1-2):
 * nb_select_active (waits for the stream; t_next, m to the host pointers), then,
 * if t_next <= t_end, nb_predict6 to t_next, nb_force6_active of the m active
 * bodies from all n (eps, precision) and nb_correct6 (eta, dt_max, dt_min) —
 * the same kernels and results as those calls made one by one.  Otherwise
 * *done_host = 1 and nothing is enqueued.  i_idx (capacity n), acc, jerk, snap
 * (3n each) are device arrays; t_next_host, m_host, done_host host scalars.
 * Returns the first failing call's status (latched kernel errors included). */
nb_status nb_step6(nb_ctx *ctx, const nb_system *sys, const nb_hermite6 *h6, int32_t *i_idx,
                   double *acc, double *jerk, double *snap, double eps, nb_precision precision,
                   double eta, double dt_max, double dt_min, double t_end, double *t_next_host,
                   int32_t *m_host, int32_t *done_host);

/* nb_step_batch at 6th order (Sec. 2 item 1): one iteration of an ensemble loop
 * in one call.  h6s[k] and snaps[k] (device, 3*n doubles) are item k's 6th-order
 * arrays; its acc and jerk buffers hold the forces as in nb_step_batch.  A
 * startup item takes the whole 6th-order startup in this call (the 4th-order
 * force and startup steps, prediction to t = 0, acc + jerk + snap and
 * nb_init_steps6's steps); the others take nb_predict6, nb_force6_active and
 * nb_correct6 — the same kernels, plans and results as those calls on each
 * system alone.  Host fields, errors and done as in nb_step_batch. */
nb_status nb_step6_batch(nb_ctx *ctx, nb_batch_item *items, const nb_hermite6 *h6s,
                         double *const *snaps, int32_t n_items, nb_precision precision,
                         double eta, double eta_s, double dt_max, double dt_min);

/* ---- tight pairs (the HiGPUs-R scheme of Sec. 3) -------------------------------------
 * Tight groups are taken out of the N-body integration and advanced apart from
 * it, on CPU threads, while the GPU kernels run.  Here a group is a bound pair:
 * the block-step system carries it as one body of mass M = m1 + m2 at its
 * centre of mass, and its relative coordinate r = x2 - x1, w = v2 - v1 is
 * advanced over each step of that body by exact two-body drifts and kicks from
 * the tidal tensor of the rest of the system (linear about the centre of mass).
 * The two-body motion is unsoftened. */

/* Tidal tensor T_ab = d a_a / d x_b of the softened field of the predicted bodies
 * j in [j0, j1), j != i, at the predicted position of each listed body i
 * (i = i_idx[k], or k when i_idx is NULL):
 *   T_ab = sum_j m_j (3 r_a r_b / s^(5/2) - delta_ab / s^(3/2)),  r = xp_j - xp_i,
 * s = |r|^2 + eps^2.  FP64.  tensor: device, 9*m doubles, T_ab of body k at
 * tensor[(3a+b)*m + k].  One workgroup per listed body; bitwise reproducible.
 * Returns NB_EINVAL for eps < 0, bad ranges or m < 0; m == 0 is a no-op. */
nb_status nb_tidal_active(nb_ctx *ctx, const nb_system *sys, const int32_t *i_idx,
                          int32_t m, int64_t j0, int64_t j1, double eps, double *tensor);

/* The tidal tensor of many systems in one launch (a served ensemble whose pairs
 * are carried as centre-of-mass bodies).  Per item, as nb_tidal_active over the
 * whole j-range [0, sys.n), at the bodies i = i_idx[0 .. m).  With row0 < 0 body k
 * of the list writes row k; with row0 >= 0 body i writes row i - row0 and bodies
 * with i < row0 write nothing, so the active list of a block step gives the
 * tensors of exactly the centre-of-mass bodies (rows row0 .. row0 + nrows - 1 of
 * the system) that were in the block.  `tensor`: device, 9 rows of nrows doubles
 * (nrows = m when row0 < 0), T_ab of row q at tensor[(3a+b)*nrows + q]; `t_out`
 * (device, one double per row, or NULL) receives the body's time t_i, so the host
 * can tell which pairs were in the last block.  `status`: the item's device error
 * word (NULL: the context's).  Items with m == 0 are skipped.  Returns NB_EINVAL
 * for a bad item (nothing enqueued). */
typedef struct {
    nb_system sys;
    const int32_t *i_idx;  /* device: listed bodies                       */
    int32_t m;
    double eps;            /* >= 0                                        */
    double *tensor;        /* device, 9 * nrows                           */
    double *t_out;         /* device, nrows, or NULL                      */
    int32_t *status;       /* device word, or NULL                        */
    int64_t row0;          /* < 0: row = list position; else row = i - row0 */
    int64_t nrows;         /* rows of the outputs when row0 >= 0          */
} nb_tidal_item;
nb_status nb_tidal_active_batch(nb_ctx *ctx, const nb_tidal_item *items, int32_t n_items);

/* The tidal tensor of the rest of the system at k arbitrary points: at the centre
 * of mass of two bodies that are about to become a pair (Sec. 3 of the paper:
 * tight systems found during the run are taken out of the N-body integration),
 * the field of every body but the two.  As nb_tidal_active over [0, sys.n), with
 * point q at (pts[q], pts[k + q], pts[2k + q]) in place of a body and the rows
 * excl[q] and excl[k + q] left out (-1: none; excl may be NULL).  pts, excl,
 * tensor: device; tensor as in nb_tidal_active (T_ab of point q at
 * tensor[(3a+b)*k + q]).  Returns NB_EINVAL for eps < 0 or k < 0; k == 0 is a
 * no-op. */
nb_status nb_tidal_points(nb_ctx *ctx, const nb_system *sys, int32_t k, const double *pts,
                          const int32_t *excl, double eps, double *tensor);

/* The nearest neighbour of listed bodies, many systems in one launch: the
 * search for new tight pairs during the run (Sec. 3 of the paper: groups of
 * particles in tight systems are identified as the system evolves).  For body
 * i = i_idx[q] of an item: the other body j in [0, sys.n) of least squared
 * distance over the predicted set, |r|^2 = (dx dx + dy dy) + dz dz in FP64 with
 * every operation rounded (no fused multiply-add), the lowest j among equal
 * distances; nn[q] = j, r2[q] = |r|^2.  Bodies with i >= row_end (the
 * centre-of-mass bodies of a grouped system) or dt_i > dt_cap are not searched:
 * nn[q] = -1, r2[q] = +inf (also when the system has one body).  One workgroup
 * per listed body; integer results are exact and reproducible.  i_idx, nn, r2:
 * device; `status`: the item's device error word (NULL: the context's), which
 * receives NB_EINDEX for an index outside [0, n).  Items with m == 0 are
 * skipped.  Returns NB_EINVAL for a bad item (nothing enqueued). */
typedef struct {
    nb_system sys;
    const int32_t *i_idx;  /* device: listed bodies                            */
    int32_t m;
    int64_t row_end;       /* bodies at or above this row are not searched     */
    double dt_cap;         /* bodies with a larger step are not searched       */
    int32_t *nn;           /* device, m: nearest other body, or -1             */
    double *r2;            /* device, m: its squared distance, or +inf         */
    int32_t *status;       /* device word, or NULL                             */
} nb_nearest_item;
nb_status nb_nearest_active_batch(nb_ctx *ctx, const nb_nearest_item *items, int32_t n_items);

/* Host.  The reduced system of n bodies with n_pairs bound pairs (pairs[2k],
 * pairs[2k+1]: distinct indices in [0, n)): the bodies in no pair, in index
 * order, then one body per pair at its centre of mass, mass M = m1 + m2,
 *   x_c = (m1 x1 + m2 x2) / M,  v_c likewise;
 * and per pair M[k], r = x2 - x1, w = v2 - v1.  x, v: (n, 3) row-major; xr, vr:
 * (n - n_pairs, 3); mr: n - n_pairs; r, w: (n_pairs, 3).  All HOST memory.
 * Returns NB_OK or NB_EINVAL (bad or repeated indices). */
nb_status nb_pairs_reduce(int64_t n, const double *x, const double *v, const double *m,
                          int32_t n_pairs, const int64_t *pairs, double *xr, double *vr,
                          double *mr, double *M, double *r, double *w);

/* Host.  The inverse: members' positions and velocities from the reduced state
 * (xr, vr as written by nb_pairs_reduce, later advanced) and each pair's r, w:
 *   x1 = x_c - (m2 / M) r,  x2 = x_c + (m1 / M) r  (v alike).
 * x, v: (n, 3) outputs.  Returns NB_OK or NB_EINVAL. */
nb_status nb_pairs_members(int64_t n, const double *xr, const double *vr, const double *m,
                           int32_t n_pairs, const int64_t *pairs, const double *r,
                           const double *w, double *x, double *v);

/* Host.  The pairs' part of the quantity the scheme conserves:
 *   sum_k mu_k (|w_k|^2 / 2 - M_k / |r_k| - r_k . T_k r_k / 2),  mu = m1 m2 / M,
 * with T_k the tidal tensor (row-major 3x3 at T[9k..]) at the pair's current
 * time; compensated sum over k in order.  Returns NB_OK or NB_EINVAL. */
nb_status nb_pairs_energy(int32_t n_pairs, const double *m, const int64_t *pairs,
                          const double *r, const double *w, const double *T, double *out);

/* Host.  Per pair: the semimajor axis a of its relative orbit, written from r
 * and w as a = 1 / (2/|r| - |w|^2/M) (INFINITY if unbound) -- or, with r == NULL,
 * read from a -- and its perturbation
 *   gamma = |T|_F (2a)^3 / M,
 * the tidal acceleration across the orbit's diameter over the pair's own
 * acceleration at that distance (T row-major 3x3 at T[9k..]; T == NULL gives
 * gamma = 0 for a bound pair, INFINITY for an unbound one).  A server groups a
 * pair while gamma is small and returns it to the N-body system as two bodies
 * otherwise.  All arrays HOST memory.  Returns NB_OK or NB_EINVAL. */
nb_status nb_pairs_perturbation(int32_t n_pairs, const double *M, const double *r,
                                const double *w, const double *T, double *a, double *gamma);

/* Host.  When pairs return to the N-body system as two bodies, the quantity the
 * scheme conserves changes by their mutual potential turning from the unsoftened
 * into the softened one:  out = sum_k m1 m2 (1/|r_k| - 1/sqrt(|r_k|^2 + eps^2)).
 * Returns NB_OK or NB_EINVAL (a pair at r = 0). */
nb_status nb_pairs_split_energy(int32_t n_pairs, const double *m, const int64_t *pairs,
                                const double *r, double eps, double *out);

/* Host.  Two-body motion of a bound relative coordinate (r0, v0) of total mass M
 * over dt (any sign, any length): r'' = -M r / |r|^3.  All pointers are HOST
 * arrays of 3 doubles.  Returns NB_OK, NB_EINVAL, or NB_EUNBOUND when
 * |v0|^2/2 - M/|r0| >= 0. */
nb_status nb_kepler_drift(double M, const double *r0, const double *v0, double dt,
                          double *r1, double *v1);

/* Host.  Advance n pairs: pair k is row q = idx[k] (q = k when idx is NULL) of
 * M, r, v and status: mass M[q], relative r[3q..], v[3q..] (updated in place),
 * advanced over H[k] >= 0 in nsub = min(max_sub, max(1, ceil(per_period H / P)))
 * equal substeps (P its current orbital period), each kick (h/2) - drift h -
 * kick (h/2), a kick adding T(t) r times its length with T linear in t from
 * T0[9k..] to T1[9k..] (row-major 3x3).  H, T0 and T1 are indexed by k.  The
 * rows in idx must be distinct and >= 0; the caller's arrays must hold every
 * row named.  OpenMP over pairs.  status (may be NULL): per pair NB_OK or
 * NB_EUNBOUND.  All arrays are HOST memory.  Returns NB_OK, NB_EINVAL or
 * NB_EUNBOUND if any pair failed. */
nb_status nb_groups_advance(int32_t n, const int32_t *idx, const double *M, double *r,
                            double *v, const double *H, const double *T0, const double *T1,
                            int32_t per_period, int64_t max_sub, int32_t *status);

/* The same, queued on a host thread of the context: returns at once, so that the
 * caller can enqueue GPU work meanwhile.  Calls run one after another in call
 * order (each with one OpenMP thread fewer than the default, leaving a core to
 * the caller), so a later call may name rows that an earlier one is still
 * advancing.  Every array of every queued call must stay valid, and r, v and
 * status untouched, until nb_groups_wait, which blocks until the queue is empty
 * and returns the first failure since the previous wait (NB_OK if none).
 * NB_EINVAL (bad arguments) is returned at once and nothing is queued.
 * nb_ctx_destroy runs what is queued before it returns. */
nb_status nb_groups_advance_async(nb_ctx *ctx, int32_t n, const int32_t *idx, const double *M,
                                  double *r, double *v, const double *H, const double *T0,
                                  const double *T1, int32_t per_period, int64_t max_sub,
                                  int32_t *status);
nb_status nb_groups_wait(nb_ctx *ctx);

/* Library version string. */
const char *nb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
