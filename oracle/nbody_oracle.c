/*
 * nbody_oracle.c -- plain FP64 CPU reference for the direct N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the benchmark's
 * CPU-baseline leg call this library; the GPU product path never does, and the
 * two share no source.
 *
 * What it computes (Spera 2014, "Using GPUs to solve the classical N-body
 * problem", GPUHEP2014):
 *   - the gravitational pair sum of Eq. 1 with G = 1, softened as in Eq. 2
 *     (Plummer softening, Sec. 1), together with its time derivative (the jerk),
 *     which the Hermite scheme of Sec. 2 item 1 needs;
 *   - the 4th-order Hermite predictor and corrector (Sec. 2 item 1; the
 *     standard Makino-Aarseth form from Aarseth's book, cited there);
 *   - power-of-two block time steps (Sec. 2 item 2) with Aarseth's step
 *     criterion and the active-block selection;
 *   - the total energy, kinetic plus softened potential, used as the
 *     conservation diagnostic (Sec. 3, Fig. 3 right).
 *
 * Conventions: FP64 throughout, round to nearest, compiled without contraction
 * or fast-math.  Arrays of vectors are (n, 3) row-major.  The pair vector is
 * r_ij = r_j - r_i with a plus sign, which is Eq. 1 with its minus sign folded
 * into the direction of r_ij.  Sums over j run sequentially j = j0 .. j1-1 with
 * Neumaier's compensated summation, so the reference's own rounding error does
 * not grow with N.  OpenMP parallelises over i only; each i's sum is computed
 * by one thread in fixed order, so results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- compensated summation (Neumaier 1974) ---------------------------------- */
typedef struct { double s, c; } csum;

static void cs_add(csum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double cs_val(const csum *a) { return a->s + a->c; }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- acceleration and jerk (Eq. 1 with the softening of Eq. 2) --------------
 *
 * For each listed body i (ilist[k], k < ni) and each j in [j0, j1) with j != i:
 *   r  = x_j - x_i,  w = v_j - v_i,  s = r.r + eps^2
 *   a_i += m_j r / s^(3/2)
 *   jerk_i += m_j [ w / s^(3/2) - 3 (r.w) r / s^(5/2) ]
 * The jerk term is the time derivative of the acceleration term.  Positions and
 * velocities are those of the (predicted) j-set for both i and j.
 * Returns 0, or -1 if an index is out of range.
 */
int orc_force(int64_t n, const double *x, const double *v, const double *m,
              int64_t ni, const int64_t *ilist, int64_t j0, int64_t j1,
              double eps, double *acc, double *jerk)
{
    if (j0 < 0 || j1 > n || j0 > j1)
        return -1;
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        csum a[3] = {{0, 0}, {0, 0}, {0, 0}};
        csum jk[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = j0; j < j1; j++) {
            if (j == i)
                continue;
            double r[3], w[3];
            for (int d = 0; d < 3; d++) {
                r[d] = x[3 * j + d] - x[3 * i + d];
                w[d] = v[3 * j + d] - v[3 * i + d];
            }
            const double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + eps2;
            const double rinv = 1.0 / sqrt(s);
            const double rinv2 = rinv * rinv;
            const double mu = m[j] * rinv * rinv2;                  /* m_j s^(-3/2) */
            const double rw = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
            const double alpha = 3.0 * rw * rinv2;                  /* 3 (r.w) / s  */
            for (int d = 0; d < 3; d++) {
                cs_add(&a[d], mu * r[d]);
                cs_add(&jk[d], mu * (w[d] - alpha * r[d]));
            }
        }
        for (int d = 0; d < 3; d++) {
            acc[3 * k + d] = cs_val(&a[d]);
            jerk[3 * k + d] = cs_val(&jk[d]);
        }
    }
    return 0;
}

/* ---- magnitude scale of the pair sums -------------------------------------------
 * For each listed body i: S_a = sum_j |a_ij| and S_j = sum_j |jerk_ij|, the sums of
 * the magnitudes of the same pair terms orc_force adds (j != i, j in [j0, j1)).
 * S / |sum| is the cancellation factor of body i: rounding errors of size u per
 * term can move the sum by about u * S.  Returns 0, or -1 on a bad index/range.
 */
int orc_force_scale(int64_t n, const double *x, const double *v, const double *m,
                    int64_t ni, const int64_t *ilist, int64_t j0, int64_t j1,
                    double eps, double *sa, double *sj)
{
    if (j0 < 0 || j1 > n || j0 > j1)
        return -1;
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        csum ta = {0, 0}, tj = {0, 0};
        for (int64_t j = j0; j < j1; j++) {
            if (j == i)
                continue;
            double dr[3], dw[3], term[3];
            for (int d = 0; d < 3; d++) {
                dr[d] = x[3 * j + d] - x[3 * i + d];
                dw[d] = v[3 * j + d] - v[3 * i + d];
            }
            const double d2 = dr[0] * dr[0] + dr[1] * dr[1] + dr[2] * dr[2];
            const double q = 1.0 / sqrt(d2 + eps2);                /* s^(-1/2) */
            const double mq3 = m[j] * q * q * q;                    /* m_j s^(-3/2) */
            const double radial = 3.0 * (dr[0] * dw[0] + dr[1] * dw[1] + dr[2] * dw[2]) * q * q;
            for (int d = 0; d < 3; d++)
                term[d] = mq3 * (dw[d] - radial * dr[d]);
            cs_add(&ta, mq3 * sqrt(d2));
            cs_add(&tj, sqrt(term[0] * term[0] + term[1] * term[1] + term[2] * term[2]));
        }
        sa[k] = cs_val(&ta);
        sj[k] = cs_val(&tj);
    }
    return 0;
}

/* ---- velocity magnitude scale ------------------------------------------------
 * Per listed body: sum_j m_j (|v_i| + |v_j|) / (|r_ij|^2 + eps^2)^(3/2) over j in
 * [j0, j1), j != i.  A scale for the error that rounding the velocities to FP32
 * (before their difference is formed) can cause in the jerk sum.
 */
int orc_velocity_scale(int64_t n, const double *x, const double *v, const double *m,
                       int64_t ni, const int64_t *ilist, int64_t j0, int64_t j1, double eps,
                       double *sv)
{
    if (j0 < 0 || j1 > n || j0 > j1)
        return -1;
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        const double vi = sqrt(v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] +
                               v[3 * i + 2] * v[3 * i + 2]);
        csum t = {0, 0};
        for (int64_t j = j0; j < j1; j++) {
            if (j == i)
                continue;
            double dr[3];
            for (int d = 0; d < 3; d++)
                dr[d] = x[3 * j + d] - x[3 * i + d];
            const double s = dr[0] * dr[0] + dr[1] * dr[1] + dr[2] * dr[2] + eps2;
            const double vj = sqrt(v[3 * j] * v[3 * j] + v[3 * j + 1] * v[3 * j + 1] +
                                   v[3 * j + 2] * v[3 * j + 2]);
            cs_add(&t, m[j] * (vi + vj) / (s * sqrt(s)));
        }
        sv[k] = cs_val(&t);
    }
    return 0;
}

/* ---- total energy ------------------------------------------------------------
 * E = sum_i m_i |v_i|^2 / 2  -  sum_{i<j} m_i m_j / sqrt(|r_ij|^2 + eps^2)
 * (the softened potential whose gradient is the force of Eq. 2; the self term
 * i = j is excluded).  Kinetic and potential parts are returned separately.
 * Each row i sums j > i in order; rows are then combined in order i = 0..n-1.
 */
void orc_energy(int64_t n, const double *x, const double *v, const double *m,
                double eps, double *kinetic, double *potential)
{
    const double eps2 = eps * eps;
    double *row = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; i++) {
        csum p = {0, 0};
        for (int64_t j = i + 1; j < n; j++) {
            double r2 = 0.0;
            for (int d = 0; d < 3; d++) {
                const double dr = x[3 * j + d] - x[3 * i + d];
                r2 += dr * dr;
            }
            cs_add(&p, m[i] * m[j] / sqrt(r2 + eps2));
        }
        row[i] = cs_val(&p);
    }
    csum pot = {0, 0}, kin = {0, 0};
    for (i = 0; i < n; i++) {
        cs_add(&pot, row[i]);
        const double v2 = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
        cs_add(&kin, 0.5 * m[i] * v2);
    }
    free(row);
    *kinetic = cs_val(&kin);
    *potential = -cs_val(&pot);
}

/* ---- predictor (Hermite 4th order) -------------------------------------------
 * Every body is Taylor-expanded from its own time t_i to t_next (Sec. 2 item 2:
 * bodies outside the active block are only predicted), with d = t_next - t_i:
 *   xp = x + v d + a d^2/2 + j d^3/6,   vp = v + a d + j d^2/2
 */
void orc_predict(int64_t n, const double *x, const double *v, const double *a,
                 const double *jk, const double *t, double t_next,
                 double *xp, double *vp)
{
    for (int64_t i = 0; i < n; i++) {
        const double d = t_next - t[i];
        for (int c = 0; c < 3; c++) {
            const int64_t q = 3 * i + c;
            xp[q] = x[q] + v[q] * d + a[q] * d * d / 2.0 + jk[q] * d * d * d / 6.0;
            vp[q] = v[q] + a[q] * d + jk[q] * d * d / 2.0;
        }
    }
}

/* ---- active block (Sec. 2 item 2) ---------------------------------------------
 * t_next = min_i (t_i + dt_i); the active block is every i with t_i + dt_i equal
 * to t_next, in ascending order of i.  Returns the block size m.
 */
int64_t orc_select(int64_t n, const double *t, const double *dt, double *t_next,
                   int64_t *ilist)
{
    double tn = INFINITY;
    for (int64_t i = 0; i < n; i++)
        if (t[i] + dt[i] < tn)
            tn = t[i] + dt[i];
    int64_t mcount = 0;
    for (int64_t i = 0; i < n; i++)
        if (t[i] + dt[i] == tn)
            ilist[mcount++] = i;
    *t_next = tn;
    return mcount;
}

static double norm3(const double *u)
{
    return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
}

/* ---- startup step --------------------------------------------------------------
 * At t = 0 every body gets dt = the largest power of two not above
 * min(eta_s |a| / |j|, dt_max).  Returns 0, -4 if a step falls below dt_min,
 * -5 on a non-finite value.
 */
int orc_init_dt(int64_t n, const double *a, const double *jk, double eta_s,
                double dt_max, double dt_min, double *dt)
{
    for (int64_t i = 0; i < n; i++) {
        const double an = norm3(a + 3 * i), jn = norm3(jk + 3 * i);
        if (!isfinite(an) || !isfinite(jn))
            return -5;
        double want = (jn > 0.0) ? eta_s * an / jn : dt_max;
        if (want > dt_max)
            want = dt_max;
        double step = dt_max;
        while (step > want)
            step /= 2.0;
        if (step < dt_min)
            return -4;
        dt[i] = step;
    }
    return 0;
}

/* ---- corrector and new step (Hermite 4th order, block steps) ------------------
 * For active body i with h = t_next - t_i, old (a0, j0) at t_i, new (a1, j1) at
 * t_next and predicted (xp, vp):
 *   a2 = [-6 (a0 - a1) - h (4 j0 + 2 j1)] / h^2       (second derivative at t_i)
 *   a3 = [12 (a0 - a1) + 6 h (j0 + j1)] / h^3          (third derivative)
 *   x  = xp + a2 h^4/24 + a3 h^5/120,   v = vp + a2 h^3/6 + a3 h^4/24
 * The new step follows Aarseth's criterion evaluated at t_next, with the second
 * derivative there a2' = a2 + a3 h:
 *   dtA = sqrt( eta (|a1| |a2'| + |j1|^2) / (|j1| |a3| + |a2'|^2) )
 * and is kept a power of two (Sec. 2 item 2): halve while larger than dtA; if no
 * halving was needed, double once when dtA >= 2 h, t_next is a multiple of 2 h
 * and 2 h <= dt_max.  The body's time becomes t_next.
 * dta_out (may be NULL) receives the unquantised dtA of each active body.
 * Returns 0, -4 if a new step falls below dt_min, -5 on a non-finite value.
 */
int orc_correct(int64_t n, int64_t mcount, const int64_t *ilist, double t_next,
                const double *xp, const double *vp, const double *acc_new,
                const double *jerk_new, double *x, double *v, double *a,
                double *jk, double *t, double *dt, double eta, double dt_max,
                double dt_min, double *dta_out)
{
    int status = 0;
    for (int64_t k = 0; k < mcount; k++) {
        const int64_t i = ilist[k];
        if (i < 0 || i >= n)
            return -1;
        const double h = t_next - t[i];
        double a2[3], a3[3], a2e[3];
        for (int c = 0; c < 3; c++) {
            const double a0 = a[3 * i + c], j0 = jk[3 * i + c];
            const double a1 = acc_new[3 * k + c], j1 = jerk_new[3 * k + c];
            a2[c] = (-6.0 * (a0 - a1) - h * (4.0 * j0 + 2.0 * j1)) / (h * h);
            a3[c] = (12.0 * (a0 - a1) + 6.0 * h * (j0 + j1)) / (h * h * h);
            x[3 * i + c] = xp[3 * i + c] + a2[c] * h * h * h * h / 24.0
                           + a3[c] * h * h * h * h * h / 120.0;
            v[3 * i + c] = vp[3 * i + c] + a2[c] * h * h * h / 6.0
                           + a3[c] * h * h * h * h / 24.0;
            a[3 * i + c] = a1;
            jk[3 * i + c] = j1;
            a2e[c] = a2[c] + a3[c] * h;
        }
        const double an = norm3(acc_new + 3 * k), jn = norm3(jerk_new + 3 * k);
        const double sn = norm3(a2e), cn = norm3(a3);
        const double num = an * sn + jn * jn, den = jn * cn + sn * sn;
        double dta;
        if (den > 0.0)
            dta = sqrt(eta * num / den);
        else
            dta = INFINITY;
        if (isnan(dta) || !isfinite(an) || !isfinite(jn))
            return -5;
        if (dta_out)
            dta_out[k] = dta;
        double step = h;
        if (step > dta) {
            while (step > dta)
                step /= 2.0;
        } else if (dta >= 2.0 * h && fmod(t_next, 2.0 * h) == 0.0 && 2.0 * h <= dt_max) {
            step = 2.0 * h;
        }
        if (step < dt_min)
            status = -4;
        t[i] = t_next;
        dt[i] = step;
    }
    return status;
}

/* =========================================================================
 * 6th-order Hermite (the integrator of the paper's HiGPUs, Sec. 2 item 1).
 * ========================================================================= */

/* ---- acceleration, jerk and snap ---------------------------------------------
 * For each listed body i and each j in [j0, j1) with j != i, with the
 * (predicted) relative position r, velocity w and acceleration b of j:
 *   s = r.r + eps^2,  A = m_j r / s^(3/2)                 (Eq. 1-2)
 *   alpha = (r.w)/s,  J = m_j w / s^(3/2) - 3 alpha A      (dA/dt)
 *   beta = (w.w + r.b)/s + alpha^2,
 *   S = m_j b / s^(3/2) - 6 alpha J - 3 beta A            (d^2A/dt^2)
 * summed with compensated sums in order j = j0 .. j1-1.
 */
int orc_force6(int64_t n, const double *x, const double *v, const double *ac,
               const double *m, int64_t ni, const int64_t *ilist, int64_t j0, int64_t j1,
               double eps, double *acc, double *jerk, double *snap)
{
    if (j0 < 0 || j1 > n || j0 > j1)
        return -1;
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        csum sa[3] = {{0, 0}, {0, 0}, {0, 0}};
        csum sj[3] = {{0, 0}, {0, 0}, {0, 0}};
        csum ss[3] = {{0, 0}, {0, 0}, {0, 0}};
        for (int64_t j = j0; j < j1; j++) {
            if (j == i)
                continue;
            double rij[3], vij[3], aij[3];
            for (int d = 0; d < 3; d++) {
                rij[d] = x[3 * j + d] - x[3 * i + d];
                vij[d] = v[3 * j + d] - v[3 * i + d];
                aij[d] = ac[3 * j + d] - ac[3 * i + d];
            }
            const double s = rij[0] * rij[0] + rij[1] * rij[1] + rij[2] * rij[2] + eps2;
            const double rinv = 1.0 / sqrt(s);
            const double inv_s = rinv * rinv;
            const double mu = m[j] * rinv * inv_s;
            const double alpha = (rij[0] * vij[0] + rij[1] * vij[1] + rij[2] * vij[2]) * inv_s;
            const double beta = (vij[0] * vij[0] + vij[1] * vij[1] + vij[2] * vij[2]
                                 + rij[0] * aij[0] + rij[1] * aij[1] + rij[2] * aij[2]) * inv_s
                                + alpha * alpha;
            for (int d = 0; d < 3; d++) {
                const double Ad = mu * rij[d];
                const double Jd = mu * vij[d] - 3.0 * alpha * Ad;
                const double Sd = mu * aij[d] - 6.0 * alpha * Jd - 3.0 * beta * Ad;
                cs_add(&sa[d], Ad);
                cs_add(&sj[d], Jd);
                cs_add(&ss[d], Sd);
            }
        }
        for (int d = 0; d < 3; d++) {
            acc[3 * k + d] = cs_val(&sa[d]);
            jerk[3 * k + d] = cs_val(&sj[d]);
            snap[3 * k + d] = cs_val(&ss[d]);
        }
    }
    return 0;
}

/* ---- magnitude scale of the snap sum --------------------------------------------
 * Per listed body: sum over the same j as orc_force6 of |S_ij|, the length of
 * each pair's snap term (the size of the numbers a finite-precision sum of the
 * snap adds up, for error bounds relative to that sum's own scale).
 */
int orc_force6_scale(int64_t n, const double *x, const double *v, const double *ac,
                     const double *m, int64_t ni, const int64_t *ilist, int64_t j0, int64_t j1,
                     double eps, double *ss)
{
    if (j0 < 0 || j1 > n || j0 > j1)
        return -1;
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        csum tot = {0, 0};
        for (int64_t j = j0; j < j1; j++) {
            if (j == i)
                continue;
            double px[3], pv[3], pa[3], term[3];
            for (int d = 0; d < 3; d++) {
                px[d] = x[3 * j + d] - x[3 * i + d];
                pv[d] = v[3 * j + d] - v[3 * i + d];
                pa[d] = ac[3 * j + d] - ac[3 * i + d];
            }
            const double ss2 = px[0] * px[0] + px[1] * px[1] + px[2] * px[2] + eps2;
            const double q2 = 1.0 / ss2;
            const double mq3 = m[j] * q2 / sqrt(ss2);
            const double al = (px[0] * pv[0] + px[1] * pv[1] + px[2] * pv[2]) * q2;
            const double bt = (pv[0] * pv[0] + pv[1] * pv[1] + pv[2] * pv[2]
                               + px[0] * pa[0] + px[1] * pa[1] + px[2] * pa[2]) * q2 + al * al;
            for (int d = 0; d < 3; d++) {
                const double jt = pv[d] - 3.0 * al * px[d];
                term[d] = mq3 * (pa[d] - 6.0 * al * jt - 3.0 * bt * px[d]);
            }
            cs_add(&tot, sqrt(term[0] * term[0] + term[1] * term[1] + term[2] * term[2]));
        }
        ss[k] = cs_val(&tot);
    }
    return 0;
}

/* ---- 6th-order startup step ------------------------------------------------------
 * At t = 0 every body gets dt = the largest power of two not above
 * min(eta_s (sqrt(|a||s|) + |j|) / (|s| + |j|^2 / |a|), dt_max): the step form of
 * the 6th-order scheme from the computed acceleration, jerk and snap (no crackle
 * exists yet).  It equals eta_s/omega on a circular orbit, like the 4th-order
 * rule eta_s |a|/|j|, and also sees an approaching neighbour through the snap.
 * Returns 0, -4 if a step falls below dt_min, -5 on a non-finite value.
 */
int orc_init_dt6(int64_t n, const double *a, const double *jk, const double *sn,
                 double eta_s, double dt_max, double dt_min, double *dt)
{
    for (int64_t i = 0; i < n; i++) {
        const double an = norm3(a + 3 * i), jn = norm3(jk + 3 * i), sm = norm3(sn + 3 * i);
        if (!isfinite(an) || !isfinite(jn) || !isfinite(sm))
            return -5;
        const double top = sqrt(an * sm) + jn;
        const double bottom = sm + (an > 0.0 ? jn * jn / an : 0.0);
        double want = (bottom > 0.0) ? eta_s * (top / bottom) : dt_max;
        if (want > dt_max)
            want = dt_max;
        double pow2 = dt_max;
        while (pow2 > want)
            pow2 /= 2.0;
        if (pow2 < dt_min)
            return -4;
        dt[i] = pow2;
    }
    return 0;
}

/* ---- 6th-order predictor --------------------------------------------------------
 * d = t_next - t_i:
 *   xp = x + v d + a d^2/2 + j d^3/6 + s d^4/24 + c d^5/120
 *   vp = v + a d + j d^2/2 + s d^3/6 + c d^4/24
 *   ap = a + j d + s d^2/2 + c d^3/6
 * (s = snap, c = crackle: the second and third derivatives of the acceleration).
 */
void orc_predict6(int64_t n, const double *x, const double *v, const double *a,
                  const double *jk, const double *sn, const double *cr, const double *t,
                  double t_next, double *xp, double *vp, double *ap)
{
    for (int64_t i = 0; i < n; i++) {
        const double tau = t_next - t[i];
        for (int c = 0; c < 3; c++) {
            const int64_t q = 3 * i + c;
            xp[q] = x[q] + v[q] * tau + a[q] * tau * tau / 2.0 + jk[q] * tau * tau * tau / 6.0
                    + sn[q] * tau * tau * tau * tau / 24.0 + cr[q] * tau * tau * tau * tau * tau / 120.0;
            vp[q] = v[q] + a[q] * tau + jk[q] * tau * tau / 2.0 + sn[q] * tau * tau * tau / 6.0
                    + cr[q] * tau * tau * tau * tau / 24.0;
            ap[q] = a[q] + jk[q] * tau + sn[q] * tau * tau / 2.0 + cr[q] * tau * tau * tau / 6.0;
        }
    }
}

/* Solve the 3x3 system M u = r by Gaussian elimination with partial pivoting. */
static void solve3(double M[3][3], double r[3], double u[3])
{
    for (int col = 0; col < 3; col++) {
        int piv = col;
        for (int row = col + 1; row < 3; row++)
            if (fabs(M[row][col]) > fabs(M[piv][col]))
                piv = row;
        for (int q = 0; q < 3; q++) {
            const double tmp = M[col][q];
            M[col][q] = M[piv][q];
            M[piv][q] = tmp;
        }
        const double tr = r[col];
        r[col] = r[piv];
        r[piv] = tr;
        for (int row = col + 1; row < 3; row++) {
            const double f = M[row][col] / M[col][col];
            for (int q = col; q < 3; q++)
                M[row][q] -= f * M[col][q];
            r[row] -= f * r[col];
        }
    }
    for (int row = 2; row >= 0; row--) {
        double acc = r[row];
        for (int q = row + 1; q < 3; q++)
            acc -= M[row][q] * u[q];
        u[row] = acc / M[row][row];
    }
}

/* Crackle (third derivative) at tau = h of the degree-5 polynomial a(tau) with
 * a(0) = a0, a'(0) = j0, a''(0) = s0, a(h) = a1, a'(h) = j1, a''(h) = s1
 * (the Hermite interpolant of the step).  Coefficients k0..k5 of
 * sum k_n tau^n: k0, k1, k2 from the conditions at 0; k3, k4, k5 from the three
 * conditions at h, solved as a linear system in u_n = k_n h^n. */
static double hermite5_crackle(double h, double a0, double j0, double s0, double a1,
                               double j1, double s1)
{
    const double k0 = a0, k1 = j0, k2 = s0 / 2.0;
    double M[3][3] = {{1.0, 1.0, 1.0}, {3.0, 4.0, 5.0}, {6.0, 12.0, 20.0}};
    double r[3] = {a1 - (k0 + k1 * h + k2 * h * h),
                   (j1 - (k1 + 2.0 * k2 * h)) * h,
                   (s1 - 2.0 * k2) * h * h};
    double u[3];
    solve3(M, r, u);
    const double k3 = u[0] / (h * h * h), k4 = u[1] / (h * h * h * h),
                 k5 = u[2] / (h * h * h * h * h);
    return 6.0 * k3 + 24.0 * k4 * h + 60.0 * k5 * h * h;
}

/* ---- 6th-order corrector and new step -------------------------------------------
 * Active body i, h = t_next - t_i, (a0, j0, s0) stored at t_i and (a1, j1, s1)
 * new at t_next; the two-point Hermite quadratures (exact for a quartic
 * acceleration):
 *   v1 = v0 + h/2 (a0 + a1) - h^2/10 (j1 - j0) + h^3/120 (s0 + s1)
 *   x1 = x0 + h/2 (v0 + v1) - h^2/10 (a1 - a0) + h^3/120 (j0 + j1)
 * The crackle c1 at t_next comes from the degree-5 Hermite interpolant of the
 * step and is stored for the predictor.  New step: the lowest generalized
 * Aarseth form
 *   dtC = eta (sqrt(|a1||s1|) + |j1|) / (sqrt(|j1||c1|) + |s1|),
 * not below one eighth of the same form with the crackle term replaced by
 * |j1|^2/|a1| (a term of the same dimension built from computed derivatives
 * only):
 *   dtD = eta (sqrt(|a1||s1|) + |j1|) / (|s1| + |j1|^2 / |a1|),
 *   dtA = max(dtC, dtD / 8).
 * The crackle is what anticipates an approaching close encounter (its pair
 * term grows as r^-5); the floor keeps the step from running away where the
 * interpolated crackle is dominated by the forces' rounding error, which it
 * carries multiplied by 60/h^3.  Both give eta/omega on a circular orbit.
 * The step is kept a power of two by the same rule as the 4th-order scheme.
 * dta_out (may be NULL) receives the unquantised dtA.
 */
int orc_correct6(int64_t n, int64_t mcount, const int64_t *ilist, double t_next,
                 const double *acc_new, const double *jerk_new, const double *snap_new,
                 double *x, double *v, double *a, double *jk, double *sn, double *cr,
                 double *t, double *dt, double eta, double dt_max, double dt_min,
                 double *dta_out)
{
    int status = 0;
    for (int64_t k = 0; k < mcount; k++) {
        const int64_t i = ilist[k];
        if (i < 0 || i >= n)
            return -1;
        const double h = t_next - t[i];
        double d3v[3];
        for (int c = 0; c < 3; c++) {
            const int64_t q = 3 * i + c;
            const double a0 = a[q], j0 = jk[q], s0 = sn[q];
            const double a1 = acc_new[3 * k + c], j1 = jerk_new[3 * k + c],
                         s1 = snap_new[3 * k + c];
            const double v0 = v[q], x0 = x[q];
            const double v1 = v0 + h / 2.0 * (a0 + a1) - h * h / 10.0 * (j1 - j0)
                              + h * h * h / 120.0 * (s0 + s1);
            const double x1 = x0 + h / 2.0 * (v0 + v1) - h * h / 10.0 * (a1 - a0)
                              + h * h * h / 120.0 * (j0 + j1);
            d3v[c] = hermite5_crackle(h, a0, j0, s0, a1, j1, s1);
            x[q] = x1;
            v[q] = v1;
            a[q] = a1;
            jk[q] = j1;
            sn[q] = s1;
            cr[q] = d3v[c];
        }
        const double an = norm3(acc_new + 3 * k), jn = norm3(jerk_new + 3 * k),
                     sN = norm3(snap_new + 3 * k);
        const double cn = norm3(d3v);
        const double num = sqrt(an * sN) + jn;
        const double den_d = sN + (an > 0.0 ? jn * jn / an : 0.0);
        const double den_c = sN + sqrt(jn * cn);
        const double dtd = den_d > 0.0 ? eta * (num / den_d) : INFINITY;
        double dta = den_c > 0.0 ? eta * (num / den_c) : INFINITY;
        if (dta < dtd / 8.0)
            dta = dtd / 8.0;
        if (isnan(dta) || !isfinite(an) || !isfinite(jn) || !isfinite(sN))
            return -5;
        if (dta_out)
            dta_out[k] = dta;
        double step = h;
        if (step > dta) {
            while (step > dta)
                step /= 2.0;
        } else {
            const double h2 = 2.0 * h;
            if (dta >= h2 && fmod(t_next, h2) == 0.0 && h2 <= dt_max)
                step = h2;
        }
        if (step < dt_min)
            status = -4;
        t[i] = t_next;
        dt[i] = step;
    }
    return status;
}

/* =========================================================================
 * Tight groups (the HiGPUs-R scheme of Sec. 3): a bound pair is carried in the
 * N-body system as one body at its centre of mass, and its relative orbit is
 * advanced separately: exact two-body (Kepler) motion plus the tidal field of
 * the rest of the system, linearised about the centre of mass.
 * ========================================================================= */

/* ---- tidal tensor ------------------------------------------------------------------
 * For each listed body i: T_ab = d a_a / d x_b of the softened field of the
 * bodies j in [j0, j1), j != i, at x_i:
 *   T_ab = sum_j m_j (3 r_a r_b / s^(5/2) - delta_ab / s^(3/2)),  r = x_j - x_i,
 * s = |r|^2 + eps^2; row-major 3x3 per body (T[9k + 3a + b]).
 */
int orc_tidal(int64_t n, const double *x, const double *m, int64_t ni, const int64_t *ilist,
              int64_t j0, int64_t j1, double eps, double *T)
{
    if (j0 < 0 || j1 > n || j0 > j1)
        return -1;
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        csum acc[9];
        for (int q = 0; q < 9; q++) {
            acc[q].s = 0.0;
            acc[q].c = 0.0;
        }
        for (int64_t j = j0; j < j1; j++) {
            if (j == i)
                continue;
            double d[3];
            for (int c = 0; c < 3; c++)
                d[c] = x[3 * j + c] - x[3 * i + c];
            const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
            const double s32 = s * sqrt(s);
            const double s52 = s32 * s;
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    cs_add(&acc[3 * a + b],
                           m[j] * (3.0 * d[a] * d[b] / s52 - (a == b ? 1.0 : 0.0) / s32));
        }
        for (int q = 0; q < 9; q++)
            T[9 * k + q] = cs_val(&acc[q]);
    }
    return 0;
}

/* ---- tidal tensor at a point -----------------------------------------------------
 * The tidal tensor of the softened field at arbitrary points p_k, with up to two
 * bodies left out per point (excl[2k], excl[2k+1]; -1 leaves out none): the field
 * of the rest of the system at the centre of mass of a pair that is about to be
 * taken out of the N-body system.  The same sum as orc_tidal with r = x_j - p_k.
 */
int orc_tidal_points(int64_t n, const double *x, const double *m, int64_t np,
                     const double *p, const int64_t *excl, double eps, double *T)
{
    for (int64_t k = 0; k < 2 * np; k++)
        if (excl[k] < -1 || excl[k] >= n)
            return -1;
    const double eps2 = eps * eps;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < np; k++) {
        csum acc[9];
        for (int q = 0; q < 9; q++) {
            acc[q].s = 0.0;
            acc[q].c = 0.0;
        }
        for (int64_t j = 0; j < n; j++) {
            if (j == excl[2 * k] || j == excl[2 * k + 1])
                continue;
            double d[3];
            for (int c = 0; c < 3; c++)
                d[c] = x[3 * j + c] - p[3 * k + c];
            const double s = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] + eps2;
            const double w3 = m[j] / (s * sqrt(s));          /* m / s^(3/2) */
            const double w5 = 3.0 * w3 / s;                  /* 3 m / s^(5/2) */
            for (int a = 0; a < 3; a++)
                for (int b = 0; b < 3; b++)
                    cs_add(&acc[3 * a + b], w5 * d[a] * d[b] - (a == b ? w3 : 0.0));
        }
        for (int q = 0; q < 9; q++)
            T[9 * k + q] = cs_val(&acc[q]);
    }
    return 0;
}

/* ---- nearest neighbour ------------------------------------------------------------
 * For each listed body i: the other body j (any index in [0, n)) with the least
 * squared distance |x_j - x_i|^2, formed as (dx dx + dy dy) + dz dz in FP64 without
 * contraction; the lowest j among equal distances.  A listed body is searched
 * only if i < row_end and dt_i <= dt_cap (dt may be NULL: every body qualifies);
 * otherwise, or when no other body exists, nn = -1 and r2 = +inf.  This is how
 * candidates for a new bound pair are found: two bodies of the same block that
 * are each other's nearest neighbour.
 */
int orc_nearest(int64_t n, const double *x, int64_t ni, const int64_t *ilist, int64_t row_end,
                const double *dt, double dt_cap, int64_t *nn, double *r2)
{
    for (int64_t k = 0; k < ni; k++)
        if (ilist[k] < 0 || ilist[k] >= n)
            return -1;
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16)
    for (k = 0; k < ni; k++) {
        const int64_t i = ilist[k];
        int64_t best = -1;
        double bd = INFINITY;
        if (i < row_end && (!dt || dt[i] <= dt_cap)) {
            for (int64_t j = 0; j < n; j++) {
                if (j == i)
                    continue;
                const double dx = x[3 * j] - x[3 * i];
                const double dy = x[3 * j + 1] - x[3 * i + 1];
                const double dz = x[3 * j + 2] - x[3 * i + 2];
                const double d = dx * dx + dy * dy + dz * dz;
                if (d < bd) {
                    bd = d;
                    best = j;
                }
            }
        }
        nn[k] = best;
        r2[k] = best >= 0 ? bd : INFINITY;
    }
    return 0;
}

/* ---- Kepler drift -----------------------------------------------------------------
 * Exact motion of the relative coordinate of an isolated bound pair of total
 * mass M over a time dt (r'' = -M r / |r|^3), by the f and g functions of the
 * eccentric-anomaly change dE, which solves
 *   n dt = dE - (1 - r0/a) sin dE + (sigma0 / sqrt(a)) (1 - cos dE),
 * with 1/a = 2/r0 - v0^2/M, n = sqrt(M/a^3), sigma0 = r0.v0 / sqrt(M):
 *   f = 1 - (a/r0)(1 - cos dE),           g = dt - (dE - sin dE)/n,
 *   r = a + (r0 - a) cos dE + sigma0 sqrt(a) sin dE,
 *   fd = -sqrt(M a) sin dE / (r r0),      gd = 1 - (a/r)(1 - cos dE),
 *   r1 = f r0 + g v0,  v1 = fd r0 + gd v0.
 * Returns 0, or -1 for an unbound or degenerate pair.
 */
int orc_kepler_drift(double M, const double *r0, const double *v0, double dt, double *r1,
                     double *v1)
{
    const double rr = sqrt(r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
    const double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    if (!(M > 0.0) || !(rr > 0.0))
        return -1;
    const double inv_a = 2.0 / rr - vv / M;
    if (!(inv_a > 0.0))
        return -1;
    const double a = 1.0 / inv_a;
    const double nmean = sqrt(M * inv_a * inv_a * inv_a);
    const double sig = (r0[0] * v0[0] + r0[1] * v0[1] + r0[2] * v0[2]) / sqrt(M);
    const double ce = 1.0 - rr / a, se = sig / sqrt(a);   /* e cos E0, e sin E0 */
    /* reduce n dt by whole periods, solve for the remainder */
    const double twopi = 6.283185307179586476925286766559;
    const double phase = nmean * dt;
    const double turns = floor(phase / twopi);
    const double Mrem = phase - turns * twopi;
    /* F(x) = x - ce sin x + se (1 - cos x) - Mrem increases monotonically
     * (F' = 1 - e cos(E0 + x) >= 1 - e > 0), F(0) = -Mrem <= 0 < F(2 pi): Newton
     * steps kept inside a shrinking bracket, bisection when a step leaves it */
    double lo = 0.0, hi = twopi, x = Mrem;                /* x = dE - 2 pi turns */
    for (int it = 0; it < 200; it++) {
        const double F = x - ce * sin(x) + se * (1.0 - cos(x)) - Mrem;
        if (F > 0.0)
            hi = x;
        else
            lo = x;
        const double Fp = 1.0 - ce * cos(x) + se * sin(x);
        double xn = x - F / Fp;
        if (!(xn > lo && xn < hi))
            xn = 0.5 * (lo + hi);
        const double dx = xn - x;
        x = xn;
        if (fabs(dx) <= 4e-16 * (1.0 + fabs(x)) || hi - lo <= 4e-16 * (1.0 + hi))
            break;
    }
    const double cx = cos(x), sx = sin(x);
    const double f = 1.0 - (a / rr) * (1.0 - cx);
    const double g = (Mrem - (x - sx)) / nmean;
    const double r = a + (rr - a) * cx + sig * sqrt(a) * sx;
    const double fd = -sqrt(M * a) * sx / (r * rr);
    const double gd = 1.0 - (a / r) * (1.0 - cx);
    for (int c = 0; c < 3; c++) {
        r1[c] = f * r0[c] + g * v0[c];
        v1[c] = fd * r0[c] + gd * v0[c];
    }
    return 0;
}

/* ---- relative orbit under a tidal field ---------------------------------------------
 * Advance (r, v) of a pair of mass M over [0, H] in nsub equal substeps of
 * h = H / nsub, each kick (h/2) - drift h - kick (h/2): the drift is the exact
 * Kepler motion, a kick adds T(t) r times its length, and T(t) is interpolated
 * linearly between T0 (at 0) and T1 (at H).  Second order in h for the tidal
 * part, exact for T = 0.  Returns 0 or the drift's error.
 */
int orc_group_advance(double M, double *r, double *v, double H, int64_t nsub, const double *T0,
                      const double *T1)
{
    if (nsub < 1)
        return -1;
    const double h = H / (double)nsub;
    for (int64_t q = 0; q < nsub; q++) {
        const double wa = (double)q / (double)nsub, wb = (double)(q + 1) / (double)nsub;
        for (int half = 0; half < 2; half++) {
            const double w = half == 0 ? wa : wb;
            if (half == 1) {
                double r1[3], v1[3];
                const int rc = orc_kepler_drift(M, r, v, h, r1, v1);
                if (rc)
                    return rc;
                for (int c = 0; c < 3; c++) {
                    r[c] = r1[c];
                    v[c] = v1[c];
                }
            }
            for (int a = 0; a < 3; a++) {
                double tr = 0.0;
                for (int b = 0; b < 3; b++)
                    tr += ((1.0 - w) * T0[3 * a + b] + w * T1[3 * a + b]) * r[b];
                v[a] += 0.5 * h * tr;
            }
        }
    }
    return 0;
}
