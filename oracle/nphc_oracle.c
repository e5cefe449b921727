/*
 * nphc_oracle.c -- plain, slow FP64 CPU oracle for numerical polynomial
 * homotopy continuation (NPHC) on the power-law XY ring.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the HIP
 * path under paper_1104_5497_amd/ and neither side includes the other.
 *
 * What it computes (Mehta, "Finding all the stationary points of a potential
 * energy landscape via numerical polynomial homotopy continuation method"):
 *
 *   target system P  -- eq. (1): for free spins k = 1..N-1 (theta_N = 0, so
 *                       x_N = cos 0 = 1, y_N = sin 0 = 0)
 *                         F_k     = sum_{j != k} J_kj (y_k x_j - x_k y_j)
 *                         F_{m+k} = x_k^2 + y_k^2 - 1
 *                       with x = cos(theta) = c, y = sin(theta) = s.
 *   start system Q   -- section "NPHC method": q_k = z_k^{d_k} - 1 with
 *                       d_k = 2, start solutions z_k = +-1.
 *   homotopy         -- H(z, t) = gamma (1 - t) Q(z) + t P(z), t: 0 -> 1.
 *   path tracking    -- predictor (classical RK4 on the Davidenko equation
 *                       dz/dt = -H_z^{-1} H_t, or the paper's Euler) followed
 *                       by Newton's corrector, with adaptive step size.
 *   refinement       -- Newton on P at t = 1 ("refined up to machine
 *                       precision", section "NPHC method").
 *
 * Every linear solve is a dense n x n Gaussian elimination with partial
 * pivoting (largest |re| + |im| in the column, ties to the lower row).
 * Unknowns are ordered z = (x_1..x_m, y_1..y_m), m = N - 1, n = 2m, and row k
 * of Q is paired with row k of P.  A path id p in [0, 2^n) starts at
 * z_k = 1 - 2 * bit_k(p).
 *
 * A second system kind, F_k = a_k z_k^2 - c_k (separable quadratics), exists
 * only so that tests can pin the tracker against closed-form paths (the
 * paper's univariate example x^2 - 5 from x^2 - 1 is a = 1, c = 5).
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORACLE_NMAX 48 /* unknowns; N <= 25 */

enum { SYS_XY = 0, SYS_SEPARABLE = 1 };

/* path outcomes (tracking) and endpoint classes (refinement) */
enum {
    ST_PENDING = 0,
    ST_REACHED = 1,        /* tracked to t = t_end */
    ST_DIVERGED = 2,       /* ||z||_inf > R_inf during tracking */
    ST_FAIL_MINSTEP = 3,   /* step size underflow away from t = 1 */
    ST_FAIL_MAXSTEPS = 4,
    ST_FAIL_NONFINITE = 5,
    ST_STALLED = 6         /* step size underflow with t >= t_stall (near 1) */
};

typedef struct {
    int32_t kind;
    int32_t n;        /* unknowns */
    int32_t N;        /* ring size (SYS_XY), n = 2(N-1) */
    int32_t pad;
    const double* J;  /* SYS_XY: N*N row-major, symmetric, zero diagonal */
    const double* a;  /* SYS_SEPARABLE: n coefficients */
    const double* c;  /* SYS_SEPARABLE: n constants */
} oracle_sys;

typedef struct {
    double h0;        /* initial step */
    double hmax;      /* largest step */
    double hmin;      /* smallest step */
    double corr_tol;  /* Newton corrector: ||dz||_inf <= corr_tol (1 + ||z||_inf) */
    double R_inf;     /* divergence radius on ||z||_inf */
    double t_stall;   /* a step-size underflow at t >= t_stall is a stall near t = 1 */
    double t_end;     /* track from 0 to t_end (1 for the full homotopy) */
    int32_t max_corr; /* Newton iterations per step */
    int32_t max_steps;/* accepted + rejected steps */
    int32_t predictor;/* 0 = RK4, 1 = Euler */
    int32_t pad;
} oracle_track_opts;

/* ---------------------------------------------------------------------------
 * Target system P(z) and its Jacobian.
 * ------------------------------------------------------------------------- */

/* Spin coordinates with the gauge theta_N = 0 applied: spin N-1 (0-based) is
 * (x, y) = (1, 0). */
static cplx spin_x(const oracle_sys* s, const cplx* z, int j)
{
    int m = s->N - 1;
    return j < m ? z[j] : 1.0;
}
static cplx spin_y(const oracle_sys* s, const cplx* z, int j)
{
    int m = s->N - 1;
    return j < m ? z[m + j] : 0.0;
}

static void eval_P(const oracle_sys* s, const cplx* z, cplx* F)
{
    if (s->kind == SYS_SEPARABLE) {
        for (int k = 0; k < s->n; ++k) F[k] = s->a[k] * z[k] * z[k] - s->c[k];
        return;
    }
    int N = s->N, m = N - 1;
    for (int k = 0; k < m; ++k) {
        cplx xk = z[k], yk = z[m + k], acc = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == k) continue;
            acc += s->J[k * N + j] * (yk * spin_x(s, z, j) - xk * spin_y(s, z, j));
        }
        F[k] = acc;
        F[m + k] = xk * xk + yk * yk - 1.0;
    }
}

/* Jacobian dP/dz, row-major n x n. */
static void eval_Pz(const oracle_sys* s, const cplx* z, cplx* A)
{
    int n = s->n;
    for (int i = 0; i < n * n; ++i) A[i] = 0.0;
    if (s->kind == SYS_SEPARABLE) {
        for (int k = 0; k < n; ++k) A[k * n + k] = 2.0 * s->a[k] * z[k];
        return;
    }
    int N = s->N, m = N - 1;
    for (int k = 0; k < m; ++k) {
        cplx xk = z[k], yk = z[m + k];
        cplx sum_Jx = 0.0, sum_Jy = 0.0;
        for (int j = 0; j < N; ++j) {
            if (j == k) continue;
            double Jkj = s->J[k * N + j];
            sum_Jx += Jkj * spin_x(s, z, j);
            sum_Jy += Jkj * spin_y(s, z, j);
            if (j < m) {
                A[k * n + j] = Jkj * yk;          /* dF_k/dx_j = J_kj y_k */
                A[k * n + m + j] = -Jkj * xk;     /* dF_k/dy_j = -J_kj x_k */
            }
        }
        A[k * n + k] = -sum_Jy;                   /* dF_k/dx_k = -sum_j J_kj y_j */
        A[k * n + m + k] = sum_Jx;                /* dF_k/dy_k =  sum_j J_kj x_j */
        A[(m + k) * n + k] = 2.0 * xk;
        A[(m + k) * n + m + k] = 2.0 * yk;
    }
}

/* ---------------------------------------------------------------------------
 * Homotopy H(z,t) = gamma (1-t) Q(z) + t P(z),   Q_k = z_k^2 - 1.
 * ------------------------------------------------------------------------- */

static void eval_H(const oracle_sys* s, cplx g, const cplx* z, double t, cplx* H)
{
    int n = s->n;
    cplx F[ORACLE_NMAX];
    eval_P(s, z, F);
    for (int k = 0; k < n; ++k) H[k] = g * (1.0 - t) * (z[k] * z[k] - 1.0) + t * F[k];
}

/* dH/dt = P(z) - gamma Q(z) */
static void eval_Ht(const oracle_sys* s, cplx g, const cplx* z, cplx* Ht)
{
    int n = s->n;
    cplx F[ORACLE_NMAX];
    eval_P(s, z, F);
    for (int k = 0; k < n; ++k) Ht[k] = F[k] - g * (z[k] * z[k] - 1.0);
}

/* dH/dz = gamma (1-t) diag(2 z) + t P_z */
static void eval_Hz(const oracle_sys* s, cplx g, const cplx* z, double t, cplx* A)
{
    int n = s->n;
    eval_Pz(s, z, A);
    for (int i = 0; i < n * n; ++i) A[i] *= t;
    for (int k = 0; k < n; ++k) A[k * n + k] += g * (1.0 - t) * 2.0 * z[k];
}

/* ---------------------------------------------------------------------------
 * Dense linear solve A x = b (A and b are overwritten; x may alias b).
 * Gaussian elimination with partial pivoting on |re| + |im|.
 * Returns 0, or -1 when a pivot is exactly zero.
 * ------------------------------------------------------------------------- */
static double abs1(cplx v) { return fabs(creal(v)) + fabs(cimag(v)); }

static int lu_solve(int n, cplx* A, cplx* b, cplx* x)
{
    for (int k = 0; k < n; ++k) {
        int p = k;
        double best = abs1(A[k * n + k]);
        for (int i = k + 1; i < n; ++i) {
            double v = abs1(A[i * n + k]);
            if (v > best) { best = v; p = i; }
        }
        if (!(best > 0.0)) return -1;
        if (p != k) {
            for (int j = 0; j < n; ++j) {
                cplx tmp = A[k * n + j]; A[k * n + j] = A[p * n + j]; A[p * n + j] = tmp;
            }
            cplx tb = b[k]; b[k] = b[p]; b[p] = tb;
        }
        for (int i = k + 1; i < n; ++i) {
            cplx l = A[i * n + k] / A[k * n + k];
            if (l == 0.0) continue;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= l * A[k * n + j];
            b[i] -= l * b[k];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        cplx acc = b[i];
        for (int j = i + 1; j < n; ++j) acc -= A[i * n + j] * x[j];
        x[i] = acc / A[i * n + i];
    }
    return 0;
}

static double norm_inf(int n, const cplx* v)
{
    double r = 0.0;
    for (int k = 0; k < n; ++k) {
        double a = cabs(v[k]);
        if (a > r || a != a) r = a;  /* a NaN propagates */
    }
    return r;
}

static int all_finite(int n, const cplx* v)
{
    for (int k = 0; k < n; ++k)
        if (!isfinite(creal(v[k])) || !isfinite(cimag(v[k]))) return 0;
    return 1;
}

/* Davidenko right-hand side: out = -H_z^{-1} H_t at (z, t). */
static int tangent(const oracle_sys* s, cplx g, const cplx* z, double t, cplx* out)
{
    int n = s->n;
    cplx A[ORACLE_NMAX * ORACLE_NMAX], rhs[ORACLE_NMAX];
    eval_Hz(s, g, z, t, A);
    eval_Ht(s, g, z, rhs);
    for (int k = 0; k < n; ++k) rhs[k] = -rhs[k];
    return lu_solve(n, A, rhs, out);
}

/* ---------------------------------------------------------------------------
 * One path from t = 0 to opts->t_end.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t status, accepted, rejected, pad;
    double t;
} path_result;

static path_result track_one(const oracle_sys* s, cplx g, int64_t path_id,
                             const oracle_track_opts* o, cplx* z)
{
    int n = s->n;
    path_result r = {ST_PENDING, 0, 0, 0, 0.0};
    for (int k = 0; k < n; ++k) z[k] = ((path_id >> k) & 1) ? -1.0 : 1.0;

    double t = 0.0, h = o->h0;
    int streak = 0;
    cplx k1[ORACLE_NMAX], k2[ORACLE_NMAX], k3[ORACLE_NMAX], k4[ORACLE_NMAX];
    cplx zs[ORACLE_NMAX], zp[ORACLE_NMAX], d[ORACLE_NMAX];
    cplx A[ORACLE_NMAX * ORACLE_NMAX], rhs[ORACLE_NMAX];

    while (t < o->t_end) {
        if (r.accepted + r.rejected >= o->max_steps) { r.status = ST_FAIL_MAXSTEPS; break; }
        int last = 0;
        if (h >= o->t_end - t) { h = o->t_end - t; last = 1; }
        double t1 = last ? o->t_end : t + h;

        /* predictor */
        int ok = tangent(s, g, z, t, k1) == 0;
        if (ok && o->predictor == 0) {
            for (int k = 0; k < n; ++k) zs[k] = z[k] + 0.5 * h * k1[k];
            ok = tangent(s, g, zs, t + 0.5 * h, k2) == 0;
            if (ok) {
                for (int k = 0; k < n; ++k) zs[k] = z[k] + 0.5 * h * k2[k];
                ok = tangent(s, g, zs, t + 0.5 * h, k3) == 0;
            }
            if (ok) {
                for (int k = 0; k < n; ++k) zs[k] = z[k] + h * k3[k];
                ok = tangent(s, g, zs, t1, k4) == 0;
            }
            if (ok)
                for (int k = 0; k < n; ++k)
                    zp[k] = z[k] + (h / 6.0) * (k1[k] + 2.0 * k2[k] + 2.0 * k3[k] + k4[k]);
        } else if (ok) {
            for (int k = 0; k < n; ++k) zp[k] = z[k] + h * k1[k];
        }

        /* Newton corrector at t1: converge to the tolerance, each iteration
         * after the first at least halving the update. */
        int converged = 0;
        double prev = INFINITY;
        for (int it = 0; ok && it < o->max_corr; ++it) {
            eval_Hz(s, g, zp, t1, A);
            eval_H(s, g, zp, t1, rhs);
            for (int k = 0; k < n; ++k) rhs[k] = -rhs[k];
            if (lu_solve(n, A, rhs, d) != 0) { ok = 0; break; }
            for (int k = 0; k < n; ++k) zp[k] += d[k];
            double nd = norm_inf(n, d);
            if (!(nd == nd)) { ok = 0; break; }
            if (it > 0 && nd > 0.5 * prev) { ok = 0; break; }
            prev = nd;
            if (nd <= o->corr_tol * (1.0 + norm_inf(n, zp))) { converged = 1; break; }
        }
        if (ok && converged && !all_finite(n, zp)) {
            r.status = ST_FAIL_NONFINITE;
            break;
        }

        if (ok && converged) {
            memcpy(z, zp, sizeof(cplx) * n);
            t = t1;
            r.accepted++;
            if (++streak == 3) { h = fmin(2.0 * h, o->hmax); streak = 0; }
            if (norm_inf(n, z) > o->R_inf) { r.status = ST_DIVERGED; break; }
        } else {
            r.rejected++;
            streak = 0;
            h *= 0.5;
            if (h < o->hmin) {
                r.status = (t >= o->t_stall) ? ST_STALLED : ST_FAIL_MINSTEP;
                break;
            }
        }
    }
    if (r.status == ST_PENDING) r.status = ST_REACHED;
    r.t = t;
    return r;
}

/* ---------------------------------------------------------------------------
 * Newton refinement on P at t = 1: z <- z - P_z^{-1} P(z), at most max_iter
 * iterations; stops when ||dz||_inf <= tol (1 + ||z||_inf), or before
 * applying an update that is larger than the previous one.
 * ------------------------------------------------------------------------- */
static int refine_one(const oracle_sys* s, cplx* z, int max_iter, double tol, double* last_step)
{
    int n = s->n, it;
    cplx A[ORACLE_NMAX * ORACLE_NMAX], rhs[ORACLE_NMAX], d[ORACLE_NMAX];
    double prev = INFINITY;
    *last_step = INFINITY;
    for (it = 0; it < max_iter; ++it) {
        eval_Pz(s, z, A);
        eval_P(s, z, rhs);
        for (int k = 0; k < n; ++k) rhs[k] = -rhs[k];
        if (lu_solve(n, A, rhs, d) != 0) break;
        double nd = norm_inf(n, d);
        if (!(nd == nd) || (it > 0 && nd > prev)) break;
        for (int k = 0; k < n; ++k) z[k] += d[k];
        prev = nd;
        *last_step = nd;
        if (nd <= tol * (1.0 + norm_inf(n, z))) { ++it; break; }
    }
    return it;
}

/* ---------------------------------------------------------------------------
 * Thread pool over path ids (dynamic chunks).
 * ------------------------------------------------------------------------- */
typedef struct {
    const oracle_sys* s;
    cplx g;
    const int64_t* ids;
    int64_t count;
    const oracle_track_opts* o;
    double* z_out;      /* count x n x 2 */
    double* t_out;
    int32_t* status;
    int32_t* accepted;
    int32_t* rejected;
    _Atomic int64_t next;
} track_job;

static void* track_worker(void* arg)
{
    track_job* jb = (track_job*)arg;
    int n = jb->s->n;
    cplx z[ORACLE_NMAX];
    for (;;) {
        int64_t begin = atomic_fetch_add(&jb->next, 16);
        if (begin >= jb->count) break;
        int64_t end = begin + 16 < jb->count ? begin + 16 : jb->count;
        for (int64_t i = begin; i < end; ++i) {
            int64_t pid = jb->ids ? jb->ids[i] : i;
            path_result r = track_one(jb->s, jb->g, pid, jb->o, z);
            for (int k = 0; k < n; ++k) {
                jb->z_out[(i * n + k) * 2] = creal(z[k]);
                jb->z_out[(i * n + k) * 2 + 1] = cimag(z[k]);
            }
            if (jb->t_out) jb->t_out[i] = r.t;
            jb->status[i] = r.status;
            if (jb->accepted) jb->accepted[i] = r.accepted;
            if (jb->rejected) jb->rejected[i] = r.rejected;
        }
    }
    return NULL;
}

static int check_sys(const oracle_sys* s)
{
    if (!s || s->n < 1 || s->n > ORACLE_NMAX) return -1;
    if (s->kind == SYS_XY && (s->N < 2 || s->n != 2 * (s->N - 1) || !s->J)) return -1;
    if (s->kind == SYS_SEPARABLE && (!s->a || !s->c)) return -1;
    if (s->kind != SYS_XY && s->kind != SYS_SEPARABLE) return -1;
    return 0;
}

/* Track the paths `ids` (or 0..count-1 when ids is NULL).  Outputs are indexed
 * by position in `ids`.  z_out holds count x n interleaved (re, im) pairs. */
int oracle_track(const oracle_sys* s, double gamma_re, double gamma_im,
                 const int64_t* ids, int64_t count, const oracle_track_opts* o,
                 double* z_out, double* t_out, int32_t* status,
                 int32_t* accepted, int32_t* rejected, int nthreads)
{
    if (check_sys(s) || !o || count < 0 || !z_out || !status) return -1;
    if (count == 0) return 0;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    track_job jb = {s, gamma_re + I * gamma_im, ids, count, o, z_out, t_out, status,
                    accepted, rejected, 0};
    pthread_t th[256];
    int started = 0;
    for (int i = 1; i < nthreads; ++i)
        if (pthread_create(&th[started], NULL, track_worker, &jb) == 0) ++started;
    track_worker(&jb);
    for (int i = 0; i < started; ++i) pthread_join(th[i], NULL);
    return 0;
}

/* Refine `count` endpoints in place (interleaved re/im, count x n). */
int oracle_refine(const oracle_sys* s, double* z_io, int64_t count, int max_iter, double tol,
                  int32_t* iters, double* last_step)
{
    if (check_sys(s) || count < 0 || !z_io) return -1;
    int n = s->n;
    cplx z[ORACLE_NMAX];
    for (int64_t i = 0; i < count; ++i) {
        for (int k = 0; k < n; ++k) z[k] = z_io[(i * n + k) * 2] + I * z_io[(i * n + k) * 2 + 1];
        double ls;
        int it = refine_one(s, z, max_iter, tol, &ls);
        for (int k = 0; k < n; ++k) {
            z_io[(i * n + k) * 2] = creal(z[k]);
            z_io[(i * n + k) * 2 + 1] = cimag(z[k]);
        }
        if (iters) iters[i] = it;
        if (last_step) last_step[i] = ls;
    }
    return 0;
}

/* Plain evaluations for tests: P(z), P_z(z), H(z,t), H_t, H_z (interleaved). */
static void load_z(int n, const double* zi, cplx* z)
{
    for (int k = 0; k < n; ++k) z[k] = zi[2 * k] + I * zi[2 * k + 1];
}
static void store_v(int n, const cplx* v, double* out)
{
    for (int k = 0; k < n; ++k) { out[2 * k] = creal(v[k]); out[2 * k + 1] = cimag(v[k]); }
}

int oracle_eval_P(const oracle_sys* s, const double* z_in, double* F_out)
{
    if (check_sys(s)) return -1;
    cplx z[ORACLE_NMAX], F[ORACLE_NMAX];
    load_z(s->n, z_in, z);
    eval_P(s, z, F);
    store_v(s->n, F, F_out);
    return 0;
}

int oracle_eval_Pz(const oracle_sys* s, const double* z_in, double* A_out)
{
    if (check_sys(s)) return -1;
    cplx z[ORACLE_NMAX], A[ORACLE_NMAX * ORACLE_NMAX];
    load_z(s->n, z_in, z);
    eval_Pz(s, z, A);
    store_v(s->n * s->n, A, A_out);
    return 0;
}

int oracle_eval_H(const oracle_sys* s, double gre, double gim, const double* z_in, double t,
                  double* H_out, double* Ht_out, double* Hz_out)
{
    if (check_sys(s)) return -1;
    cplx z[ORACLE_NMAX], v[ORACLE_NMAX], A[ORACLE_NMAX * ORACLE_NMAX];
    cplx g = gre + I * gim;
    load_z(s->n, z_in, z);
    if (H_out) { eval_H(s, g, z, t, v); store_v(s->n, v, H_out); }
    if (Ht_out) { eval_Ht(s, g, z, v); store_v(s->n, v, Ht_out); }
    if (Hz_out) { eval_Hz(s, g, z, t, A); store_v(s->n * s->n, A, Hz_out); }
    return 0;
}

/* Dense solve exposed for tests: A (n x n interleaved) and b (n) are copied. */
int oracle_solve(int n, const double* A_in, const double* b_in, double* x_out)
{
    if (n < 1 || n > ORACLE_NMAX) return -1;
    cplx A[ORACLE_NMAX * ORACLE_NMAX], b[ORACLE_NMAX], x[ORACLE_NMAX];
    load_z(n * n, A_in, A);
    load_z(n, b_in, b);
    int rc = lu_solve(n, A, b, x);
    store_v(n, x, x_out);
    return rc;
}

int oracle_nmax(void) { return ORACLE_NMAX; }
