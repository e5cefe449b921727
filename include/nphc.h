/*
 * nphc.h -- C ABI of libnphc.so: numerical polynomial homotopy continuation
 * (NPHC) for the stationary points of the power-law XY ring on AMD MI355X
 * (gfx950).  Method: D. Mehta, "Finding all the stationary points of a
 * potential energy landscape via numerical polynomial homotopy continuation
 * method" (arXiv:1104.5497).
 *
 * Problem (paper, section "A First Application", eq. (1)): for a ring of N
 * spins with symmetric couplings J (J_ii = 0) and the gauge theta_N = 0, the
 * stationary points of V = sum_{i<k} J_ik (1 - cos(theta_i - theta_k)) are the
 * real solutions of the 2m = 2(N-1) quadratics
 *     F_k     = sum_{j != k} J_kj (y_k x_j - x_k y_j) = 0,   (x_N, y_N) = (1, 0)
 *     F_{m+k} = x_k^2 + y_k^2 - 1                     = 0,   k = 1..m
 * in z = (x_1..x_m, y_1..y_m), x = cos(theta), y = sin(theta).
 *
 * Method (paper, section "Numerical Polynomial Homotopy Continuation
 * Method"): the total-degree homotopy H(z,t) = gamma (1-t) Q(z) + t F(z) with
 * Q_k = z_k^2 - 1 has 2^(2m) = 4^(N-1) start solutions z_k = +-1 (the
 * classical Bezout number); every path is tracked from t = 0 to t = 1 by a
 * predictor and Newton's corrector.  Item p of a system starts at
 * z_k = 1 - 2 * bit_k(p), k = 0..2m-1.
 *
 * Conventions shared by every entry point:
 *  - "device" pointers are HIP device memory on the current device; "host"
 *    pointers are ordinary host memory read during the call only.
 *  - All work is enqueued asynchronously on `stream`; no entry point waits
 *    for the device or allocates memory.  The caller owns every buffer.
 *  - Per-item arrays are indexed by the batch-global item id
 *    g = path_off[b] + p (system b, local path p); `item_stride` is the
 *    total number of items, path_off[num_systems].
 *  - Complex unknowns are stored as planes: for unknown k (k < 2 m_max,
 *    ordering x_1..x_m, y_1..y_m of each item's own system), the real parts
 *    are at z[(2k) * item_stride + g] and the imaginary parts at
 *    z[(2k+1) * item_stride + g] (float64).
 *  - An id list `ids` (device, int64, strictly increasing item ids) selects
 *    items; ids == NULL means all items.  `count` is its length, and when
 *    `count_dev` (device int64) is non-NULL the length is min(count,
 *    *count_dev), read on the device (so lists produced by nphc_select can be
 *    chained without a host round trip).
 *  - Return value: NPHC_OK, or a negative NPHC_E* code; per-path outcomes are
 *    never reported through the return value.  Argument errors are detected
 *    before anything is enqueued.
 */
#ifndef NPHC_H
#define NPHC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NPHC_MAX_N 13        /* largest ring size (m = 12 free spins, 24 unknowns) */
#define NPHC_BATCH_MAX_N 9   /* largest ring size when a batch mixes ring sizes */

/* return codes */
#define NPHC_OK 0
#define NPHC_EINVAL (-1)       /* null or inconsistent argument */
#define NPHC_EUNSUPPORTED (-2) /* ring size or precision not built */
#define NPHC_EHIP (-3)         /* a HIP call or kernel launch failed */
#define NPHC_EWORKSPACE (-4)   /* workspace too small or misaligned */

/* arithmetic of the path tracker */
#define NPHC_FP64 0
#define NPHC_FP32 1

/* per-item path outcomes written by nphc_track_paths */
#define NPHC_PATH_PENDING 0
#define NPHC_PATH_REACHED 1        /* tracked to t = t_end */
#define NPHC_PATH_DIVERGED 2       /* ||z||_inf exceeded R_inf */
#define NPHC_PATH_FAIL_MINSTEP 3   /* step size fell below h_min before t_stall */
#define NPHC_PATH_FAIL_MAXSTEPS 4
#define NPHC_PATH_FAIL_NONFINITE 5
#define NPHC_PATH_STALLED 6        /* step size fell below h_min at t >= t_stall */
#define NPHC_PATH_HANDOFF 7        /* stopped for a float64 continuation (z, t, h saved) */

/* per-item endpoint classes written by nphc_refine_certify / nphc_mark_duplicates */
#define NPHC_END_NONSINGULAR 10
#define NPHC_END_SINGULAR 11
#define NPHC_END_DIVERGED 12
#define NPHC_END_FAIL 13
#define NPHC_END_DUPLICATE 14

/*
 * A batch of rings.  Systems must be sorted by nondecreasing N.  A batch
 * with one ring size may use any 2 <= N <= NPHC_MAX_N; a batch that mixes
 * ring sizes needs N <= NPHC_BATCH_MAX_N.
 */
typedef struct nphc_batch {
    int32_t num_systems;
    int32_t pad;
    const int32_t* N_host;         /* host [num_systems] */
    const int64_t* path_off_host;  /* host [num_systems+1], prefix sums of 4^(N_b-1) */
    const int32_t* N;              /* device copy of N_host */
    const int64_t* path_off;       /* device copy of path_off_host */
    const double* J;               /* device, system b's N_b x N_b row-major couplings at J + J_off[b] */
    const int64_t* J_off;          /* device [num_systems] */
    const double* gamma;           /* device [2*num_systems]: (re, im) of the homotopy constant */
} nphc_batch;

/* Path-tracker settings (the paper leaves them open; defaults from
 * nphc_default_track_opts). */
typedef struct nphc_track_opts {
    double h0;        /* first step in t */
    double hmax;      /* largest step */
    double hmin;      /* smallest step */
    double corr_tol;  /* Newton corrector converged: ||dz|| <= corr_tol (1 + ||z||) */
    double R_inf;     /* the path diverges when ||z||_inf > R_inf */
    double t_stall;   /* a step-size underflow at t >= t_stall is a stall near t = 1 */
    double t_end;     /* track t from 0 to t_end (1 for the whole homotopy) */
    int32_t max_corr; /* Newton iterations per step (default 2 for float32, 3 for float64) */
    int32_t max_steps;/* accepted + rejected steps */
    int32_t predictor;/* 0: classical RK4, 1: Euler (the paper's predictor) */
    int32_t resume;   /* 1: continue each selected path from its saved z, t, h and step counts */
    double handoff_norm;     /* > 0: stop a path with NPHC_PATH_HANDOFF once ||z||_inf > handoff_norm */
    int32_t handoff_rejects; /* > 0: stop with NPHC_PATH_HANDOFF after this many rejected steps
                                in a row, or when the step size collapses */
    int32_t pad;
    /* end zone t >= t_endzone (near t = 1):
     *  - after an accepted step that grew ||z||_inf by more than grow_ratio,
     *    the next step is at most grow_cap (1 - t) (the path is heading to
     *    infinity: no attempt to finish at t_end);
     *  - a step below hmin_rel (1 - t) while ||z||_inf > collapse_norm is a
     *    collapse, like a step below hmin.
     * grow_cap = 0 or hmin_rel = 0 disables the rule. */
    double t_endzone;
    double hmin_rel;
    double collapse_norm;
    double grow_ratio;
    double grow_cap;
    int32_t grid_blocks;     /* persistent grid size in 64-lane workgroups (0: one per resident wave slot) */
    int32_t handoff_steps;   /* > 0: stop with NPHC_PATH_HANDOFF after this many steps (bounds the
                                float32 work of paths that creep through ill-conditioned stretches) */
    double pred_tol;         /* > 0: reject a step whose first Newton correction exceeds
                                pred_tol (1 + ||z||_inf) (the predictor was too far off: guards
                                against jumping to a neighbouring path) */
    int32_t step_ctrl;       /* 0: double h after three accepted steps, halve on rejection;
                                1: scale h by (pred_tol / first correction)^(1/5) */
    int32_t lanes_per_path;  /* 1: one path per lane (throughput); 16: one path per group of 16
                                lanes sharing each linear solve (lower latency per step, for the
                                few long paths left at the end of a launch; float64 only) */
    int32_t drain_steps;     /* > 0: once the launch's work queue is empty, a path still in flight
                                stops with NPHC_PATH_HANDOFF after this many more steps (its state
                                saved), so that the launch does not wait for its longest paths */
    int32_t pad3;
} nphc_track_opts;

/* Endpoint refinement and certification settings. */
typedef struct nphc_cert_opts {
    int32_t max_iter; /* Newton iterations on F at t = 1 */
    int32_t lanes_per_item; /* 1 (default; 0 means 1), 4, 8 or 16 lanes refine one endpoint:
                               Newton runs on every lane of the group and the certificate's
                               2m + 1 solves are split over them (lower latency for short
                               lists, more total work); results equal to rounding */
    double tol;       /* Newton stops when ||dz|| <= tol (1 + ||z||) */
    double res_tol;   /* NONSINGULAR needs ||F||_inf < res_tol * max(1, ||z||_inf^2) ... */
    double cond_max;  /* ... and cond(F_z) < cond_max; SINGULAR: ||F|| small, cond >= cond_max */
    double sing_res;  /* SINGULAR needs ||F||_inf < sing_res * max(1, ||z||_inf^2) */
    double div_norm;  /* a path that stopped early beyond this norm went to infinity */
    double real_tol;  /* real root: max_k |Im z_k| <= real_tol (the paper's Delta_R) */
} nphc_cert_opts;

/* Classification settings. */
typedef struct nphc_class_opts {
    double eig_rel;   /* degenerate / zero eigenvalue: |lambda| <= eig_rel * max(1, max|lambda|) */
    int32_t jacobi_sweeps;
    int32_t pad;
} nphc_class_opts;

void nphc_default_track_opts(int precision, nphc_track_opts* o);
void nphc_default_cert_opts(nphc_cert_opts* o);
void nphc_default_class_opts(nphc_class_opts* o);

/* Bytes of device workspace nphc_track_paths needs for this batch (256-byte
 * aligned pointer required). */
size_t nphc_track_workspace_size(const nphc_batch* b, int precision);

/*
 * Track the homotopy paths of the selected items (paper, section "NPHC
 * method": predictor-corrector continuation of every start solution).
 * Predictor: classical RK4 (or Euler) on the Davidenko equation
 * dz/dt = -H_z^{-1} H_t; corrector: up to max_corr Newton iterations at the
 * new t, each after the first at least halving the update, the first one
 * bounded by pred_tol; step size doubled after three accepted steps in a row
 * and halved on a rejected step.  One
 * persistent launch per call; each GPU lane tracks one path at a time and
 * takes the next queued item when its path ends.  precision NPHC_FP32 does
 * the linear algebra (Jacobian, tangent, elimination) in complex float32 but
 * keeps the current point in float64 and evaluates the Newton right-hand side
 * -H in float64 (mixed-precision Newton: the corrector converges to the
 * float64 path, not to float32 rounding noise); t and h are float64.  With
 * handoff_rejects > 0 a path whose step size collapses (or
 * that is rejected that many times in a row) stops with NPHC_PATH_HANDOFF and
 * its state is saved; a later call with resume = 1 continues it (normally in
 * float64).
 * Outputs (device, per item, only the selected items are written): z
 * (endpoint, planes as above), t (final t), status (NPHC_PATH_*), accepted
 * and rejected step counts, (if solves is not NULL) the number of linear
 * solves the path took (predictor stages plus corrector iterations), and (if
 * h is not NULL) the step size to continue with.  With resume = 1, z, t, h,
 * accepted, rejected and solves (when given) are also read as the start
 * state; h must then be given.
 */
int nphc_track_paths(const nphc_batch* b, const int64_t* ids, int64_t count,
                     const int64_t* count_dev, int precision, const nphc_track_opts* o,
                     double* z, int64_t item_stride, double* t, int32_t* status,
                     int32_t* accepted, int32_t* rejected, int32_t* solves, double* h,
                     void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Refine and certify the endpoints of the selected items in float64 (paper:
 * solutions are refined "up to the machine precision" and then certified
 * with alpha-theory).  Items whose status is REACHED or STALLED (and, for
 * STALLED/FAIL_MINSTEP/FAIL_MAXSTEPS, whose ||z||_inf <= div_norm) get Newton
 * on F at t = 1 (z updated in place); then
 *   resid = ||F||_inf, cond = ||F_z||_F ||F_z^{-1}||_F,
 *   beta  = ||F_z^{-1} F||_2, alpha = beta * ||F_z^{-1}||_F * B,
 *   B = sqrt(||J~||_F^2 + 4m) / 2 >= sup ||D^2 F(u, v) / 2|| (F is quadratic),
 * and alpha_real is the same alpha evaluated at Re z (the certificate of a
 * real root).  endpoint receives NPHC_END_NONSINGULAR (reached t = t_end,
 * small residual, cond < cond_max), NPHC_END_SINGULAR, NPHC_END_DIVERGED or
 * NPHC_END_FAIL.  Output arrays are per item; unselected items untouched.
 */
int nphc_refine_certify(const nphc_batch* b, const int64_t* ids, int64_t count,
                        const int64_t* count_dev, const nphc_cert_opts* o,
                        double* z, int64_t item_stride, const double* t,
                        const int32_t* status, int32_t* endpoint, double* resid,
                        double* cond, double* beta, double* alpha, double* alpha_real,
                        hipStream_t stream);

/*
 * Path-jump check: among the selected items whose endpoint is
 * NPHC_END_NONSINGULAR, two endpoints of the same system closer than
 * dup_tol in max-norm reached the same root, which a correct tracker never
 * does (one path per isolated nonsingular root).  Both are marked
 * NPHC_END_DUPLICATE.  *num_marked (device int64) receives the number of
 * items marked (it is overwritten, not accumulated).
 * ids (device, sorted, *count_dev entries) lists the candidates, normally
 * every NONSINGULAR item; count is the capacity (an upper bound on
 * *count_dev; candidates beyond it are ignored).  probe_ids == NULL: every
 * pair of candidates is checked.  Otherwise only pairs with a probe (device,
 * sorted, *probe_count_dev entries; e.g. the items just re-tracked) are
 * checked: each probe that is NONSINGULAR against every other candidate of
 * its system; with no probes the call does nothing on the device.
 * The candidates are bucketed in a hash table (expected work linear in their
 * number) held in the caller's workspace: nphc_duplicates_workspace_size(count)
 * bytes, 256-byte aligned.  Batches need fewer than 2^20 systems.
 */
int nphc_mark_duplicates(const nphc_batch* b, const int64_t* ids, int64_t count,
                         const int64_t* count_dev, const int64_t* probe_ids,
                         const int64_t* probe_count_dev, double dup_tol, const double* z,
                         int64_t item_stride, int32_t* endpoint, int64_t* num_marked,
                         void* workspace, size_t ws_bytes, hipStream_t stream);
size_t nphc_duplicates_workspace_size(int64_t count);

/*
 * Ordered compaction: writes, in increasing order, every item id g in
 * [0, num_items) with (1 << code[g]) & mask != 0 to out_ids (device) and
 * their number to *out_count (device int64).  out_ids needs num_items
 * entries.  With a workspace of nphc_select_workspace_size(num_items) bytes
 * (device, 8-byte aligned) the work is spread over many workgroups; with
 * workspace == NULL one workgroup does it.
 */
int nphc_select(const int32_t* code, int64_t num_items, uint64_t mask, int64_t* out_ids,
                int64_t* out_count, void* workspace, size_t ws_bytes, hipStream_t stream);
size_t nphc_select_workspace_size(int64_t num_items);

/*
 * The same compaction over an id list: writes, in list order, every ids[i]
 * (i < count, or i < min(count, *count_dev) when count_dev is non-NULL) with
 * (1 << code[ids[i]]) & mask != 0 to out_ids and their number to *out_count.
 * The pipeline uses it to split a list of handed-off paths into those a
 * continuation finished and those still handed off.  ids, count_dev, out_ids
 * and out_count are device memory; out_ids needs count entries and must not
 * overlap ids.  The workspace is nphc_select_workspace_size(count) bytes (or
 * NULL: one workgroup).  Every ids[i] must be a valid index into code.
 */
int nphc_select_list(const int32_t* code, const int64_t* ids, int64_t count,
                     const int64_t* count_dev, uint64_t mask, int64_t* out_ids,
                     int64_t* out_count, void* workspace, size_t ws_bytes, hipStream_t stream);

/*
 * Real filter and classification of the listed items (paper: a solution is
 * real when every |Im z_k| <= Delta_R; theta_k = atan2(y_k, x_k) in
 * (-pi, pi]; the stationary point is classified by the number of negative
 * Hessian eigenvalues).  For list position i (item ids[i]):
 *   is_real[i] = endpoint is NONSINGULAR, max|Im z| <= real_tol and the real
 *                projection passes the alpha-test (alpha_real < alpha_0 with
 *                alpha_0 = (13 - 3 sqrt(17)) / 4);
 * and, when is_real[i]: theta (m planes of stride `count`), the energy
 * V = sum_{i<k} J_ik (1 - cos(theta_i - theta_k)), the Hessian
 * d2V/dtheta_i dtheta_k (i, k < N) eigenvalues (ascending, m planes of stride
 * `count`, by cyclic Jacobi rotations), index = #{lambda < -tau} and
 * degenerate = (min |lambda| <= tau), tau = eig_rel * max(1, max|lambda|).
 */
int nphc_classify(const nphc_batch* b, const int64_t* ids, int64_t count, const int64_t* count_dev,
                  const nphc_class_opts* o, double real_tol, const double* z, int64_t item_stride,
                  const int32_t* endpoint, const double* alpha_real, int32_t* is_real,
                  double* theta, double* energy, int32_t* index, double* eig, int32_t* degenerate,
                  hipStream_t stream);

/*
 * Adjoint of certified real stationary points with respect to the couplings
 * (implicit-function theorem at a nonsingular root z(J):
 * dz/dJ_ab = -F_z^{-1} dF/dJ_ab at the root).  For list position i (item ids[i], a real
 * root stored in z) and the objective L = sum_i w_V[i] V(z_i) +
 * sum_i <g_z[i], z_i>, the kernel solves F_z^T lambda = dL/dz (float64) and
 * accumulates dL/dJ_ab = sum_i [w_V[i] (1 - x_a x_b - y_a y_b) - lambda^T dF/dJ_ab]
 * into dLdJ (device, per system N_b x N_b at J_off[b], symmetric, both (a,b)
 * and (b,a) receive the derivative with respect to the coupling J_ab = J_ba;
 * accumulated with atomics, so zero it first).  g_z may be NULL (energy
 * objectives only); when given it holds 2 m_max planes of stride `count`
 * (real parts of dL/dz; imaginary parts are not used since z is real).
 */
int nphc_adjoint(const nphc_batch* b, const int64_t* ids, int64_t count, const int64_t* count_dev,
                 const double* z, int64_t item_stride, const double* w_V, const double* g_z,
                 double* dLdJ, hipStream_t stream);

/* Short description of a return code. */
const char* nphc_strerror(int code);

/* Library version string. */
const char* nphc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NPHC_H */
