// path.hpp -- one path's state and one predictor-corrector step (per lane;
// also compiles for the host).
#pragma once
#include "common.hpp"
#include "xy_lane.hpp"

namespace nphc {

// The path's current point z and the RK4 accumulator w live outside the
// register file: component i (0..2M-1, ordering x_0..x_{M-1}, y_0..y_{M-1})
// of z is at base[i * stride], of w at base[(2M + i) * stride].  On the
// device base points into LDS with stride 64 (one slot per lane, so a
// wave's accesses to one component are consecutive); the register file is
// left to the linear solve.
template <class T, int M>
struct PathStore {
    cx<T>* base;
    int stride;
    NPHC_HD cx<T> z(int i) const { return base[i * stride]; }
    NPHC_HD void set_z(int i, cx<T> v) const { base[i * stride] = v; }
    NPHC_HD cx<T> w(int i) const { return base[(2 * M + i) * stride]; }
    NPHC_HD void set_w(int i, cx<T> v) const { base[(2 * M + i) * stride] = v; }
    NPHC_HD void load_z(Point<T, M>& p) const
    {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            p.x[k] = z(k);
            p.y[k] = z(M + k);
        }
    }
    NPHC_HD void store_z(const Point<T, M>& p) const
    {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            set_z(k, p.x[k]);
            set_z(M + k, p.y[k]);
        }
    }
};

template <class T, int M>
struct LanePath {
    PathStore<T, M> st;
    double t, h;
    double h_acc;       // step size of the last accepted step
    double znorm;       // ||z|| after the last accepted step
    int32_t streak, acc, rej, status, solves, rej_run;
};

template <class T, int M>
NPHC_HD void start_point(int64_t pid, Point<T, M>& z)
{
#pragma unroll
    for (int k = 0; k < M; ++k) {
        z.x[k] = {((pid >> k) & 1) ? T(-1) : T(1), T(0)};
        z.y[k] = {((pid >> (M + k)) & 1) ? T(-1) : T(1), T(0)};
    }
}

// One predictor-corrector step of one lane's path (paper, section "NPHC
// method": predictor, then Newton's corrector; step control as documented in
// nphc_track_paths).  Sets S.status when the path ends.
template <class T, int M>
NPHC_HD void path_step(const Couplings<T, M>& C, cx<T> gamma, const TrackOptsDev& o,
                       LanePath<T, M>& S)
{
    const bool last = S.h >= o.t_end - S.t;
    const double hh = last ? (o.t_end - S.t) : S.h;
    const double t1 = last ? o.t_end : S.t + hh;
    const int nst = o.predictor == 0 ? 4 : 1;
    const PathStore<T, M>& st = S.st;

    Point<T, M> zq;        // where the next linear solve is evaluated; after the
    st.load_z(zq);         // predictor, the point being corrected
    bool ok = true, conv = false, bad = false, too_far = false;
    T prev = T(0), d1 = T(0), wn1 = T(1);

    for (int s = 0; s < nst + o.max_corr; ++s) {
        const bool pred = s < nst;
        const bool want = pred ? ok : (ok && !conv && !bad);
        if (!want) continue;
        // stage times of the classical RK4: t, t + h/2, t + h/2, t + h
        const double tq = !pred ? t1 : (s == 0 ? S.t : (s == 3 ? t1 : S.t + 0.5 * hh));
        Point<T, M> d;
        const bool sok = solve_step<T, M>(C, gamma, T(tq), T(1.0 - tq), !pred, zq, d);
        S.solves += 1;
        if (pred) {
            ok = ok && sok;
            const T ws = (s == 0 || s == 3) ? T(1) : T(2);           // RK4 weights 1 2 2 1
            const bool final_stage = (s == nst - 1);
            const T f = T(nst == 4 ? hh / 6.0 : hh);
            const T ch = T((s == 2 ? 1.0 : 0.5) * hh);               // next stage offset
#pragma unroll
            for (int i = 0; i < 2 * M; ++i) {
                const cx<T> di = i < M ? d.x[i] : d.y[i - M];
                cx<T> wi = (s == 0) ? di : axpy(ws, di, st.w(i));
                const cx<T> zi = st.z(i);
                cx<T> next;
                if (final_stage) {
                    wi = axpy(f, wi, zi);                              // predicted point
                    next = wi;
                } else {
                    st.set_w(i, wi);
                    next = axpy(ch, di, zi);
                }
                if (i < M) zq.x[i] = next; else zq.y[i - M] = next;
            }
        } else {
            if (!sok) {
                bad = true;
            } else {
                const T nd = norm_inf<T, M>(d);
                // path-jumping guard: the first correction measures the
                // predictor's error; a large one means the step is too long
                if (s == nst) {
                    d1 = nd;
                    wn1 = T(1) + norm_inf<T, M>(zq);
                    if (o.pred_tol > 0.0 && nd > T(o.pred_tol) * wn1) {
                        bad = true;
                        too_far = true;
                    }
                }
#pragma unroll
                for (int i = 0; i < M; ++i) {
                    zq.x[i] = zq.x[i] + d.x[i];
                    zq.y[i] = zq.y[i] + d.y[i];
                }
                if (s > nst && nd > T(0.5) * prev) bad = true;
                prev = nd;
                if (!bad && nd <= T(o.corr_tol) * (T(1) + norm_inf<T, M>(zq))) conv = true;
            }
        }
    }

    const T wn = norm_inf<T, M>(zq);
    const bool finite = (wn - wn == T(0));
    if (ok && conv && !bad && !finite) {
        S.status = NPHC_PATH_FAIL_NONFINITE;
        return;
    }
    if (ok && conv && !bad) {
        st.store_z(zq);
        S.t = t1;
        S.acc += 1;
        S.h_acc = hh;
        S.rej_run = 0;
        if (o.step_ctrl == 1 && o.pred_tol > 0.0) {
            // predictor-error control: the RK4 local error scales as h^5
            const double e = double(d1) / (o.pred_tol * double(wn1));
            const double fct = e > 1e-12 ? fmin(2.0, fmax(0.5, 0.8 * pow(e, -0.2))) : 2.0;
            S.h = fmin(fct * hh, o.hmax);
        } else if (++S.streak == 3) {
            S.h = fmin(2.0 * hh, o.hmax);
            S.streak = 0;
        } else {
            S.h = hh;
        }
        // end zone: while ||z|| keeps growing the path is heading to infinity;
        // step a fixed fraction of the remaining distance instead of trying to
        // finish at t_end
        if (S.t >= o.t_endzone && o.grow_cap > 0.0 && double(wn) > o.grow_ratio * S.znorm)
            S.h = fmin(S.h, o.grow_cap * (o.t_end - S.t));
        S.znorm = double(wn);
        if (double(wn) > o.R_inf) S.status = NPHC_PATH_DIVERGED;
        else if (S.t >= o.t_end) S.status = NPHC_PATH_REACHED;
        else if (o.handoff_norm > 0.0 && double(wn) > o.handoff_norm) S.status = NPHC_PATH_HANDOFF;
    } else {
        S.rej += 1;
        S.rej_run += 1;
        S.streak = 0;
        if (too_far && o.step_ctrl == 1) {
            const double e = double(d1) / (o.pred_tol * double(wn1));
            S.h = hh * fmin(0.5, fmax(0.125, 0.8 * pow(e, -0.2)));
        } else {
            S.h = 0.5 * hh;
        }
        // near t = 1 a step far below the remaining distance 1 - t means the
        // path is heading to infinity or to a singular endpoint
        const bool collapse = S.h < o.hmin ||
                              (S.t >= o.t_endzone && S.h < o.hmin_rel * (o.t_end - S.t) &&
                               S.znorm > o.collapse_norm);
        if (o.handoff_rejects > 0 && S.rej_run >= o.handoff_rejects) {
            S.status = NPHC_PATH_HANDOFF;
        } else if (collapse) {
            S.status = o.handoff_rejects > 0 ? NPHC_PATH_HANDOFF
                       : (S.t >= o.t_stall) ? NPHC_PATH_STALLED : NPHC_PATH_FAIL_MINSTEP;
        }
    }
    if (S.status == NPHC_PATH_PENDING && o.handoff_steps > 0 && S.acc + S.rej >= o.handoff_steps)
        S.status = NPHC_PATH_HANDOFF;
    if (S.status == NPHC_PATH_HANDOFF) S.h = S.h_acc;  // the continuation restarts from here
    if (S.status == NPHC_PATH_PENDING && S.acc + S.rej >= o.max_steps)
        S.status = NPHC_PATH_FAIL_MAXSTEPS;
}

}  // namespace nphc
