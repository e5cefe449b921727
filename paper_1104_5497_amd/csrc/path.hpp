// path.hpp -- one path's state and one predictor-corrector step (per lane;
// also compiles for the host).
#pragma once
#include "common.hpp"
#include "xy_lane.hpp"

namespace nphc {

// Where a lane keeps its path between steps.  Component i (0..2M-1, order
// x_0..x_{M-1}, y_0..y_{M-1}) of each array is at base[i * stride]; on the
// device the arrays live in LDS with stride 64 (one slot per lane, so a
// wave's accesses to one component are consecutive) and the register file is
// left to the linear solve.
//
// A store tells the step how the point being corrected is formed:
//   load_point(p)        the current point, in the solve's type
//   stage_base(i)        base of an intermediate RK4 stage point
//   predict(i, f, w_i)   predicted component z_i + f w_i
//   correct(i, q_i, d_i) corrected component q_i + d_i
//   accept(q)            make the corrected point the current point
//   get(i) / put(i, v)   float64 exchange with the caller's arrays

// Same precision throughout: point and RK4 accumulator in T.
template <class T, int M>
struct PathStore {
    using Solve = T;
    static constexpr bool kWideResidual = false;
    cx<T>* base;
    int stride;
    NPHC_HD cx<T> z(int i) const { return base[i * stride]; }
    NPHC_HD void set_z(int i, cx<T> v) const { base[i * stride] = v; }
    NPHC_HD cx<T> w(int i) const { return base[(2 * M + i) * stride]; }
    NPHC_HD void set_w(int i, cx<T> v) const { base[(2 * M + i) * stride] = v; }

    NPHC_HD void load_point(Point<T, M>& p) const
    {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            p.x[k] = z(k);
            p.y[k] = z(M + k);
        }
    }
    NPHC_HD cx<T> stage_base(int i) const { return z(i); }
    NPHC_HD cx<T> predict(int i, T f, cx<T> wi) const { return axpy(f, wi, z(i)); }
    NPHC_HD cx<T> correct(int, cx<T> qi, cx<T> di) const { return qi + di; }
    NPHC_HD void accept(const Point<T, M>& q) const
    {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            set_z(k, q.x[k]);
            set_z(M + k, q.y[k]);
        }
    }
    NPHC_HD cx<double> get(int i) const { const cx<T> v = z(i); return {double(v.re), double(v.im)}; }
    NPHC_HD void put(int i, cx<double> v) const { set_z(i, {T(v.re), T(v.im)}); }
};

// float32 linear algebra on a float64 point.  The current point z is kept in
// float64; the point being corrected is z + dl with the increment dl in
// float32 (|dl| is one step, so its rounding is far below the tolerances),
// and the Newton right-hand side -H(z + dl) is evaluated in float64 by
// wide_residual, then handed to the float32 solve.  The Jacobian, the tangent
// and the elimination stay float32.  Without the wide residual a float32
// corrector stalls once |z| is a few tens: the terms of F_k are of size
// |z|^2 and their rounding swamps a relative tolerance.
// Arrays per lane: z (2M complex float64), the RK4 accumulator w and dl
// (2M complex float32 each).  The accumulator is idle while correcting and
// holds the float64-evaluated right-hand side (rounded) meanwhile.
template <int M>
struct MixedStore {
    using Solve = float;
    static constexpr bool kWideResidual = true;
    cx<double>* zb;
    cx<float>* wb;
    cx<float>* db;
    int stride;
    NPHC_HD cx<double> z(int i) const { return zb[i * stride]; }
    NPHC_HD void set_z(int i, cx<double> v) const { zb[i * stride] = v; }
    NPHC_HD cx<float> w(int i) const { return wb[i * stride]; }
    NPHC_HD void set_w(int i, cx<float> v) const { wb[i * stride] = v; }
    NPHC_HD cx<float> dl(int i) const { return db[i * stride]; }
    NPHC_HD void set_dl(int i, cx<float> v) const { db[i * stride] = v; }

    static NPHC_HD cx<float> narrow(cx<double> v) { return {float(v.re), float(v.im)}; }
    NPHC_HD cx<double> zc(int i) const
    {
        const cx<double> a = z(i);
        const cx<float> d = dl(i);
        return {a.re + double(d.re), a.im + double(d.im)};
    }

    NPHC_HD void load_point(Point<float, M>& p) const
    {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            p.x[k] = narrow(z(k));
            p.y[k] = narrow(z(M + k));
        }
    }
    NPHC_HD cx<float> stage_base(int i) const { return narrow(z(i)); }
    NPHC_HD cx<float> predict(int i, float f, cx<float> wi) const
    {
        set_dl(i, f * wi);
        return narrow(zc(i));
    }
    NPHC_HD cx<float> correct(int i, cx<float>, cx<float> di) const
    {
        set_dl(i, dl(i) + di);
        return narrow(zc(i));
    }
    NPHC_HD void accept(const Point<float, M>&) const
    {
#pragma unroll
        for (int i = 0; i < 2 * M; ++i) set_z(i, zc(i));
    }
    NPHC_HD cx<double> get(int i) const { return z(i); }
    NPHC_HD void put(int i, cx<double> v) const { set_z(i, v); }

    // right-hand side for solve_step, read back from the accumulator slots
    static constexpr bool kExt = true;
    NPHC_HD bool use() const { return true; }
    template <class T> NPHC_HD cx<T> rg(int k) const { return w(k); }
    template <class T> NPHC_HD cx<T> rc(int k) const { return w(M + k); }

    // -H(z + dl, t) in float64 (g = (1 - t) gamma), rounded into the
    // accumulator slots: rows 0..M-1 gradient rows, M..2M-1 constraint rows.
    NPHC_HD void wide_residual(const Couplings<double, M>& C, cx<double> gamma, double t,
                               double omt) const
    {
        Point<double, M> q;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            q.x[k] = zc(k);
            q.y[k] = zc(M + k);
        }
        const cx<double> g = omt * gamma;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            cx<double> sx = {C.w(k), 0.0}, sy = {0.0, 0.0};
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j == k) continue;
                sx = axpy(C.J(k, j), q.x[j], sx);
                sy = axpy(C.J(k, j), q.y[j], sy);
            }
            const cx<double> x = q.x[k], y = q.y[k];
            const cx<double> F = y * sx - x * sy;
            const cx<double> xx = x * x, yy = y * y;
            const cx<double> xm1 = {xx.re - 1.0, xx.im};
            const cx<double> ym1 = {yy.re - 1.0, yy.im};
            const cx<double> con = {xx.re + yy.re - 1.0, xx.im + yy.im};
            set_w(k, narrow(-(g * xm1 + t * F)));
            set_w(M + k, narrow(-(g * ym1 + t * con)));
        }
    }
};

// The float64-evaluated right-hand side of a store (corrector) or the solve's
// own (predictor), chosen per call, so that both share one inlined solve.
// From M = kOneSolveSiteM on, the mixed-precision step inlines the solve once,
// with this run-time choice; below, it inlines a predictor and a corrector
// solve.  The choice costs a few hundred instructions per solve (both
// right-hand sides are formed); the second copy costs code size.  Measured on
// gfx950: with two copies the float32 tracker's code is 90 KB at M = 9,
// 127 KB at M = 10 and 190 KB at M = 12.  One copy is 5% slower at M = 9,
// but 13% faster at M = 10 and 31% faster at M = 12, where the loop no
// longer fits the instruction cache.
constexpr int kOneSolveSiteM = 10;
template <class Store>
struct SelRhs {
    static constexpr bool kExt = true;
    const Store& st;
    bool ext;
    NPHC_HD bool use() const { return ext; }
    template <class T> NPHC_HD cx<T> rg(int k) const { return st.template rg<T>(k); }
    template <class T> NPHC_HD cx<T> rc(int k) const { return st.template rc<T>(k); }
};

// The linear solve of one lane's own path.
struct LaneSolver {
    template <class T, int M>
    NPHC_HD bool operator()(const Couplings<T, M>& C, cx<T> gamma, T t, T omt, bool newton,
                            const Point<T, M>& z, Point<T, M>& d) const
    {
        return solve_step<T, M>(C, gamma, t, omt, newton, z, d);
    }
};

template <class S> constexpr bool kLaneSolver = false;
template <> constexpr bool kLaneSolver<LaneSolver> = true;

template <class Store, int M>
struct LanePath {
    Store st;
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
// nphc_track_paths).  Sets S.status when the path ends.  C and gamma are in the
// solve's type; C64 and gamma64 (float64) serve a store with a wide residual.
// solver performs the linear solves (one lane, or a lane group whose lanes all
// run this step on the same replicated state).
template <class Store, int M, class Solver = LaneSolver>
NPHC_HD void path_step(const Couplings<typename Store::Solve, M>& C,
                       cx<typename Store::Solve> gamma, const Couplings<double, M>& C64,
                       cx<double> gamma64, const TrackOptsDev& o, LanePath<Store, M>& S,
                       const Solver& solver = Solver{})
{
    using T = typename Store::Solve;
    const bool last = S.h >= o.t_end - S.t;
    const double hh = last ? (o.t_end - S.t) : S.h;
    const double t1 = last ? o.t_end : S.t + hh;
    const int nst = o.predictor == 0 ? 4 : 1;
    const Store& st = S.st;

    Point<T, M> zq;        // where the next linear solve is evaluated; after the
    st.load_point(zq);     // predictor, the point being corrected
    bool ok = true, conv = false, bad = false, too_far = false;
    T prev = T(0), d1 = T(0), wn1 = T(1);

    for (int s = 0; s < nst + o.max_corr; ++s) {
        const bool pred = s < nst;
        const bool want = pred ? ok : (ok && !conv && !bad);
        if (!want) continue;
        // stage times of the classical RK4: t, t + h/2, t + h/2, t + h
        const double tq = !pred ? t1 : (s == 0 ? S.t : (s == 3 ? t1 : S.t + 0.5 * hh));
        Point<T, M> d;
        bool sok;
        if constexpr (Store::kWideResidual) {
            if (!pred) st.wide_residual(C64, gamma64, tq, 1.0 - tq);
            if constexpr (M >= kOneSolveSiteM) {
                sok = solve_step<T, M>(C, gamma, T(tq), T(1.0 - tq), !pred, zq, d,
                                       SelRhs<Store>{st, !pred});
            } else if (!pred) {
                sok = solve_step<T, M>(C, gamma, T(tq), T(1.0 - tq), true, zq, d, st);
            } else {
                sok = solve_step<T, M>(C, gamma, T(tq), T(1.0 - tq), false, zq, d);
            }
        } else if constexpr (kLaneSolver<Solver>) {
            // (direct call: going through the policy object costs registers)
            sok = solve_step<T, M>(C, gamma, T(tq), T(1.0 - tq), !pred, zq, d);
        } else {
            sok = solver(C, gamma, T(tq), T(1.0 - tq), !pred, zq, d);
        }
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
                const cx<T> wi = (s == 0) ? di : axpy(ws, di, st.w(i));
                cx<T> next;
                if (final_stage) {
                    next = st.predict(i, f, wi);                      // predicted point
                } else {
                    st.set_w(i, wi);
                    next = axpy(ch, di, st.stage_base(i));
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
                    zq.x[i] = st.correct(i, zq.x[i], d.x[i]);
                    zq.y[i] = st.correct(M + i, zq.y[i], d.y[i]);
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
        st.accept(zq);
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
