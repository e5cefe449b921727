// xy_lane.hpp -- per-lane homotopy evaluation and Newton/tangent solves for
// the gauge-fixed XY-ring stationary system, one path per lane.
//
// System (paper, eq. (1), with the couplings written as a symmetric matrix J
// and theta_N = 0, i.e. x_N = 1, y_N = 0):
//   F_k     = y_k Sx_k - x_k Sy_k,     Sx_k = sum_{j != k} J_kj x_j  (x_N = 1)
//                                      Sy_k = sum_{j != k} J_kj y_j  (y_N = 0)
//   F_{M+k} = x_k^2 + y_k^2 - 1,       k = 0..M-1, M = N - 1 free spins.
// Homotopy (paper, section "NPHC method"): H = gamma (1-t) Q + t F with the
// start system Q_k = z_k^2 - 1, unknowns z = (x_0..x_{M-1}, y_0..y_{M-1}).
//
// Linear solves H_z d = rhs use the structure of the constraint rows, which
// have exactly two nonzeros: row M+k is a_k dx_k + b_k dy_k = s_k with
// a_k = 2 t x_k and b_k = 2 (g + t) y_k, g = (1-t) gamma.  Its solutions are
//   (dx_k, dy_k) = v_k (b_k, -a_k) + (px_k, py_k),
//   (px_k, py_k) = s_k (conj a_k, conj b_k) / (|a_k|^2 + |b_k|^2),
// a null-space parametrisation that needs no case split and is well
// conditioned whenever (a_k, b_k) != 0 (true along every path: a_k = b_k = 0
// would force (1-t) gamma + t = 0).  Substituting into the gradient rows
// leaves an M x M complex system in v,
//   R_kj = A_kj b_j - B_kj a_j,   R v = r - A px - B py,
// with A = dH_grad/dx and B = dH_grad/dy.  Off the diagonal
//   R_kj = 2 t J_kj ((g + t) y_j y_k + t x_j x_k),
// (complex symmetric), on the diagonal
//   R_kk = (2 g x_k - t Sy_k) b_k - t Sx_k a_k.
// R is solved by Gaussian elimination with partial pivoting (largest
// |re|+|im|), the right-hand side carried along, rows exchanged with selects so
// that the matrix stays in registers.
#pragma once
#include "cx.hpp"

namespace nphc {

// Couplings of one system: rows k = 0..M-1 of the N x N matrix (N = M + 1,
// row-major), i.e. J_kj for free spins k, j at p[k*N + j] and the coupling to
// the fixed spin w_k = J_{k,N} at p[k*N + M].  Diagonal entries are never read.
template <class T, int M>
struct Couplings {
    const NPHC_RO T* p;
    NPHC_HD T J(int k, int j) const { return p[k * (M + 1) + j]; }
    NPHC_HD T w(int k) const { return p[k * (M + 1) + M]; }
};

// The same view through a generic pointer, for couplings whose address
// differs between lanes (the constant address space only pays for
// wave-uniform reads).
template <class T, int M>
struct CouplingsG {
    const T* p;
    NPHC_HD T J(int k, int j) const { return p[k * (M + 1) + j]; }
    NPHC_HD T w(int k) const { return p[k * (M + 1) + M]; }
};

template <class T, int M>
struct Point {
    cx<T> x[M], y[M];
};

// Constraint row k of the homotopy at (x_k, y_k): the coefficients a_k, b_k
// and the minimum-norm particular solution (px_k, py_k) of
// a_k dx_k + b_k dy_k = s_k, where s_k is the row's right-hand side
// -(c1 (y_k^2 - 1) + c2 (x_k^2 + y_k^2 - 1)).
// With EXT the right-hand side s_ext is given instead, where use_ext holds.
template <class T, bool EXT = false>
NPHC_HD void constraint_row(T t, cx<T> gt, cx<T> c1, T c2, cx<T> x, cx<T> y, cx<T>& a, cx<T>& b,
                            cx<T>& px, cx<T>& py, cx<T> s_ext = cx<T>{}, bool use_ext = true)
{
    const cx<T> xx = x * x, yy = y * y;
    const cx<T> ym1 = {yy.re - T(1), yy.im};
    const cx<T> con = {xx.re + yy.re - T(1), xx.im + yy.im};
    cx<T> s = -(c1 * ym1 + c2 * con);
    if constexpr (EXT) s = use_ext ? s_ext : s;
    a = (T(2) * t) * x;
    b = T(2) * (gt * y);
    const cx<T> sk = s * rrcp(norm2(a) + norm2(b));
    px = sk * conj(a);
    py = sk * conj(b);
}

// Right-hand side policies of solve_step.  kExt: the policy may supply the
// right-hand side (rg, rc); use(): whether it does for this call (a runtime
// choice lets one inlined solve serve both kinds of call).
// Right-hand side computed inside the solve (from z, in the solve's type).
struct OwnRhs {
    static constexpr bool kExt = false;
    NPHC_HD bool use() const { return false; }
    template <class T> NPHC_HD cx<T> rg(int) const { return cx<T>{}; }
    template <class T> NPHC_HD cx<T> rc(int) const { return cx<T>{}; }
};

// Unit right-hand side e_j (j < M: gradient row j, j >= M: constraint row
// j - M): the solve then returns column j of H_z^{-1}.
template <int M>
struct UnitRhs {
    static constexpr bool kExt = true;
    int j;
    NPHC_HD bool use() const { return true; }
    template <class T> NPHC_HD cx<T> rg(int k) const { return {k == j ? T(1) : T(0), T(0)}; }
    template <class T> NPHC_HD cx<T> rc(int k) const { return {M + k == j ? T(1) : T(0), T(0)}; }
};

// Pivot threshold of the elimination in tracking solves: 0 is partial
// pivoting; tau > 0 keeps the diagonal pivot while it is at least tau times
// the largest candidate (threshold pivoting, growth per step at most
// 1 + 1/tau).  Tracking solves only feed Newton corrections and predictor
// tangents, so their rounding costs iterations, not accuracy.  Solves with
// TRACK = false (certification) always pivot partially.  Measured on gfx950:
// float32 gains at every M; float64 gains up to M = 11 (less spill), but
// loses at M = 12, where it stays off.
template <class T, int M>
constexpr T pivot_tau()
{
    if constexpr (sizeof(T) == 4) return T(0.01);
    else return M <= 11 ? T(0.01) : T(0);
}

// Scheduling barriers between the phases of a solve (assembly, elimination,
// back substitution) bound the values live at once.  They keep the float64
// solve's spill down (968 instead of 1240 B per lane at M = 9).  The float32
// solve fits its registers either way and runs 1-3% faster without them.
#ifndef NPHC_FP32_SOLVE_PHASES
#define NPHC_FP32_SOLVE_PHASES 0
#endif
template <class T>
NPHC_HD void solve_phase()
{
    if constexpr (sizeof(T) == 8 || NPHC_FP32_SOLVE_PHASES) NPHC_PHASE();
}

// true if the predicate holds on any active lane of the wave (host: itself)
NPHC_HD bool wave_any(bool v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_ballot_w64(v) != 0ull;
#else
    return v;
#endif
}

// Solves H_z(z, t) d = -H(z, t) (newton = true) or -H_t(z, t) (the Davidenko
// tangent, newton = false).  gamma is the homotopy constant, t in [0, 1] and
// omt = 1 - t (passed separately so that it keeps its relative precision near
// t = 1).  Returns false when a pivot vanishes or the result is not finite.
// Only R, its right-hand side and z stay live through the elimination; the
// constraint parametrisation is recomputed for the back substitution.
// Rhs::kExt: the right-hand side is supplied by rhs (rg(k): gradient row k,
// rc(k): constraint row k), e.g. -H evaluated in a wider type; H_z is still
// formed from z in type T.
template <class T, int M, class Rhs = OwnRhs, class Cp = Couplings<T, M>, bool TRACK = true>
NPHC_HD bool solve_step(const Cp& C, cx<T> gamma, T t, T omt, bool newton,
                        const Point<T, M>& z, Point<T, M>& d, const Rhs& rhs = Rhs{})
{
    const cx<T> g = omt * gamma;             // (1 - t) gamma
    const cx<T> gt = {g.re + t, g.im};       // g + t
    // -H = -(c1 Q + c2 F) with (c1, c2) = (g, t); -H_t = -(F - gamma Q), i.e.
    // (c1, c2) = (-gamma, 1)
    const cx<T> c1 = newton ? g : -gamma;
    const T c2 = newton ? t : T(1);

    cx<T> R[M][M];   // reduced matrix (row-major, registers)
    cx<T> v[M];      // its right-hand side, then the solution
    {
        cx<T> px[M], py[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            cx<T> aj, bj;
            constraint_row<T, Rhs::kExt>(t, gt, c1, c2, z.x[j], z.y[j], aj, bj, px[j], py[j],
                                         rhs.template rc<T>(j), rhs.use());
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const cx<T> xk = z.x[k], yk = z.y[k];
            cx<T> sx = {C.w(k), T(0)}, sy = {T(0), T(0)};
            cx<T> U = {T(0), T(0)}, W = {T(0), T(0)};
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j == k) continue;
                const T Jkj = C.J(k, j);
                sx = axpy(Jkj, z.x[j], sx);
                sy = axpy(Jkj, z.y[j], sy);
                U = axpy(Jkj, px[j], U);
                W = axpy(Jkj, py[j], W);
            }
            const cx<T> F = yk * sx - xk * sy;
            const cx<T> xx = xk * xk;
            const cx<T> xm1 = {xx.re - T(1), xx.im};
            cx<T> rk = -(c1 * xm1 + c2 * F);
            if constexpr (Rhs::kExt) rk = rhs.use() ? rhs.template rg<T>(k) : rk;
            const cx<T> ak = (T(2) * t) * xk;
            const cx<T> bk = T(2) * (gt * yk);
            const cx<T> Akk = (T(2) * g) * xk - t * sy;
            const cx<T> Bkk = t * sx;
            R[k][k] = Akk * bk - Bkk * ak;
            // sum_{j != k} (A_kj px_j + B_kj py_j) = t (y_k U - x_k W)
            const cx<T> off = t * (yk * U - xk * W);
            v[k] = rk - off - Akk * px[k] - Bkk * py[k];
        }
    }
    // (px, py are dead from here on)
    // off-diagonal entries 2 t J_kj ((g + t) y_j y_k + t x_j x_k)
    {
        const cx<T> sg = csqrt(gt);
        const T st = sqrt(t);
        const T two_t = T(2) * t;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const cx<T> Xk = st * z.x[k], Yk = sg * z.y[k];
#pragma unroll
            for (int j = k + 1; j < M; ++j) {
                const cx<T> e = (sg * z.y[j]) * Yk + (st * z.x[j]) * Xk;
                const cx<T> val = (two_t * C.J(k, j)) * e;
                R[k][j] = val;
                R[j][k] = val;
            }
        }
    }


    solve_phase<T>();
    // Gaussian elimination with partial pivoting, right-hand side attached;
    // the reciprocal of pivot k replaces R[k][k].
    bool ok = true;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        solve_phase<T>();
        const T diag = abs1(R[k][k]);
        T best = diag;
        int p = k;
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            T m = abs1(R[i][k]);
            bool bigger = m > best;
            best = bigger ? m : best;
            p = bigger ? i : p;
        }
        ok = ok && (best > T(0));
        // threshold pivoting (pivot_tau > 0): keep the diagonal unless it is
        // below pivot_tau times the column maximum; the exchange code runs
        // only when some lane of the wave needs it
        bool exchange = true;
        if constexpr (TRACK && pivot_tau<T, M>() > T(0)) {
            const bool need = diag < pivot_tau<T, M>() * best;
            p = need ? p : k;
            exchange = wave_any(need);
        }
        if (k + 1 < M && exchange) {
            cx<T> rowk[M];
            const cx<T> vk = v[k];
#pragma unroll
            for (int j = k; j < M; ++j) rowk[j] = R[k][j];
#pragma unroll
            for (int i = k + 1; i < M; ++i) {
                const bool sw = (p == i);
#pragma unroll
                for (int j = k; j < M; ++j) {
                    const cx<T> ri = R[i][j];
                    R[k][j] = sel(sw, ri, R[k][j]);
                    R[i][j] = sel(sw, rowk[j], ri);
                }
                const cx<T> vi = v[i];
                v[k] = sel(sw, vi, v[k]);
                v[i] = sel(sw, vk, vi);
            }
        }
        const cx<T> inv = rcp(R[k][k]);
        R[k][k] = inv;
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const cx<T> l = R[i][k] * inv;
#pragma unroll
            for (int j = k + 1; j < M; ++j) R[i][j] = fnma(l, R[k][j], R[i][j]);
            v[i] = fnma(l, v[k], v[i]);
        }
    }
    solve_phase<T>();
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        cx<T> acc = v[i];
#pragma unroll
        for (int j = i + 1; j < M; ++j) acc = fnma(R[i][j], v[j], acc);
        v[i] = acc * R[i][i];
    }

    solve_phase<T>();
    // back to the full unknowns: (dx_k, dy_k) = v_k (b_k, -a_k) + (px_k, py_k)
    T mag = T(0);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        cx<T> ak, bk, pxk, pyk;
        constraint_row<T, Rhs::kExt>(t, gt, c1, c2, z.x[k], z.y[k], ak, bk, pxk, pyk,
                                     rhs.template rc<T>(k), rhs.use());
        d.x[k] = fma(bk, v[k], pxk);
        d.y[k] = fnma(ak, v[k], pyk);
        mag = fmax(mag, fmax(absmax(d.x[k]), absmax(d.y[k])));
    }
    ok = ok && (mag - mag == T(0));  // false for inf and NaN
    return ok;
}

// The target system F(z) (t = 1): F.x[k] gradient row k, F.y[k] constraint row k.
template <class T, int M, class Cp = Couplings<T, M>>
NPHC_HD void eval_F(const Cp& C, const Point<T, M>& z, Point<T, M>& F)
{
#pragma unroll
    for (int k = 0; k < M; ++k) {
        cx<T> sx = {C.w(k), T(0)}, sy = {T(0), T(0)};
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j == k) continue;
            sx = axpy(C.J(k, j), z.x[j], sx);
            sy = axpy(C.J(k, j), z.y[j], sy);
        }
        F.x[k] = z.y[k] * sx - z.x[k] * sy;
        const cx<T> xx = z.x[k] * z.x[k], yy = z.y[k] * z.y[k];
        F.y[k] = {xx.re + yy.re - T(1), xx.im + yy.im};
    }
}

// ||F_z(z)||_F^2.  Gradient row k: dF_k/dx_j = J_kj y_k, dF_k/dy_j = -J_kj x_k
// (j != k), dF_k/dx_k = -Sy_k, dF_k/dy_k = Sx_k; constraint row k: 2 x_k, 2 y_k.
template <class T, int M, class Cp = Couplings<T, M>>
NPHC_HD T jac_frob2(const Cp& C, const Point<T, M>& z)
{
    T s = T(0);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        cx<T> sx = {C.w(k), T(0)}, sy = {T(0), T(0)};
        T jj = T(0);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j == k) continue;
            sx = axpy(C.J(k, j), z.x[j], sx);
            sy = axpy(C.J(k, j), z.y[j], sy);
            jj += C.J(k, j) * C.J(k, j);
        }
        const T xk = norm2(z.x[k]), yk = norm2(z.y[k]);
        s += norm2(sx) + norm2(sy) + jj * (xk + yk) + T(4) * (xk + yk);
    }
    return s;
}

// max_k |z_k| (modulus)
template <class T, int M>
NPHC_HD T norm_mod(const Point<T, M>& z)
{
    T r = T(0);
#pragma unroll
    for (int k = 0; k < M; ++k) r = fmax(r, fmax(norm2(z.x[k]), norm2(z.y[k])));
    return sqrt(r);
}

// ||z||_inf in the max-of-|re|,|im| sense per coordinate (within sqrt(2) of
// the modulus norm; used for the divergence radius and tolerances)
template <class T, int M>
NPHC_HD T norm_inf(const Point<T, M>& z)
{
    T r = T(0);
#pragma unroll
    for (int k = 0; k < M; ++k) r = fmax(r, fmax(absmax(z.x[k]), absmax(z.y[k])));
    return r;
}

}  // namespace nphc
