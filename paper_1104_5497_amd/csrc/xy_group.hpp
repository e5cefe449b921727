// xy_group.hpp -- the Newton/tangent solve of xy_lane.hpp spread over a
// group of 16 lanes (one path per group), for the last paths of a launch,
// where the latency of one step matters more than throughput.
//
// Lane r < M of the group owns row r of the reduced M x M system R v = rhs
// (see xy_lane.hpp for its derivation) and assembles it from the point z,
// which every lane of the group holds.  Lane r also owns constraint row r:
// it forms its parametrisation once, the other lanes gather the particular
// solutions they need, and after the solve lane r forms (dx_r, dy_r), which
// every lane then gathers.  Elimination uses partial pivoting
// without moving rows: for column k the unused row with the largest
// |re| + |im| is found by a 16-lane reduction, becomes pivot row k (its lane
// is marked used) and is broadcast to the other unused rows, which eliminate
// column k.  Back substitution runs in reverse pivot order, each solution
// component broadcast from the lane of its pivot row.  All 16 lanes of a
// group must call it together; the result d is returned on every lane.
#pragma once
#include "xy_lane.hpp"

namespace nphc {

constexpr int kGroup = 16;

template <class T>
__device__ __forceinline__ cx<T> gshfl(cx<T> v, int src)
{
    return {__shfl(v.re, src, kGroup), __shfl(v.im, src, kGroup)};
}

// Row r of the couplings, loaded once per path: Jr[j] = J_rj (0 for j = r),
// wr = J_{r,N}.
template <class T, int M>
struct GroupRow {
    T Jr[M];
    T wr;
};

template <class T, int M>
__device__ __forceinline__ void load_group_row(const Couplings<T, M>& C, int r, GroupRow<T, M>& G)
{
    const int rr = r < M ? r : 0;
#pragma unroll
    for (int j = 0; j < M; ++j) G.Jr[j] = (j == rr || r >= M) ? T(0) : C.p[rr * (M + 1) + j];
    G.wr = r < M ? C.p[rr * (M + 1) + M] : T(0);
}

// c ? a : b as an integer bit blend.  A plain select between two locals can
// be rewritten into a load through a selected address, which puts both in
// scratch memory; the blend keeps them in registers.
__device__ __forceinline__ double blend(bool c, double a, double b)
{
    const unsigned long long m = 0ull - (unsigned long long)c;
    return __builtin_bit_cast(double, (__builtin_bit_cast(unsigned long long, a) & m) |
                                          (__builtin_bit_cast(unsigned long long, b) & ~m));
}
__device__ __forceinline__ float blend(bool c, float a, float b)
{
    const unsigned m = 0u - (unsigned)c;
    return __builtin_bit_cast(float, (__builtin_bit_cast(unsigned, a) & m) |
                                         (__builtin_bit_cast(unsigned, b) & ~m));
}
template <class T>
__device__ __forceinline__ cx<T> blend(bool c, cx<T> a, cx<T> b)
{
    return {blend(c, a.re, b.re), blend(c, a.im, b.im)};
}

// Butterfly exchange inside a DPP row (16 lanes, which is one group):
// quad permutations [1,0,3,2] and [2,3,0,1] (partners lane ^ 1, lane ^ 2),
// then the half-row mirror (lane i of 8 reads 7 - i) and the row mirror
// (lane i of 16 reads 15 - i).  After the four stages a commutative,
// associative combine has seen all 16 lanes.  The partner is always inside
// the row, so no bound control is needed.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v)
{
    return __builtin_amdgcn_update_dpp(v, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_x(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = (unsigned)dpp_i<CTRL>((int)(unsigned)u);
    const unsigned hi = (unsigned)dpp_i<CTRL>((int)(unsigned)(u >> 32));
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_x(float v)
{
    return __builtin_bit_cast(float, dpp_i<CTRL>(__builtin_bit_cast(int, v)));
}

// one stage of the group argmax: largest val, ties to the lower lane
template <int CTRL, class T>
__device__ __forceinline__ void argmax_stage(T& val, int& who)
{
    const T v2 = dpp_x<CTRL>(val);
    const int w2 = dpp_i<CTRL>(who);
    const bool take = (v2 > val) || (v2 == val && w2 < who);
    val = take ? v2 : val;
    who = take ? w2 : who;
}

// maximum over the 16 lanes of the group (fmax: NaN operands are skipped)
template <class T>
__device__ __forceinline__ T group_max(T v)
{
    v = fmax(v, dpp_x<kDppXor1>(v));
    v = fmax(v, dpp_x<kDppXor2>(v));
    v = fmax(v, dpp_x<kDppHalfMirror>(v));
    v = fmax(v, dpp_x<kDppMirror>(v));
    return v;
}

// a[r] for the lane's row r (bit r of sel set; a[0] when no bit is set)
template <class T, int M>
__device__ __forceinline__ cx<T> pick(const cx<T> (&a)[M], unsigned sel)
{
    cx<T> v = a[0];
#pragma unroll
    for (int k = 1; k < M; ++k) v = blend(((sel >> k) & 1u) != 0u, a[k], v);
    return v;
}

template <class T, int M>
__device__ __forceinline__ bool group_solve_step(const GroupRow<T, M>& G, cx<T> gamma, T t, T omt, bool newton,
                                 const Point<T, M>& z, Point<T, M>& d)
{
    const int r = __lane_id() & (kGroup - 1);
    const unsigned onehot = 1u << r;
    const cx<T> g = omt * gamma;
    const cx<T> gt = {g.re + t, g.im};
    const cx<T> c1 = newton ? g : -gamma;
    const T c2 = newton ? t : T(1);
    const bool have_row = r < M;

    // --- constraint row r (lane r only; the others gather what they need)
    const cx<T> xr = pick<T, M>(z.x, onehot), yr = pick<T, M>(z.y, onehot);
    cx<T> ar, br, pxr, pyr;
    constraint_row<T>(t, gt, c1, c2, xr, yr, ar, br, pxr, pyr);

    // --- row r of R and its right-hand side
    cx<T> R[M];
    cx<T> v = {T(0), T(0)};
    {
        cx<T> sx = {G.wr, T(0)}, sy = {T(0), T(0)}, U = {T(0), T(0)}, W = {T(0), T(0)};
        const cx<T> Yr = gt * yr;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const cx<T> pxj = gshfl(pxr, j), pyj = gshfl(pyr, j);
            const T Jrj = G.Jr[j];  // zero for j = r
            sx = axpy(Jrj, z.x[j], sx);
            sy = axpy(Jrj, z.y[j], sy);
            U = axpy(Jrj, pxj, U);
            W = axpy(Jrj, pyj, W);
            // off-diagonal 2 t J_rj ((g + t) y_r y_j + t x_r x_j)
            R[j] = (T(2) * t * Jrj) * (Yr * z.y[j] + t * (xr * z.x[j]));
        }
        const cx<T> F = yr * sx - xr * sy;
        const cx<T> xx = xr * xr;
        const cx<T> xm1 = {xx.re - T(1), xx.im};
        const cx<T> rk = -(c1 * xm1 + c2 * F);
        const cx<T> Akk = (T(2) * g) * xr - t * sy;
        const cx<T> Bkk = t * sx;
        const cx<T> diag = Akk * br - Bkk * ar;
#pragma unroll
        for (int j = 0; j < M; ++j) R[j] = blend(((onehot >> j) & 1u) != 0u, diag, R[j]);
        v = rk - t * (yr * U - xr * W) - Akk * pxr - Bkk * pyr;
    }

    // --- elimination with partial pivoting, rows left in place
    bool used = !have_row;
    bool ok = true;
    int piv[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        T val = blend(used, T(-1), abs1(R[k]));
        int who = r;
        argmax_stage<kDppXor1>(val, who);
        argmax_stage<kDppXor2>(val, who);
        argmax_stage<kDppHalfMirror>(val, who);
        argmax_stage<kDppMirror>(val, who);
        const int p = who;
        piv[k] = p;
        ok = ok && (val > T(0));
        const cx<T> pk = gshfl(R[k], p);
        const cx<T> inv = rcp(pk);
        const bool elim = !used && r != p;
        const cx<T> l = blend(elim, R[k] * inv, cx<T>{T(0), T(0)});
#pragma unroll
        for (int j = k + 1; j < M; ++j) {
            const cx<T> pj = gshfl(R[j], p);
            R[j] = fnma(l, pj, R[j]);
        }
        const cx<T> vp = gshfl(v, p);
        v = fnma(l, vp, v);
        R[k] = blend(r == p, inv, R[k]);  // the pivot row keeps its reciprocal pivot
        used = used || r == p;
    }

    // --- back substitution in reverse pivot order: x_k on every lane
    cx<T> x[M];
#pragma unroll
    for (int k = M - 1; k >= 0; --k) {
        cx<T> acc = v;
#pragma unroll
        for (int j = k + 1; j < M; ++j) acc = fnma(R[j], x[j], acc);
        const cx<T> mine = acc * R[k];
        x[k] = gshfl(mine, piv[k]);
    }

    // --- back to (dx, dy): lane r forms component r, every lane gathers all
    const cx<T> vr = pick<T, M>(x, onehot);
    const cx<T> dxr = fma(br, vr, pxr);
    const cx<T> dyr = fnma(ar, vr, pyr);
    T mag = have_row ? fmax(absmax(dxr), absmax(dyr)) : T(0);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        d.x[k] = gshfl(dxr, k);
        d.y[k] = gshfl(dyr, k);
    }
    mag = group_max(mag);
    ok = ok && (mag - mag == T(0));
    return ok;
}

// The solve policy of path_step for a lane group.
template <int M>
struct GroupSolver {
    const GroupRow<double, M>* G;
    __device__ __forceinline__ bool operator()(const Couplings<double, M>&, cx<double> gamma,
                                               double t, double omt,
                               bool newton, const Point<double, M>& z, Point<double, M>& d) const
    {
        return group_solve_step<double, M>(*G, gamma, t, omt, newton, z, d);
    }
};

}  // namespace nphc
