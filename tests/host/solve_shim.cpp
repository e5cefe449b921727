// Host build of the tracker's per-lane linear solve (paper_1104_5497_amd/csrc/
// xy_lane.hpp) for CPU tests: solve_step and eval_F in float64 and float32,
// M = 2..12.  Test infrastructure only.
#include <cstdint>
#include <vector>

#include "../../paper_1104_5497_amd/csrc/xy_lane.hpp"

using namespace nphc;

namespace {

// right-hand side given by the caller: rows 0..M-1 gradient rows, M..2M-1
// constraint rows
template <class T, int M>
struct GivenRhs {
    static constexpr bool kExt = true;
    const double* r;  // 2M complex, interleaved
    bool use() const { return true; }
    template <class U> cx<U> rg(int k) const { return {U(r[2 * k]), U(r[2 * k + 1])}; }
    template <class U> cx<U> rc(int k) const { return {U(r[2 * (M + k)]), U(r[2 * (M + k) + 1])}; }
};

template <class T, int M>
int run(const double* J, double gre, double gim, double t, int newton, const double* z,
        const double* rhs, double* d_out, double* F_out)
{
    const int N = M + 1;
    std::vector<T> pack(M * (M + 1));
    for (int k = 0; k < M; ++k)
        for (int j = 0; j <= M; ++j) pack[k * (M + 1) + j] = (j == k) ? T(0) : T(J[k * N + j]);
    Couplings<T, M> C;
    C.p = pack.data();
    Point<T, M> p, d;
    for (int k = 0; k < M; ++k) {
        p.x[k] = {T(z[2 * k]), T(z[2 * k + 1])};
        p.y[k] = {T(z[2 * (M + k)]), T(z[2 * (M + k) + 1])};
    }
    const cx<T> g = {T(gre), T(gim)};
    bool ok;
    if (rhs)
        ok = solve_step<T, M>(C, g, T(t), T(1.0 - t), newton != 0, p, d, GivenRhs<T, M>{rhs});
    else
        ok = solve_step<T, M>(C, g, T(t), T(1.0 - t), newton != 0, p, d);
    for (int k = 0; k < M; ++k) {
        d_out[2 * k] = double(d.x[k].re);
        d_out[2 * k + 1] = double(d.x[k].im);
        d_out[2 * (M + k)] = double(d.y[k].re);
        d_out[2 * (M + k) + 1] = double(d.y[k].im);
    }
    if (F_out) {
        Point<T, M> F;
        eval_F<T, M>(C, p, F);
        for (int k = 0; k < M; ++k) {
            F_out[2 * k] = double(F.x[k].re);
            F_out[2 * k + 1] = double(F.x[k].im);
            F_out[2 * (M + k)] = double(F.y[k].re);
            F_out[2 * (M + k) + 1] = double(F.y[k].im);
        }
    }
    return ok ? 0 : 1;
}

template <class T>
int dispatch(int M, const double* J, double gre, double gim, double t, int newton, const double* z,
             const double* rhs, double* d, double* F)
{
    switch (M) {
#define NPHC_SHIM_CASE(m) \
    case m: return run<T, m>(J, gre, gim, t, newton, z, rhs, d, F);
        NPHC_SHIM_CASE(2) NPHC_SHIM_CASE(3) NPHC_SHIM_CASE(4) NPHC_SHIM_CASE(5) NPHC_SHIM_CASE(6)
        NPHC_SHIM_CASE(7) NPHC_SHIM_CASE(8) NPHC_SHIM_CASE(9) NPHC_SHIM_CASE(10) NPHC_SHIM_CASE(11)
        NPHC_SHIM_CASE(12)
#undef NPHC_SHIM_CASE
    default: return -1;
    }
}

}  // namespace

// precision 0: float64, 1: float32.  Returns 0 (solved), 1 (the solve
// reported failure) or -1 (M not built).
extern "C" int shim_solve(int precision, int M, const double* J, double gre, double gim, double t,
                          int newton, const double* z, const double* rhs, double* d, double* F)
{
    return precision ? dispatch<float>(M, J, gre, gim, t, newton, z, rhs, d, F)
                     : dispatch<double>(M, J, gre, gim, t, newton, z, rhs, d, F);
}
