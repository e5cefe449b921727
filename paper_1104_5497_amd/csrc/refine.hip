// refine.hip -- float64 endpoint refinement and certification.
//
// Refinement runs each endpoint on the structured solver of the tracker
// (nphc::solve_step at t = 1, where H = F): Newton on F, then the
// certificate quantities, with ||F_z^{-1}||_F from the 2m columns of the
// inverse (one solve per unit right-hand side).  One lane per endpoint, or a
// group of G lanes per endpoint (short lists, where latency matters): the
// group runs Newton identically on every lane and splits the certificate's
// 2m + 1 solves over its lanes.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "xy_lane.hpp"

namespace nphc {

struct RefineArgs {
    int32_t num_systems;
    int32_t M;                 // free spins of this launch's class
    int64_t item_lo, item_hi;  // the class's item range
    const int32_t* N;
    const int64_t* path_off;
    const double* J;
    const int64_t* J_off;
    const int64_t* ids;
    int64_t count;
    const int64_t* count_dev;
    nphc_cert_opts o;
    double* z;
    int64_t stride;
    const double* t;
    const int32_t* status;
    int32_t* endpoint;
    double *resid, *cond, *beta, *alpha, *alpha_real;
};

// Right-hand side chosen at run time: -F (j < 0, a Newton step) or e_j.
template <int M>
struct RefineRhs {
    static constexpr bool kExt = true;
    NPHC_HD bool use() const { return true; }
    int j;
    const Point<double, M>* F;
    template <class T> NPHC_HD cx<T> rg(int k) const
    {
        return j < 0 ? -F->x[k] : cx<T>{k == j ? T(1) : T(0), T(0)};
    }
    template <class T> NPHC_HD cx<T> rc(int k) const
    {
        return j < 0 ? -F->y[k] : cx<T>{M + k == j ? T(1) : T(0), T(0)};
    }
};

// Per endpoint, one sequence of linear solves at t = 1 (one solve site, so
// that the register frame of the float64 solve exists once):
//   NEWTON     z <- z + d, d = -F_z^{-1} F, until the update stops
//              decreasing or is below tol (1 + |z|), at most max_iter times;
//   CERT       at the refined z: beta = ||F_z^{-1} F||_2 (j = -1), then the
//              columns F_z^{-1} e_j (j = 0..2m-1) for ||F_z^{-1}||_F;
//   CERT_REAL  the same at Re z, for a nonsingular endpoint with
//              max |Im z_k| <= real_tol (certificate of a real root).
enum { PH_NEWTON = 0, PH_CERT = 1, PH_CERT_REAL = 2, PH_DONE = 3 };

// sum / logical and over the G lanes of a group (G a power of two <= 64)
template <int G>
__device__ __forceinline__ double group_sum(double v)
{
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, G);
    return v;
}
template <int G>
__device__ __forceinline__ bool group_all(bool v)
{
    int x = v ? 1 : 0;
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, G));
    return x != 0;
}

template <int M, int G>
__global__ __launch_bounds__(64) void refine_kernel(RefineArgs A)
{
    static_assert(G >= 1 && G <= 64 && (G & (G - 1)) == 0, "group size");
    // certificate rounds per phase: lane r solves columns r - 1, r - 1 + G, ...
    // (column -1: beta); every lane of a group runs all rounds, so the group
    // reaches the end of a phase together
    constexpr int kRounds = (2 * M + 1 + G - 1) / G;
    const int r = G > 1 ? int(threadIdx.x) % G : 0;
    const cx<double> none = {0.0, 0.0};
    int64_t n = A.count;
    if (A.count_dev) n = min(n, *A.count_dev);
    // list positions of this class
    int64_t lo = 0, hi = n;
    if (A.ids) {
        int64_t a = 0, b = n;
        while (a < b) { int64_t mid = (a + b) >> 1; if (A.ids[mid] < A.item_lo) a = mid + 1; else b = mid; }
        lo = a;
        b = n;
        while (a < b) { int64_t mid = (a + b) >> 1; if (A.ids[mid] < A.item_hi) a = mid + 1; else b = mid; }
        hi = a;
    } else {
        lo = A.item_lo;
        hi = A.item_hi;
    }
    const int64_t step = int64_t(gridDim.x) * blockDim.x / G;
    for (int64_t pos = lo + (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / G; pos < hi;
         pos += step) {
        const int64_t g = A.ids ? A.ids[pos] : pos;
        const int64_t sys = find_system(A.path_off, A.num_systems, g);
        CouplingsG<double, M> C;
        C.p = A.J + A.J_off[sys];
        Point<double, M> z;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            z.x[k] = {A.z[(2 * k) * A.stride + g], A.z[(2 * k + 1) * A.stride + g]};
            z.y[k] = {A.z[(2 * (M + k)) * A.stride + g], A.z[(2 * (M + k) + 1) * A.stride + g]};
        }
        const int32_t st = A.status[g];
        const double zmod0 = norm_mod<double, M>(z);
        const bool early = (st == NPHC_PATH_STALLED || st == NPHC_PATH_FAIL_MINSTEP ||
                            st == NPHC_PATH_FAIL_MAXSTEPS);
        const bool big = !(zmod0 <= A.o.div_norm);
        int32_t code = NPHC_END_FAIL;
        double resid = INFINITY, cond = INFINITY, beta = INFINITY, alpha = INFINITY, areal = INFINITY;
        if (st == NPHC_PATH_DIVERGED || (early && big)) {
            code = NPHC_END_DIVERGED;
        } else if (st == NPHC_PATH_REACHED || st == NPHC_PATH_STALLED) {
            // B = sqrt(||J~||_F^2 + 4m) / 2 over the free spins' block
            double jf = 0.0;
            for (int k = 0; k < M; ++k)
                for (int j = 0; j < M; ++j)
                    if (j != k) jf += C.J(k, j) * C.J(k, j);
            const double Bnd = 0.5 * sqrt(jf + 4.0 * M);
            const bool reached_one = (st == NPHC_PATH_REACHED) && (A.t[g] == 1.0);

            Point<double, M> F;       // F at the point of the current solves
            eval_F<double, M>(C, z, F);
            int phase = PH_NEWTON, it = 0, j = -1, round = 0;
            double prev = INFINITY, inv2 = 0.0, b2 = 0.0, an2 = 0.0, res = 0.0;
            bool cok = true;
            Point<double, M> zr;      // the real projection (CERT_REAL)
            while (phase != PH_DONE) {
                const Point<double, M>& zc = (phase == PH_CERT_REAL) ? zr : z;
                Point<double, M> d;
                // this lane's column in a certificate round (a valid one
                // stands in past the last column; its result is not used)
                const bool col = (phase == PH_NEWTON) || j < 2 * M;
                const int jj = col ? j : 0;
                const bool sok = solve_step<double, M, RefineRhs<M>, CouplingsG<double, M>, false>(
                    C, none, 1.0, 0.0, true, zc, d, RefineRhs<M>{jj, &F});
                double dd = 0.0;
#pragma unroll
                for (int k = 0; k < M; ++k) dd += norm2(d.x[k]) + norm2(d.y[k]);
                if (phase == PH_NEWTON) {
                    const double nd = norm_mod<double, M>(d);
                    bool stop = !sok || !(nd == nd) || (it > 0 && nd > prev);
                    if (!stop) {
#pragma unroll
                        for (int k = 0; k < M; ++k) {
                            z.x[k] = z.x[k] + d.x[k];
                            z.y[k] = z.y[k] + d.y[k];
                        }
                        prev = nd;
                        ++it;
                        stop = (nd <= A.o.tol * (1.0 + norm_mod<double, M>(z))) || it >= A.o.max_iter;
                    }
                    eval_F<double, M>(C, z, F);   // residual at the (possibly) updated point
                    if (stop) {
                        res = norm_mod<double, M>(F);
                        an2 = jac_frob2<double, M>(C, z);
                        phase = PH_CERT;
                        j = r - 1;
                        round = 0;
                        cok = true;
                        b2 = 0.0;
                        inv2 = 0.0;
                    }
                    continue;
                }
                // certificate phases
                if (col) {
                    cok = cok && sok;
                    if (j < 0) b2 = dd; else inv2 += dd;
                }
                j += G;
                if (++round < kRounds) continue;
                if constexpr (G > 1) {
                    b2 = group_sum<G>(b2);
                    inv2 = group_sum<G>(inv2);
                    cok = group_all<G>(cok);
                }
                if (phase == PH_CERT) {
                    resid = res;
                    if (cok) {
                        beta = sqrt(b2);
                        cond = sqrt(an2) * sqrt(inv2);
                        alpha = beta * sqrt(inv2) * Bnd;
                    }
                    const double zmod = norm_mod<double, M>(z);
                    const double scale = fmax(1.0, zmod * zmod);
                    if (cok && reached_one && resid < A.o.res_tol * scale && cond < A.o.cond_max)
                        code = NPHC_END_NONSINGULAR;
                    else if (resid < A.o.sing_res * scale && !(cond < A.o.cond_max))
                        code = NPHC_END_SINGULAR;
                    else
                        code = NPHC_END_FAIL;
                    double imax = 0.0;
#pragma unroll
                    for (int k = 0; k < M; ++k) imax = fmax(imax, fmax(fabs(z.x[k].im), fabs(z.y[k].im)));
                    if (code == NPHC_END_NONSINGULAR && imax <= A.o.real_tol) {
#pragma unroll
                        for (int k = 0; k < M; ++k) {
                            zr.x[k] = {z.x[k].re, 0.0};
                            zr.y[k] = {z.y[k].re, 0.0};
                        }
                        eval_F<double, M>(C, zr, F);
                        phase = PH_CERT_REAL;
                        j = r - 1;
                        round = 0;
                        cok = true;
                        b2 = 0.0;
                        inv2 = 0.0;
                    } else {
                        phase = PH_DONE;
                    }
                } else {
                    if (cok) areal = sqrt(b2) * sqrt(inv2) * Bnd;
                    phase = PH_DONE;
                }
            }
            if (r == 0) {
#pragma unroll
                for (int k = 0; k < M; ++k) {
                    A.z[(2 * k) * A.stride + g] = z.x[k].re;
                    A.z[(2 * k + 1) * A.stride + g] = z.x[k].im;
                    A.z[(2 * (M + k)) * A.stride + g] = z.y[k].re;
                    A.z[(2 * (M + k) + 1) * A.stride + g] = z.y[k].im;
                }
            }
        }
        if (r != 0) continue;   // the group's results are the same on every lane
        A.endpoint[g] = code;
        if (A.resid) A.resid[g] = resid;
        if (A.cond) A.cond[g] = cond;
        if (A.beta) A.beta[g] = beta;
        if (A.alpha) A.alpha[g] = alpha;
        if (A.alpha_real) A.alpha_real[g] = areal;
    }
}

int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN);

}  // namespace nphc

using namespace nphc;

extern "C" int nphc_refine_certify(const nphc_batch* b, const int64_t* ids, int64_t count,
                                   const int64_t* count_dev, const nphc_cert_opts* o, double* z,
                                   int64_t item_stride, const double* t, const int32_t* status,
                                   int32_t* endpoint, double* resid, double* cond, double* beta,
                                   double* alpha, double* alpha_real, hipStream_t stream)
{
    bool mixed;
    int minN, maxN;
    int rc = check_batch(b, &mixed, &minN, &maxN);
    if (rc) return rc;
    if (!o || !z || !t || !status || !endpoint || count < 0) return NPHC_EINVAL;
    const int64_t total = b->path_off_host[b->num_systems];
    if (item_stride < total) return NPHC_EINVAL;
    if (!ids) count = total;
    const int G = o->lanes_per_item <= 1 ? 1 : o->lanes_per_item;
    if (G != 1 && G != 4 && G != 8 && G != 16) return NPHC_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;
    int s = 0;
    while (s < b->num_systems) {
        int e = s;
        while (e < b->num_systems && b->N_host[e] == b->N_host[s]) ++e;
        RefineArgs A = {};
        A.num_systems = b->num_systems;
        A.M = b->N_host[s] - 1;
        A.item_lo = b->path_off_host[s];
        A.item_hi = b->path_off_host[e];
        A.N = b->N;
        A.path_off = b->path_off;
        A.J = b->J;
        A.J_off = b->J_off;
        A.ids = ids;
        A.count = count;
        A.count_dev = count_dev;
        A.o = *o;
        A.z = z;
        A.stride = item_stride;
        A.t = t;
        A.status = status;
        A.endpoint = endpoint;
        A.resid = resid;
        A.cond = cond;
        A.beta = beta;
        A.alpha = alpha;
        A.alpha_real = alpha_real;
        // G lanes per endpoint, several rounds per group
        const int64_t items = A.item_hi - A.item_lo;
        int64_t grid = int64_t(cus) * 4;
        const int64_t need = (items * G + 63) / 64;
        if (need < grid) grid = need;
        if (grid < 1) grid = 1;
        const void* fn = nullptr;
        switch (A.M) {
#define NPHC_RCASE(m)                                                                      \
    case m:                                                                                \
        fn = G == 1 ? reinterpret_cast<const void*>(&refine_kernel<m, 1>)                  \
           : G == 4 ? reinterpret_cast<const void*>(&refine_kernel<m, 4>)                  \
           : G == 8 ? reinterpret_cast<const void*>(&refine_kernel<m, 8>)                  \
                    : reinterpret_cast<const void*>(&refine_kernel<m, 16>);                \
        break;
            NPHC_RCASE(1) NPHC_RCASE(2) NPHC_RCASE(3) NPHC_RCASE(4) NPHC_RCASE(5) NPHC_RCASE(6)
            NPHC_RCASE(7) NPHC_RCASE(8) NPHC_RCASE(9) NPHC_RCASE(10) NPHC_RCASE(11) NPHC_RCASE(12)
#undef NPHC_RCASE
            default: return NPHC_EUNSUPPORTED;
        }
        void* args[] = {&A};
        if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64), args, 0, stream) != hipSuccess) return NPHC_EHIP;
        s = e;
    }
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}
