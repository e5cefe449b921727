// refine.hip -- float64 endpoint refinement, certification and the
// path-jump (duplicate endpoint) check.
//
// One wavefront per endpoint: lane i < 2m evaluates row i of F and F_z, and
// the 2m x 2m system is solved by wave_gauss_jordan.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "wave_dense.hpp"
#include "xy_dense.hpp"

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

template <int M>
struct RefineShared {
    GJShared<2 * M> gj;
    cd z[2 * M];
    double J[M * (M + 1) + 1];  // rows 0..M-1 of the ring's couplings, N = M+1 columns
};

// Evaluates F and F_z at zs, then solves.  WITH_INV also returns the inverse
// row and the Frobenius norms; x = F_z^{-1} F is returned in `sol`.
template <int M, bool WITH_INV>
__device__ __forceinline__ bool newton_solve(RefineShared<M>& sh, int lane, cd& sol, double* Fmax,
                                             double* Anorm2, double* Ainvnorm2)
{
    constexpr int NN = 2 * M;
    cd row[NN], inv[NN];
    cd F;
    const double* Jrow = sh.J + (lane < M ? lane : 0) * (M + 1);
    xy_row<M>(lane, Jrow, sh.z, row, F);
    if (Fmax) *Fmax = wave_max(lane < NN ? sqrt(norm2(F)) : 0.0);
    if (Anorm2) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NN; ++j) s += norm2(row[j]);
        *Anorm2 = wave_sum(lane < NN ? s : 0.0);
    }
#pragma unroll
    for (int j = 0; j < NN; ++j) inv[j] = {(j == lane) ? 1.0 : 0.0, 0.0};
    sol = F;
    const bool ok = wave_gauss_jordan<NN, WITH_INV>(row, sol, inv, sh.gj);
    if (WITH_INV && Ainvnorm2) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < NN; ++j) s += norm2(inv[j]);
        *Ainvnorm2 = wave_sum(lane < NN ? s : 0.0);
    }
    return ok;
}

template <int M>
__global__ __launch_bounds__(64) void refine_kernel(RefineArgs A)
{
    constexpr int NN = 2 * M;
    __shared__ RefineShared<M> sh;
    const int lane = threadIdx.x;
    int64_t n = A.count;
    if (A.count_dev) n = min(n, *A.count_dev);
    // queue positions of this class
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

    for (int64_t pos = lo + blockIdx.x; pos < hi; pos += gridDim.x) {
        const int64_t g = A.ids ? A.ids[pos] : pos;
        const int64_t sys = find_system(A.path_off, A.num_systems, g);
        const int N = M + 1;
        const double* Jb = A.J + A.J_off[sys];
        for (int e = lane; e < M * N; e += 64) sh.J[e] = Jb[(e / N) * N + (e % N)];
        // B = sqrt(||J~||_F^2 + 4m) / 2 over the free spins' block
        double jf = 0.0;
        for (int e = lane; e < M * M; e += 64) {
            const int r = e / M, c = e % M;
            const double v = (r == c) ? 0.0 : Jb[r * N + c];
            jf += v * v;
        }
        const double Bnd = 0.5 * sqrt(wave_sum(jf) + 4.0 * M);
        if (lane < NN) sh.z[lane] = {A.z[(2 * lane) * A.stride + g], A.z[(2 * lane + 1) * A.stride + g]};
        __syncthreads();
        const int32_t st = A.status[g];
        double zmod = wave_max(lane < NN ? sqrt(norm2(sh.z[lane])) : 0.0);
        const bool early = (st == NPHC_PATH_STALLED || st == NPHC_PATH_FAIL_MINSTEP ||
                            st == NPHC_PATH_FAIL_MAXSTEPS);
        const bool big = !(zmod <= A.o.div_norm);
        int32_t code;
        double resid = INFINITY, cond = INFINITY, beta = INFINITY, alpha = INFINITY, areal = INFINITY;
        if (st == NPHC_PATH_DIVERGED || (early && big)) {
            code = NPHC_END_DIVERGED;
        } else if (st == NPHC_PATH_REACHED || st == NPHC_PATH_STALLED) {
            // Newton on F at t = 1
            double prev = INFINITY;
            for (int it = 0; it < A.o.max_iter; ++it) {
                cd d;
                if (!newton_solve<M, false>(sh, lane, d, nullptr, nullptr, nullptr)) break;
                const double nd = wave_max(lane < NN ? sqrt(norm2(d)) : 0.0);
                if (!(nd == nd) || (it > 0 && nd > prev)) break;
                if (lane < NN) sh.z[lane] = sh.z[lane] - d;
                __syncthreads();
                prev = nd;
                const double zn = wave_max(lane < NN ? sqrt(norm2(sh.z[lane])) : 0.0);
                if (nd <= A.o.tol * (1.0 + zn)) break;
            }
            zmod = wave_max(lane < NN ? sqrt(norm2(sh.z[lane])) : 0.0);
            cd x;
            double an2 = 0.0, ain2 = 0.0;
            const bool ok = newton_solve<M, true>(sh, lane, x, &resid, &an2, &ain2);
            if (ok) {
                beta = sqrt(wave_sum(lane < NN ? norm2(x) : 0.0));
                cond = sqrt(an2) * sqrt(ain2);
                alpha = beta * sqrt(ain2) * Bnd;
            }
            const double scale = fmax(1.0, zmod * zmod);
            const bool reached_one = (st == NPHC_PATH_REACHED) && (A.t[g] == 1.0);
            if (ok && reached_one && resid < A.o.res_tol * scale && cond < A.o.cond_max)
                code = NPHC_END_NONSINGULAR;
            else if (resid < A.o.sing_res * scale && !(cond < A.o.cond_max))
                code = NPHC_END_SINGULAR;
            else
                code = NPHC_END_FAIL;
            // certificate of the real projection
            const double imax = wave_max(lane < NN ? fabs(sh.z[lane].im) : 0.0);
            if (code == NPHC_END_NONSINGULAR && imax <= A.o.real_tol) {
                __syncthreads();
                cd keep = (lane < NN) ? sh.z[lane] : cd{0.0, 0.0};
                if (lane < NN) sh.z[lane] = {keep.re, 0.0};
                __syncthreads();
                cd xr;
                double ai2 = 0.0, rres = 0.0;
                if (newton_solve<M, true>(sh, lane, xr, &rres, nullptr, &ai2)) {
                    const double br = sqrt(wave_sum(lane < NN ? norm2(xr) : 0.0));
                    areal = br * sqrt(ai2) * Bnd;
                }
                __syncthreads();
                if (lane < NN) sh.z[lane] = keep;
                __syncthreads();
            }
            if (lane < NN) {
                A.z[(2 * lane) * A.stride + g] = sh.z[lane].re;
                A.z[(2 * lane + 1) * A.stride + g] = sh.z[lane].im;
            }
        } else {
            code = NPHC_END_FAIL;
        }
        if (lane == 0) {
            A.endpoint[g] = code;
            if (A.resid) A.resid[g] = resid;
            if (A.cond) A.cond[g] = cond;
            if (A.beta) A.beta[g] = beta;
            if (A.alpha) A.alpha[g] = alpha;
            if (A.alpha_real) A.alpha_real[g] = areal;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// duplicate endpoints
// ---------------------------------------------------------------------------
struct DupArgs {
    int32_t num_systems;
    int32_t n_max;             // unknowns of the largest ring
    const int32_t* N;
    const int64_t* path_off;
    const int64_t* cand;       // sorted NONSINGULAR item ids (candidates)
    const int64_t* cand_count; // device
    int64_t tiles_per_system;
    double tol;
    const double* z;
    int64_t stride;
    int32_t* endpoint;
    unsigned long long* marked;
};

__global__ void zero_counter_kernel(unsigned long long* c) { *c = 0ull; }

__device__ __forceinline__ void mark_dup(int32_t* endpoint, int64_t g, unsigned long long* marked)
{
    const int old = atomicExch(&endpoint[g], NPHC_END_DUPLICATE);
    if (old != NPHC_END_DUPLICATE) atomicAdd(marked, 1ull);
}

// Candidates of one system form a contiguous run of the sorted list.  Work
// unit u = (system b, tile of 256 candidates); each thread owns one
// candidate i of the tile and compares it with every later candidate j of the
// same system, first on the first coordinate (staged through LDS), then on
// all of them.
__global__ __launch_bounds__(256) void duplicates_kernel(DupArgs A)
{
    __shared__ double s_re[256], s_im[256];
    __shared__ int64_t s_g[256];
    const int64_t K = *A.cand_count;
    const int64_t units = int64_t(A.num_systems) * A.tiles_per_system;
    for (int64_t u = blockIdx.x; u < units; u += gridDim.x) {
        const int64_t b = u / A.tiles_per_system;
        const int64_t tile = u % A.tiles_per_system;
        const int64_t glo = A.path_off[b], ghi = A.path_off[b + 1];
        // candidate range of system b
        int64_t lo = 0, hi = K;
        {
            int64_t a = 0, e = K;
            while (a < e) { int64_t mid = (a + e) >> 1; if (A.cand[mid] < glo) a = mid + 1; else e = mid; }
            lo = a;
            e = K;
            while (a < e) { int64_t mid = (a + e) >> 1; if (A.cand[mid] < ghi) a = mid + 1; else e = mid; }
            hi = a;
        }
        const int64_t i0 = lo + tile * 256;
        if (i0 >= hi) continue;  // uniform across the block
        const int64_t i = i0 + threadIdx.x;
        const bool have = i < hi;
        const int64_t gi = have ? A.cand[i] : 0;
        const int n = 2 * (A.N[b] - 1);
        const double re0 = have ? A.z[gi] : 0.0;
        const double im0 = have ? A.z[A.stride + gi] : 0.0;
        for (int64_t j0 = i0; j0 < hi; j0 += 256) {
            __syncthreads();
            const int64_t jj = j0 + threadIdx.x;
            if (jj < hi) {
                const int64_t gj = A.cand[jj];
                s_g[threadIdx.x] = gj;
                s_re[threadIdx.x] = A.z[gj];
                s_im[threadIdx.x] = A.z[A.stride + gj];
            }
            __syncthreads();
            const int lim = (int)min<int64_t>(256, hi - j0);
            if (have) {
                for (int q = 0; q < lim; ++q) {
                    if (j0 + q <= i) continue;
                    if (fabs(s_re[q] - re0) >= A.tol || fabs(s_im[q] - im0) >= A.tol) continue;
                    const int64_t gj = s_g[q];
                    bool close = true;
                    for (int k = 1; k < n && close; ++k) {
                        close = fabs(A.z[(2 * k) * A.stride + gi] - A.z[(2 * k) * A.stride + gj]) < A.tol &&
                                fabs(A.z[(2 * k + 1) * A.stride + gi] - A.z[(2 * k + 1) * A.stride + gj]) < A.tol;
                    }
                    if (close) {
                        mark_dup(A.endpoint, gi, A.marked);
                        mark_dup(A.endpoint, gj, A.marked);
                    }
                }
            }
        }
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
        const int64_t items = A.item_hi - A.item_lo;
        int64_t grid = int64_t(cus) * 16;
        if (items < grid) grid = items;
        if (grid < 1) grid = 1;
        const void* fn = nullptr;
        switch (A.M) {
#define NPHC_RCASE(m) case m: fn = reinterpret_cast<const void*>(&refine_kernel<m>); break;
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

extern "C" int nphc_mark_duplicates(const nphc_batch* b, const int64_t* ids, int64_t count,
                                    const int64_t* count_dev, double dup_tol, const double* z,
                                    int64_t item_stride, int32_t* endpoint, int64_t* num_marked,
                                    void* workspace, size_t ws_bytes, hipStream_t stream)
{
    bool mixed;
    int minN, maxN;
    int rc = check_batch(b, &mixed, &minN, &maxN);
    if (rc) return rc;
    if (!ids || !count_dev || !z || !endpoint || !num_marked || !(dup_tol > 0.0)) return NPHC_EINVAL;
    (void)count;
    (void)workspace;
    (void)ws_bytes;
    const int64_t total = b->path_off_host[b->num_systems];
    if (item_stride < total) return NPHC_EINVAL;
    DupArgs A = {};
    A.num_systems = b->num_systems;
    A.n_max = 2 * (maxN - 1);
    A.N = b->N;
    A.path_off = b->path_off;
    A.cand = ids;
    A.cand_count = count_dev;
    int64_t maxp = 0;
    for (int s = 0; s < b->num_systems; ++s) {
        const int64_t p = b->path_off_host[s + 1] - b->path_off_host[s];
        maxp = p > maxp ? p : maxp;
    }
    A.tiles_per_system = (maxp + 255) / 256;
    A.tol = dup_tol;
    A.z = z;
    A.stride = item_stride;
    A.endpoint = endpoint;
    A.marked = reinterpret_cast<unsigned long long*>(num_marked);
    hipLaunchKernelGGL(zero_counter_kernel, dim3(1), dim3(1), 0, stream, A.marked);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;
    const int64_t units = int64_t(b->num_systems) * A.tiles_per_system;
    int64_t grid = int64_t(cus) * 8;
    if (units < grid) grid = units;
    hipLaunchKernelGGL(duplicates_kernel, dim3((unsigned)grid), dim3(256), 0, stream, A);
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}
