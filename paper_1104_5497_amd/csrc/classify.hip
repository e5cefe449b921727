// classify.hip -- real filter, angles, energies and Hessian-index
// classification of certified endpoints (float64, one lane per endpoint).
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace nphc {

struct ClassArgs {
    int32_t num_systems;
    int32_t M;
    int64_t item_lo, item_hi;
    const int32_t* N;
    const int64_t* path_off;
    const double* J;
    const int64_t* J_off;
    const int64_t* ids;
    int64_t count;
    const int64_t* count_dev;
    double eig_rel;
    int32_t sweeps;
    int32_t pad;
    double real_tol;
    const double* z;
    int64_t stride;
    const int32_t* endpoint;
    const double* alpha_real;
    int32_t* is_real;
    double* theta;
    double* energy;
    int32_t* index;
    double* eig;
    int32_t* degenerate;
};

// Eigenvalues of the symmetric M x M matrix a (destroyed) by cyclic Jacobi
// rotations: each rotation zeroes a_pq with t = tan(phi) the smaller root of
// t^2 + 2 theta t - 1 = 0, theta = (a_qq - a_pp) / (2 a_pq).
template <int M>
__device__ __forceinline__ void jacobi_eigenvalues(double (&a)[M][M], int max_sweeps, double (&w)[M])
{
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0, dia = 0.0;
#pragma unroll
        for (int p = 0; p < M; ++p) {
            dia += a[p][p] * a[p][p];
#pragma unroll
            for (int q = p + 1; q < M; ++q) off += a[p][q] * a[p][q];
        }
        if (!(off > 1e-34 * dia) ) break;
#pragma unroll
        for (int p = 0; p < M; ++p) {
#pragma unroll
            for (int q = p + 1; q < M; ++q) {
                const double apq = a[p][q];
                const bool rot = apq != 0.0;
                const double th = rot ? (a[q][q] - a[p][p]) / (2.0 * apq) : 0.0;
                double t = 1.0 / (fabs(th) + sqrt(th * th + 1.0));
                t = th < 0.0 ? -t : t;
                t = rot ? t : 0.0;
                const double c = 1.0 / sqrt(t * t + 1.0);
                const double s = t * c;
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const double arp = a[r][p], arq = a[r][q];
                    a[r][p] = c * arp - s * arq;
                    a[r][q] = s * arp + c * arq;
                }
#pragma unroll
                for (int r = 0; r < M; ++r) {
                    const double apr = a[p][r], aqr = a[q][r];
                    a[p][r] = c * apr - s * aqr;
                    a[q][r] = s * apr + c * aqr;
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < M; ++p) w[p] = a[p][p];
    // ascending order (odd-even transposition network)
#pragma unroll
    for (int r = 0; r < M; ++r) {
#pragma unroll
        for (int p = r & 1; p + 1 < M; p += 2) {
            const double lo = fmin(w[p], w[p + 1]), hi = fmax(w[p], w[p + 1]);
            w[p] = lo;
            w[p + 1] = hi;
        }
    }
}

template <int M>
__global__ __launch_bounds__(64) void classify_kernel(ClassArgs A)
{
    const double alpha0 = (13.0 - 3.0 * sqrt(17.0)) / 4.0;
    int64_t n = A.count;
    if (A.count_dev) n = min(n, *A.count_dev);
    int64_t lo = 0, hi = n;
    {
        int64_t a = 0, b = n;
        while (a < b) { int64_t mid = (a + b) >> 1; if (A.ids[mid] < A.item_lo) a = mid + 1; else b = mid; }
        lo = a;
        b = n;
        while (a < b) { int64_t mid = (a + b) >> 1; if (A.ids[mid] < A.item_hi) a = mid + 1; else b = mid; }
        hi = a;
    }
    constexpr int N = M + 1;
    for (int64_t pos = lo + blockIdx.x * int64_t(blockDim.x) + threadIdx.x; pos < hi;
         pos += int64_t(gridDim.x) * blockDim.x) {
        const int64_t g = A.ids[pos];
        const int64_t sys = find_system(A.path_off, A.num_systems, g);
        const double* Jb = A.J + A.J_off[sys];
        double x[N], y[N], imax = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            x[k] = A.z[(2 * k) * A.stride + g];
            imax = fmax(imax, fabs(A.z[(2 * k + 1) * A.stride + g]));
            y[k] = A.z[(2 * (M + k)) * A.stride + g];
            imax = fmax(imax, fabs(A.z[(2 * (M + k) + 1) * A.stride + g]));
        }
        x[M] = 1.0;
        y[M] = 0.0;
        const bool real = A.endpoint[g] == NPHC_END_NONSINGULAR && imax <= A.real_tol &&
                          A.alpha_real[g] < alpha0;
        A.is_real[pos] = real ? 1 : 0;
        if (!real) continue;
        // angles in (-pi, pi]
#pragma unroll
        for (int k = 0; k < M; ++k) {
            double th = atan2(y[k], x[k]);
            th = (th <= -M_PI) ? M_PI : th;
            A.theta[k * A.count + pos] = th;
        }
        // energy and Hessian in the angles; cos(theta_i - theta_j) = x_i x_j + y_i y_j
        double V = 0.0;
        double H[M][M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
#pragma unroll
            for (int j = 0; j < M; ++j) H[i][j] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                const double Jij = Jb[i * N + j];
                const double cij = x[i] * x[j] + y[i] * y[j];
                V += Jij * (1.0 - cij);
                const double w = Jij * cij;
                if (i < M) H[i][i] += w;
                if (j < M) H[j][j] += w;
                if (j < M) {
                    H[i][j] = -w;
                    H[j][i] = -w;
                }
            }
        }
        double w[M];
        jacobi_eigenvalues<M>(H, A.sweeps, w);
        double big = 1.0;
#pragma unroll
        for (int k = 0; k < M; ++k) big = fmax(big, fabs(w[k]));
        const double tau = A.eig_rel * big;
        int idx = 0;
        double small = INFINITY;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            idx += (w[k] < -tau) ? 1 : 0;
            small = fmin(small, fabs(w[k]));
            A.eig[k * A.count + pos] = w[k];
        }
        A.energy[pos] = V;
        A.index[pos] = idx;
        A.degenerate[pos] = (small <= tau) ? 1 : 0;
    }
}

int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN);

}  // namespace nphc

using namespace nphc;

extern "C" int nphc_classify(const nphc_batch* b, const int64_t* ids, int64_t count,
                             const int64_t* count_dev, const nphc_class_opts* o, double real_tol,
                             const double* z, int64_t item_stride, const int32_t* endpoint,
                             const double* alpha_real, int32_t* is_real, double* theta,
                             double* energy, int32_t* index, double* eig, int32_t* degenerate,
                             hipStream_t stream)
{
    bool mixed;
    int minN, maxN;
    int rc = check_batch(b, &mixed, &minN, &maxN);
    if (rc) return rc;
    if (!ids || !o || !z || !endpoint || !alpha_real || !is_real || !theta || !energy || !index ||
        !eig || !degenerate || count < 0 || o->jacobi_sweeps < 1)
        return NPHC_EINVAL;
    if (item_stride < b->path_off_host[b->num_systems]) return NPHC_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;
    int s = 0;
    while (s < b->num_systems) {
        int e = s;
        while (e < b->num_systems && b->N_host[e] == b->N_host[s]) ++e;
        ClassArgs A = {};
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
        A.eig_rel = o->eig_rel;
        A.sweeps = o->jacobi_sweeps;
        A.real_tol = real_tol;
        A.z = z;
        A.stride = item_stride;
        A.endpoint = endpoint;
        A.alpha_real = alpha_real;
        A.is_real = is_real;
        A.theta = theta;
        A.energy = energy;
        A.index = index;
        A.eig = eig;
        A.degenerate = degenerate;
        int64_t grid = (count + 63) / 64;
        if (grid > int64_t(cus) * 8) grid = int64_t(cus) * 8;
        if (grid < 1) grid = 1;
        const void* fn = nullptr;
        switch (A.M) {
#define NPHC_CCASE(m) case m: fn = reinterpret_cast<const void*>(&classify_kernel<m>); break;
            NPHC_CCASE(1) NPHC_CCASE(2) NPHC_CCASE(3) NPHC_CCASE(4) NPHC_CCASE(5) NPHC_CCASE(6)
            NPHC_CCASE(7) NPHC_CCASE(8) NPHC_CCASE(9) NPHC_CCASE(10) NPHC_CCASE(11) NPHC_CCASE(12)
#undef NPHC_CCASE
            default: return NPHC_EUNSUPPORTED;
        }
        void* args[] = {&A};
        if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64), args, 0, stream) != hipSuccess) return NPHC_EHIP;
        s = e;
    }
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}
