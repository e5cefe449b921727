// adjoint.hip -- sensitivities of certified real stationary points to the
// couplings by the implicit-function theorem, in adjoint form: one
// transposed solve F_z^T lambda = dL/dz per stationary point (float64, one
// wavefront per point), then dL/dJ_ab = w_V dV/dJ_ab - lambda^T dF/dJ_ab.
#include <hip/hip_runtime.h>

#include "common.hpp"
#include "wave_dense.hpp"
#include "xy_dense.hpp"

namespace nphc {

struct AdjArgs {
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
    const double* z;
    int64_t stride;
    const double* w_V;
    const double* g_z;
    double* dLdJ;
};

template <int M>
struct AdjShared {
    GJShared<2 * M> gj;
    cd z[2 * M];
    double J[M * (M + 1) + 1];
    cd Fz[2 * M][2 * M + 1];
    double lam[2 * M];
};

template <int M>
__global__ __launch_bounds__(64) void adjoint_kernel(AdjArgs A)
{
    constexpr int NN = 2 * M;
    constexpr int N = M + 1;
    __shared__ AdjShared<M> sh;
    const int lane = threadIdx.x;
    int64_t n = A.count;
    if (A.count_dev) n = min(n, *A.count_dev);
    int64_t lo, hi;
    {
        int64_t a = 0, b = n;
        while (a < b) { int64_t mid = (a + b) >> 1; if (A.ids[mid] < A.item_lo) a = mid + 1; else b = mid; }
        lo = a;
        b = n;
        while (a < b) { int64_t mid = (a + b) >> 1; if (A.ids[mid] < A.item_hi) a = mid + 1; else b = mid; }
        hi = a;
    }
    for (int64_t pos = lo + blockIdx.x; pos < hi; pos += gridDim.x) {
        const int64_t g = A.ids[pos];
        const int64_t sys = find_system(A.path_off, A.num_systems, g);
        const double* Jb = A.J + A.J_off[sys];
        for (int e = lane; e < M * N; e += 64) sh.J[e] = Jb[(e / N) * N + (e % N)];
        // the stationary point is real: use the real parts
        if (lane < NN) sh.z[lane] = {A.z[(2 * lane) * A.stride + g], 0.0};
        __syncthreads();
        // row `lane` of F_z, transposed through LDS
        cd row[NN], F;
        xy_row<M>(lane, sh.J + (lane < M ? lane : 0) * N, sh.z, row, F);
        if (lane < NN) {
#pragma unroll
            for (int j = 0; j < NN; ++j) sh.Fz[lane][j] = row[j];
        }
        __syncthreads();
        cd col[NN], inv[NN];
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            col[j] = (lane < NN) ? sh.Fz[j][lane] : cd{0.0, 0.0};
            inv[j] = {0.0, 0.0};
        }
        // right-hand side dL/dz_lane = w_V dV/dz_lane + g_z[lane]
        const double wv = A.w_V ? A.w_V[pos] : 0.0;
        cd rhs = {0.0, 0.0};
        if (lane < NN) {
            const int k = lane < M ? lane : lane - M;
            const double* Jr = sh.J + k * N;
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < N; ++j) {
                if (j == k) continue;
                const double cj = (j < M) ? (lane < M ? sh.z[j].re : sh.z[M + j].re) : (lane < M ? 1.0 : 0.0);
                s += Jr[j] * cj;
            }
            rhs.re = -wv * s + (A.g_z ? A.g_z[lane * A.count + pos] : 0.0);
        }
        __syncthreads();
        const bool ok = wave_gauss_jordan<NN, false>(col, rhs, inv, sh.gj);
        if (lane < NN) sh.lam[lane] = ok ? rhs.re : 0.0;
        __syncthreads();
        // accumulate over the couplings (a, b), a < b < N: lanes stride over pairs
        double* out = A.dLdJ + A.J_off[sys];
        for (int e = lane; e < N * N; e += 64) {
            const int a = e / N, b = e % N;
            if (b <= a) continue;
            const double xa = a < M ? sh.z[a].re : 1.0, ya = a < M ? sh.z[M + a].re : 0.0;
            const double xb = b < M ? sh.z[b].re : 1.0, yb = b < M ? sh.z[M + b].re : 0.0;
            const double wab = ya * xb - xa * yb;
            const double la = a < M ? sh.lam[a] : 0.0;
            const double lb = b < M ? sh.lam[b] : 0.0;
            const double d = wv * (1.0 - xa * xb - ya * yb) - (la - lb) * wab;
            atomicAdd(&out[a * N + b], d);
            atomicAdd(&out[b * N + a], d);
        }
        __syncthreads();
    }
}

int check_batch(const nphc_batch* b, bool* mixed, int* minN, int* maxN);

}  // namespace nphc

using namespace nphc;

extern "C" int nphc_adjoint(const nphc_batch* b, const int64_t* ids, int64_t count,
                            const int64_t* count_dev, const double* z, int64_t item_stride,
                            const double* w_V, const double* g_z, double* dLdJ, hipStream_t stream)
{
    bool mixed;
    int minN, maxN;
    int rc = check_batch(b, &mixed, &minN, &maxN);
    if (rc) return rc;
    if (!ids || !z || !dLdJ || count < 0 || (!w_V && !g_z)) return NPHC_EINVAL;
    if (item_stride < b->path_off_host[b->num_systems]) return NPHC_EINVAL;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return NPHC_EHIP;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return NPHC_EHIP;
    int s = 0;
    while (s < b->num_systems) {
        int e = s;
        while (e < b->num_systems && b->N_host[e] == b->N_host[s]) ++e;
        AdjArgs A = {};
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
        A.z = z;
        A.stride = item_stride;
        A.w_V = w_V;
        A.g_z = g_z;
        A.dLdJ = dLdJ;
        int64_t grid = count < int64_t(cus) * 8 ? count : int64_t(cus) * 8;
        if (grid < 1) grid = 1;
        const void* fn = nullptr;
        switch (A.M) {
#define NPHC_ACASE(m) case m: fn = reinterpret_cast<const void*>(&adjoint_kernel<m>); break;
            NPHC_ACASE(1) NPHC_ACASE(2) NPHC_ACASE(3) NPHC_ACASE(4) NPHC_ACASE(5) NPHC_ACASE(6)
            NPHC_ACASE(7) NPHC_ACASE(8) NPHC_ACASE(9) NPHC_ACASE(10) NPHC_ACASE(11) NPHC_ACASE(12)
#undef NPHC_ACASE
            default: return NPHC_EUNSUPPORTED;
        }
        void* args[] = {&A};
        if (hipLaunchKernel(fn, dim3((unsigned)grid), dim3(64), args, 0, stream) != hipSuccess) return NPHC_EHIP;
        s = e;
    }
    if (hipGetLastError() != hipSuccess) return NPHC_EHIP;
    return NPHC_OK;
}
