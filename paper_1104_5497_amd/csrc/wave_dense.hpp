// wave_dense.hpp -- dense complex float64 linear algebra with one wavefront
// per system: lane i < NN holds row i of the matrix in registers, rows are
// exchanged and the pivot row is broadcast through LDS.  Used by the
// low-volume float64 kernels (endpoint refinement, certification, adjoint),
// where a system is a whole 2m x 2m Jacobian.
#pragma once
#include "cx.hpp"

namespace nphc {

using cd = cx<double>;

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Shared scratch of one wave's Gauss-Jordan elimination.
template <int NN>
struct GJShared {
    cd piv[2 * NN + 1];   // broadcast pivot row: matrix, right-hand side, inverse part
    cd old[2 * NN + 1];   // the row that moves out of the pivot position
};

// Gauss-Jordan elimination with partial pivoting (largest |re|+|im| in the
// column, ties to the lower row) on the rows held by lanes 0..NN-1.
// On return lane i < NN holds x_i = (A^{-1} b)_i in `b` and, if WITH_INV,
// row i of A^{-1} in `inv` (which must enter as row i of the identity).
// Returns false (on every lane) when a pivot is zero.  All 64 lanes of the
// wave must call it.
template <int NN, bool WITH_INV>
__device__ __forceinline__ bool wave_gauss_jordan(cd (&a)[NN], cd& b, cd (&inv)[NN], GJShared<NN>& sh)
{
    const int lane = __lane_id();
    bool ok = true;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        double val = (lane >= k && lane < NN) ? abs1(a[k]) : -1.0;
        int who = lane;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            double v2 = __shfl_xor(val, o);
            int w2 = __shfl_xor(who, o);
            bool take = (v2 > val) || (v2 == val && w2 < who);
            val = take ? v2 : val;
            who = take ? w2 : who;
        }
        const int p = who;
        ok = ok && (val > 0.0);
        if (lane == p) {
#pragma unroll
            for (int j = k; j < NN; ++j) sh.piv[j] = a[j];
            sh.piv[NN] = b;
            if (WITH_INV) {
#pragma unroll
                for (int j = 0; j < NN; ++j) sh.piv[NN + 1 + j] = inv[j];
            }
        }
        if (lane == k && p != k) {
#pragma unroll
            for (int j = k; j < NN; ++j) sh.old[j] = a[j];
            sh.old[NN] = b;
            if (WITH_INV) {
#pragma unroll
                for (int j = 0; j < NN; ++j) sh.old[NN + 1 + j] = inv[j];
            }
        }
        __syncthreads();
        if (lane == p && p != k) {
#pragma unroll
            for (int j = k; j < NN; ++j) a[j] = sh.old[j];
            b = sh.old[NN];
            if (WITH_INV) {
#pragma unroll
                for (int j = 0; j < NN; ++j) inv[j] = sh.old[NN + 1 + j];
            }
        }
        if (lane == k) {
#pragma unroll
            for (int j = k; j < NN; ++j) a[j] = sh.piv[j];
            b = sh.piv[NN];
            if (WITH_INV) {
#pragma unroll
                for (int j = 0; j < NN; ++j) inv[j] = sh.piv[NN + 1 + j];
            }
        }
        // eliminate column k from every other row
        if (lane < NN && lane != k) {
            const cd pk = sh.piv[k];
            const cd f = ok ? a[k] * rcp(pk) : cd{0.0, 0.0};
            a[k] = {0.0, 0.0};
#pragma unroll
            for (int j = k + 1; j < NN; ++j) a[j] = fnma(f, sh.piv[j], a[j]);
            b = fnma(f, sh.piv[NN], b);
            if (WITH_INV) {
#pragma unroll
                for (int j = 0; j < NN; ++j) inv[j] = fnma(f, sh.piv[NN + 1 + j], inv[j]);
            }
        }
        __syncthreads();
    }
    if (lane < NN) {
        cd diag = a[0];
#pragma unroll
        for (int j = 1; j < NN; ++j) diag = (lane == j) ? a[j] : diag;
        const cd r = rcp(diag);
        b = b * r;
        if (WITH_INV) {
#pragma unroll
            for (int j = 0; j < NN; ++j) inv[j] = inv[j] * r;
        }
    }
    return ok;
}

}  // namespace nphc
