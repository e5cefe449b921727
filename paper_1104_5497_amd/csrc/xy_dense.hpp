// xy_dense.hpp -- one row of F and of the dense Jacobian F_z of the
// gauge-fixed XY-ring system per lane (float64), for the one-wave-per-system
// kernels.
#pragma once
#include "cx.hpp"

namespace nphc {

using cd = cx<double>;

// Row i of F(z) and F_z(z) for the gauge-fixed XY system (see nphc.h), with
// z read from LDS.  Jrow points at row i's couplings J[i][0..N-1] (i < M):
//   F_i = y_i Sx_i - x_i Sy_i,  dF_i/dx_j = J_ij y_i,  dF_i/dy_j = -J_ij x_i (j != i),
//   dF_i/dx_i = -Sy_i,  dF_i/dy_i = Sx_i;  F_{M+k} = x_k^2 + y_k^2 - 1.
template <int M>
__device__ __forceinline__ void xy_row(int i, const double* Jrow, const cd* zs, cd (&row)[2 * M], cd& F)
{
#pragma unroll
    for (int j = 0; j < 2 * M; ++j) row[j] = {0.0, 0.0};
    if (i < M) {
        cd sx = {Jrow[M], 0.0};  // J_{i,N} x_N with x_N = 1
        cd sy = {0.0, 0.0};
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double Jij = (j == i) ? 0.0 : Jrow[j];
            sx = sx + Jij * zs[j];
            sy = sy + Jij * zs[M + j];
        }
        const cd xi = zs[i], yi = zs[M + i];
        F = yi * sx - xi * sy;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double Jij = (j == i) ? 0.0 : Jrow[j];
            row[j] = Jij * yi;
            row[M + j] = -(Jij * xi);
        }
        // diagonal entries: dF_i/dx_i = -Sy_i, dF_i/dy_i = Sx_i
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j == i) {
                row[j] = -sy;
                row[M + j] = sx;
            }
        }
    } else if (i < 2 * M) {
        const int k = i - M;
        cd xk = zs[0], yk = zs[M];
#pragma unroll
        for (int j = 1; j < M; ++j) {
            xk = (j == k) ? zs[j] : xk;
            yk = (j == k) ? zs[M + j] : yk;
        }
        const cd xx = xk * xk, yy = yk * yk;
        F = {xx.re + yy.re - 1.0, xx.im + yy.im};
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j == k) {
                row[j] = 2.0 * xk;
                row[M + j] = 2.0 * yk;
            }
        }
    } else {
        F = {0.0, 0.0};
    }
}

}  // namespace nphc
