"""Algorithmic operation counts of the per-lane tracker (real floating-point
operations; a complex multiply is 6, a complex multiply-add 8, a real times
complex product 2, a reciprocal 9, a square root 1).

One linear solve (nphc::solve_step, m = N - 1 free spins) does:
  sums Sx, Sy                     8 m (m - 1)
  right-hand side                 50 m
  constraint parametrisation      32 m
  sqrt(g + t), sqrt(t), scaling   10 + 8 m
  off-diagonal R (symmetric)      17 m (m - 1) / 2
  diagonal R and reduced rhs      m (62 + 8 (m - 1))
  elimination with pivoting       9 m (reciprocals) + 7 m (m - 1)
                                  + 8 (m - 1) m (2m - 1) / 6
  back substitution               4 m (m - 1) + 6 m
  recovery of (dx, dy)            16 m
Per step (RK4 predictor + c corrector iterations) the combinations of stage
vectors add 8 m per stage and 4 m per corrector update; the counter of linear
solves the tracker reports covers predictor stages and corrector iterations
alike, so the kernel's work is  solves * solve_flops(m) + steps * 48 m.

float32 tracking evaluates each corrector right-hand side -H(z + dl) once
more in float64 (nphc::MixedStore::wide_residual):
  point z + dl                    4 m
  sums Sx, Sy                     8 m (m - 1)
  F, squares, the two rows        50 m
  (1 - t) gamma                   4
With four predictor solves per step, the corrector solves are
solves - 4 * steps.

For comparison, the dense formulation (Gaussian elimination on the full
n x n Jacobian, n = 2m) costs dense_solve_flops(m) per solve.
"""


def solve_flops(m: int) -> int:
    return int(8 * m * (m - 1) + 50 * m + 32 * m + 10 + 8 * m + 17 * m * (m - 1) / 2
               + m * (62 + 8 * (m - 1)) + 9 * m + 7 * m * (m - 1)
               + 8 * (m - 1) * m * (2 * m - 1) / 6 + 4 * m * (m - 1) + 6 * m + 16 * m)


def step_overhead_flops(m: int) -> int:
    return 48 * m


def wide_residual_flops(m: int) -> int:
    return int(4 * m + 8 * m * (m - 1) + 50 * m + 4)


def kernel_flops(m: int, solves: int, steps: int, wide_residual: bool = False) -> int:
    """Total algorithmic flops of one tracking launch (wide_residual: float32
    tracking, whose corrector right-hand sides are evaluated in float64)."""
    f = int(solves) * solve_flops(m) + int(steps) * step_overhead_flops(m)
    if wide_residual:
        f += max(0, int(solves) - 4 * int(steps)) * wide_residual_flops(m)
    return f


def dense_solve_flops(m: int) -> int:
    """(8/3) n^3 + 8 n^2 for the dense complex LU and triangular solves, n = 2m,
    plus the dense Jacobian assembly and evaluation (~ 12 m^2 + 60 m)."""
    n = 2 * m
    return int(8 * n ** 3 / 3 + 8 * n * n + 12 * m * m + 60 * m)
