"""Seeded synthetic instances of the power-law XY ring (inputs only).

This module draws the problem data that both the HIP path and the CPU oracle
consume: the coupling matrix J of a ring of N spins and the random complex
constant gamma of the total-degree homotopy.  It holds none of the method's
arithmetic (no homotopy, no tracking, no linear algebra): it only writes down
the model's coefficients and the random numbers the method needs.

Model (paper, "A First Application"): the power-law XY ring
    V(theta) = K * sum_i sum_{j=1}^{(N-1)/2} (1 - cos(theta_i - theta_{i+j})) / j^alpha
with periodic boundary conditions and theta_N fixed to 0.  For odd N each
unordered pair (i, k) appears exactly once with ring distance
r_ik = min(|i-k|, N-|i-k|), so V = sum_{i<k} J_ik (1 - cos(theta_i - theta_k))
with J_ik = K / r_ik^alpha.  The same all-pairs form is used for even N
(pairs at distance N/2 are counted once) and for disordered rings
J_ik = g_ik / r_ik^sigma with g_ik ~ N(0, 1).

gamma (paper, homotopy H = gamma (1-t) Q + t P): a random complex number; here
|gamma| = 1 and its phase is 2*pi*U with U the first uniform draw of
numpy.random.default_rng(seed).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Sequence

import numpy as np

__all__ = [
    "ring_distance",
    "clean_ring_J",
    "paper_ring_J",
    "disordered_ring_J",
    "gamma_from_seed",
    "RingBatch",
    "batch_rings",
    "num_paths",
]


def num_paths(N: int) -> int:
    """Number of start solutions 2^(2(N-1)) = 4^(N-1) (one path each)."""
    return 4 ** (N - 1)


def ring_distance(N: int) -> np.ndarray:
    """r_ik = min(|i-k|, N-|i-k|) as an (N, N) int64 array (0 on the diagonal)."""
    i = np.arange(N)
    d = np.abs(i[:, None] - i[None, :])
    return np.minimum(d, N - d)


def clean_ring_J(N: int, sigma: float) -> np.ndarray:
    """Clean power-law ring J_ik = r_ik^(-sigma), J_ii = 0, float64 (N, N)."""
    if N < 2:
        raise ValueError("ring needs N >= 2")
    r = ring_distance(N).astype(np.float64)
    J = np.zeros((N, N), dtype=np.float64)
    off = r > 0
    J[off] = r[off] ** (-float(sigma))
    return J


def paper_ring_J(N: int, alpha: float = 0.75) -> np.ndarray:
    """The paper's normalised ring: odd N, J_ik = K r_ik^(-alpha) with
    K = (2 sum_{j=1}^{(N-1)/2} j^(-alpha))^(-1)."""
    if N % 2 != 1:
        raise ValueError("the paper's normalisation is defined for odd N")
    K = 1.0 / (2.0 * sum(j ** (-float(alpha)) for j in range(1, (N - 1) // 2 + 1)))
    return K * clean_ring_J(N, alpha)


def disordered_ring_J(N: int, sigma: float, rng: np.random.Generator) -> np.ndarray:
    """J_ik = g_ik r_ik^(-sigma), g_ik = g_ki ~ N(0,1) drawn for i<k in row-major order."""
    r = ring_distance(N).astype(np.float64)
    J = np.zeros((N, N), dtype=np.float64)
    for i in range(N):
        for k in range(i + 1, N):
            g = rng.standard_normal()
            J[i, k] = J[k, i] = g * r[i, k] ** (-float(sigma))
    return J


def gamma_from_seed(seed: int) -> complex:
    """gamma = exp(i * 2 pi U), U = default_rng(seed).random()."""
    u = np.random.default_rng(seed).random()
    return complex(math.cos(2.0 * math.pi * u), math.sin(2.0 * math.pi * u))


@dataclass
class RingBatch:
    """Many rings tracked together.  Arrays are host numpy, float64."""

    N: List[int] = field(default_factory=list)
    sigma: List[float] = field(default_factory=list)
    J: List[np.ndarray] = field(default_factory=list)
    gamma: List[complex] = field(default_factory=list)

    def __len__(self) -> int:
        return len(self.N)

    @property
    def path_offsets(self) -> np.ndarray:
        """Prefix sums of 4^(N_b - 1), length len(self)+1, int64."""
        off = np.zeros(len(self.N) + 1, dtype=np.int64)
        off[1:] = np.cumsum([num_paths(n) for n in self.N])
        return off


def batch_rings(seed: int, counts: Dict[int, int] | Sequence[tuple] = ((5, 128), (6, 128), (7, 128)),
                sigma_range=(0.5, 2.0)) -> RingBatch:
    """Disordered rings drawn from one generator: for each ring in order,
    sigma_b ~ U(sigma_range), then g_ik (i<k, row-major), then the gamma phase."""
    rng = np.random.default_rng(seed)
    items = list(counts.items()) if isinstance(counts, dict) else list(counts)
    out = RingBatch()
    for N, cnt in items:
        for _ in range(int(cnt)):
            s = float(rng.uniform(sigma_range[0], sigma_range[1]))
            J = disordered_ring_J(int(N), s, rng)
            u = rng.random()
            out.N.append(int(N))
            out.sigma.append(s)
            out.J.append(J)
            out.gamma.append(complex(math.cos(2 * math.pi * u), math.sin(2 * math.pi * u)))
    return out
