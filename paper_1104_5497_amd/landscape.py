"""Landscape analytics of the certified real stationary points (paper,
section "A First Application", Figs. 1-3), from the classification outputs
(angles, Hessian eigenvalues and energies computed on the GPU).

For a ring of N spins with theta_N = 0 and m = N - 1 free angles:
  * energy density V/N and index density I/(N - 1) of every stationary point;
  * |det H|^(1/N), with det H the product of the m Hessian eigenvalues;
  * the kind of a configuration: every theta_i in {0, pi} ("zero_pi"), or a
    twisted state, where all N consecutive differences theta_{i+1} - theta_i
    (cyclically, theta_N = 0) equal one 2 pi k / N mod 2 pi ("twisted");
  * the paper's observations: the global minimum is theta = 0 with V = 0, and
    the smallest |det H|^(1/N) sits at a zero_pi or twisted configuration.
Host arithmetic on compact per-stationary-point arrays only.
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np


def _wrap(a: np.ndarray) -> np.ndarray:
    """Angles to [-pi, pi)."""
    return (a + math.pi) % (2.0 * math.pi) - math.pi


def config_kind(theta: np.ndarray, N: int, tol: float = 1e-8) -> str:
    """'zero_pi', 'twisted' or 'other' for one configuration of the m free
    angles (theta_N = 0).  theta = 0 is both; it is reported as zero_pi."""
    th = np.asarray(theta, dtype=np.float64)
    if np.all(np.minimum(np.abs(_wrap(th)), np.abs(np.abs(_wrap(th)) - math.pi)) < tol):
        return "zero_pi"
    full = np.append(th, 0.0)
    diffs = _wrap(np.roll(full, -1) - full)          # theta_{i+1} - theta_i, cyclic
    step = 2.0 * math.pi / N
    k = np.round(diffs[0] / step)
    if abs(_wrap(diffs[0] - k * step)) < tol and np.all(np.abs(_wrap(diffs - diffs[0])) < tol):
        return "twisted"
    return "other"


def landscape(N: int, theta: np.ndarray, index: np.ndarray, V: np.ndarray, eig: np.ndarray,
              degenerate: np.ndarray) -> Dict:
    """Per nondegenerate stationary point: energy density, index density and
    |det H|^(1/N); plus the global minimum and the minimiser of |det H|^(1/N)."""
    nd = ~np.asarray(degenerate, dtype=bool)
    th = np.asarray(theta)[nd]
    idx = np.asarray(index)[nd].astype(np.int64)
    v = np.asarray(V)[nd]
    ev = np.asarray(eig)[nd]
    logdet = np.sum(np.log(np.abs(ev)), axis=1)
    det_root = np.exp(logdet / N)
    out = dict(energy_density=v / N, index_density=idx / (N - 1), det_root=det_root,
               index=idx, histogram=np.bincount(idx, minlength=N - 1))
    if v.size:
        g = int(np.argmin(v))
        out.update(global_min_V=float(v[g]), global_min_theta=th[g],
                   global_min_kind=config_kind(th[g], N))
        d = int(np.argmin(det_root))
        out.update(min_det_root=float(det_root[d]), min_det_theta=th[d],
                   min_det_kind=config_kind(th[d], N), min_det_energy_density=float(v[d] / N))
    return out


def from_result(res) -> Dict:
    """landscape() of a pipeline.SystemResult."""
    return landscape(res.N, res.theta, res.index, res.V, res.eig, res.degenerate)
