"""Brute-force stationary points of V(theta) = sum_{i<k} J_ik (1 - cos(theta_i - theta_k)).

An independent check of the oracle's completeness (the paper's Newton-Raphson
from random guesses, section "Introduction"): Newton's method directly in the
angles theta_1..theta_m (theta_N = 0) from many random real starts.  It can
miss stationary points, so it only gives a lower bound on the set; every
nondegenerate point it finds must be in the homotopy result.
"""
import numpy as np


def _grad_hess(J, th):
    K, m = th.shape
    full = np.concatenate([th, np.zeros((K, 1))], axis=1)
    D = full[:, :, None] - full[:, None, :]
    S = J[None] * np.sin(D)
    C = J[None] * np.cos(D)
    g = S.sum(axis=2)[:, :m]
    Hs = -C
    idx = np.arange(J.shape[0])
    Hs[:, idx, idx] = C.sum(axis=2) - C[:, idx, idx]
    return g, Hs[:, :m, :m]


def theta_newton(J, n_starts, seed=0, iters=80, tol=1e-11, batch=20000):
    """Return (theta (R, m) wrapped to (-pi, pi], eigenvalues (R, m)) of the
    distinct converged stationary points."""
    J = np.asarray(J, dtype=np.float64)
    m = J.shape[0] - 1
    rng = np.random.default_rng(seed)
    found = []
    for b0 in range(0, n_starts, batch):
        K = min(batch, n_starts - b0)
        th = rng.uniform(-np.pi, np.pi, size=(K, m))
        live = np.arange(K)
        for _ in range(iters):
            g, H = _grad_hess(J, th[live])
            done = np.max(np.abs(g), axis=1) < 1e-13
            live, g, H = live[~done], g[~done], H[~done]
            if live.size == 0:
                break
            try:
                step = np.linalg.solve(H, g[..., None])[..., 0]
            except np.linalg.LinAlgError:
                step = np.linalg.solve(H + 1e-12 * np.eye(m), g[..., None])[..., 0]
            step = np.nan_to_num(step, nan=0.0, posinf=0.0, neginf=0.0)
            th[live] = th[live] - np.clip(step, -1.0, 1.0)
        g, H = _grad_hess(J, th)
        ok = np.max(np.abs(g), axis=1) < tol
        found.append(th[ok])
    th = np.concatenate(found)
    th = np.mod(th + np.pi, 2 * np.pi) - np.pi
    th[np.isclose(th, -np.pi, atol=1e-9)] = np.pi
    key = np.round(th, 5)
    _, first = np.unique(key, axis=0, return_index=True)
    th = th[np.sort(first)]
    _, H = _grad_hess(J, th)
    eig = np.linalg.eigvalsh(H)
    return th, eig


def fd_hessian(J, theta, h=1e-4):
    """Central second differences of V in theta (independent of any analytic
    Hessian formula)."""
    N = J.shape[0]
    iu = np.triu_indices(N, 1)

    def V(t):
        full = np.append(t, 0.0)
        return np.sum(J[iu] * (1.0 - np.cos(full[iu[0]] - full[iu[1]])))

    m = len(theta)
    Hs = np.zeros((m, m))
    for i in range(m):
        for k in range(m):
            ei = np.zeros(m); ei[i] = h
            ek = np.zeros(m); ek[k] = h
            Hs[i, k] = (V(theta + ei + ek) - V(theta + ei - ek) - V(theta - ei + ek)
                        + V(theta - ei - ek)) / (4 * h * h)
    return Hs
