"""Comparison of stationary-point sets given by angles (modulo 2 pi)."""
import numpy as np


def match_sets(theta_a, idx_a, theta_b, idx_b, tol=1e-10):
    """Assert that two sets of stationary points coincide: same size, every
    point of b within tol (max angular distance mod 2 pi) of its partner in a,
    same Hessian index.  Returns the largest angular distance."""
    theta_a = np.asarray(theta_a, dtype=np.float64)
    theta_b = np.asarray(theta_b, dtype=np.float64)
    assert theta_a.shape == theta_b.shape, (theta_a.shape, theta_b.shape)
    if theta_b.size == 0:
        return 0.0
    key = lambda th: (np.round(np.cos(th), 6) + 2.0) * 8.0 + np.round(np.sin(th), 6)
    oa = np.lexsort(key(theta_a).T[::-1])
    ob = np.lexsort(key(theta_b).T[::-1])
    d = np.abs(np.angle(np.exp(1j * (theta_a[oa] - theta_b[ob]))))
    err = float(np.max(d))
    assert err < tol, err
    assert np.array_equal(np.asarray(idx_a)[oa], np.asarray(idx_b)[ob])
    return err
