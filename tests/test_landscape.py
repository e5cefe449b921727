"""Landscape analytics (paper, "A First Application", Figs. 1-3) on the
oracle's stationary points: the configuration classifier on closed forms,
|det H|^(1/N) from the Hessian eigenvalues against numpy's determinant of
the Hessian, and the paper's two observations (global minimum at theta = 0
with V = 0; smallest |det H|^(1/N) at a {0, pi} or twisted configuration)."""
import math

import numpy as np
import pytest

import oracle
import workload
from paper_1104_5497_amd import landscape as LS


def test_config_kind_closed_forms():
    N = 7
    assert LS.config_kind(np.zeros(N - 1), N) == "zero_pi"
    assert LS.config_kind(np.array([math.pi, 0, -math.pi, 0, math.pi, 0.0]), N) == "zero_pi"
    for k in (1, 2, 3):
        th = LS._wrap(2 * math.pi * k * np.arange(1, N) / N)
        assert LS.config_kind(th, N) == "twisted", k
    rng = np.random.default_rng(0)
    assert LS.config_kind(rng.uniform(-3, 3, N - 1), N) == "other"
    th = LS._wrap(2 * math.pi * np.arange(1, N) / N)
    th[2] += 1e-3
    assert LS.config_kind(th, N) == "other"


@pytest.mark.parametrize("N", [5, 7])
def test_paper_observations_on_oracle_sets(N):
    J = workload.paper_ring_J(N, 0.75)
    res = oracle.find_all_sps(J, workload.gamma_from_seed(0))
    L = LS.landscape(N, res.theta, res.index, res.V, res.eig, res.degenerate)
    # |det H|^(1/N) from the eigenvalues = numpy's determinant of the Hessian
    nd = ~res.degenerate
    dets = np.array([abs(np.linalg.det(oracle.hessian_theta(J, th))) for th in res.theta[nd]])
    assert np.allclose(L["det_root"], dets ** (1.0 / N), rtol=1e-9)
    assert L["global_min_kind"] == "zero_pi"
    assert np.allclose(L["global_min_theta"], 0.0, atol=1e-9) and abs(L["global_min_V"]) < 1e-12
    assert L["min_det_kind"] in ("zero_pi", "twisted")
    assert int(L["histogram"].sum()) == int(nd.sum())
