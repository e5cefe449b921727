"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.  Real stationary points must agree exactly as sets
(same count, same Hessian indices) and to 1e-10 in the angles."""
import functools

import numpy as np
import pytest

import oracle
import workload
from tests._match import match_sets

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _oracle(kind, N, p, gseed=0, jseed=None):
    J = _J(kind, N, p, jseed)
    return oracle.find_all_sps(J, workload.gamma_from_seed(gseed))


def _J(kind, N, p, jseed=None):
    if kind == "clean":
        return workload.clean_ring_J(N, p)
    if kind == "paper":
        return workload.paper_ring_J(N, p)
    return workload.disordered_ring_J(N, p, np.random.default_rng(jseed))


def _gpu(J, gamma, precision):
    import torch
    from paper_1104_5497_amd import pipeline
    res = pipeline.find_all_sps(J, gamma, precision=precision)
    torch.cuda.synchronize()
    return res


def _compare(gpu, ref, tol=1e-10):
    assert gpu.theta.shape == ref.theta.shape, (gpu.theta.shape, ref.theta.shape)
    if ref.theta.size:
        match_sets(gpu.theta, gpu.index, ref.theta, ref.index, tol)
        assert int(gpu.degenerate.sum()) == int(ref.degenerate.sum())
        assert np.max(np.abs(np.sort(gpu.V) - np.sort(ref.V))) < 1e-10 * max(1.0, np.max(np.abs(ref.V)))
        ev_g = np.sort(gpu.eig.ravel())
        ev_r = np.sort(ref.eig.ravel())
        assert np.max(np.abs(ev_g - ev_r)) < 1e-8 * max(1.0, np.max(np.abs(ev_r)))


CASES = [("paper", 3, 0.75, None), ("clean", 4, 1.0, None), ("paper", 5, 0.75, None),
         ("clean", 6, 1.0, None), ("dis", 6, 1.0, 7), ("paper", 7, 0.75, None),
         ("dis", 7, 1.3, 11)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES)
def test_real_sps_match_oracle(case, precision):
    kind, N, p, js = case
    print(f"case {case} {precision}", flush=True)
    J = _J(kind, N, p, js)
    ref = _oracle(kind, N, p, 0, js)
    res = _gpu(J, workload.gamma_from_seed(0), precision)
    _compare(res["systems"][0], ref)
    assert sum(res["endpoint_counts"].values()) == 4 ** (N - 1)
