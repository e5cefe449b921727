"""The paper's own instances at full scale: the power-law XY ring at
alpha = 0.75 with its normalisation K, theta_N = 0.  The paper (section "A
First Application") reports 4774 stationary points for N = 11 (1,048,576
paths) and 24830 for N = 13 (16,777,216 paths).  Checked here:
  * the count of certified real nondegenerate stationary points equals the
    paper's, and the Morse sum of (-1)^index over them is 0 (the Euler
    characteristic of the torus the angles live on);
  * per-path parity on random path ids that the oracle tracks one by one
    (the set of ids ending at a nonsingular root is identical, roots agree
    to 1e-9);
  * for N = 11, the whole real set (angles, indices) against the oracle's
    stored result when tests/golden/oracle_paper11.json is present."""
import json
import os

import numpy as np
import pytest

import oracle
import workload
from tests._match import match_sets

pytestmark = pytest.mark.gpu
PAPER = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_counts.json")))
GOLDEN11 = os.path.join(os.path.dirname(__file__), "golden", "oracle_paper11.json")


def _run(N, precision):
    import torch
    from paper_1104_5497_amd import pipeline
    J = workload.paper_ring_J(N, PAPER["alpha"])
    gamma = workload.gamma_from_seed(0)
    batch = pipeline.Batch([J], [gamma])
    b = pipeline.run(batch, pipeline.Options(precision=precision))
    torch.cuda.synchronize()
    res = pipeline.collect(batch, b)
    return J, gamma, res["systems"][0], b, 2 * (N - 1)


def _sampled_paths(J, gamma, b, n, k, seed):
    import torch
    P = b.endpoint.numel()
    ids = np.sort(np.random.default_rng(seed).choice(P, k, replace=False))
    it = torch.from_numpy(ids).to(b.z.device)
    zp = b.z[:, it].cpu().numpy()
    ep = np.full(P, -1)
    ep[ids] = b.endpoint[it].cpu().numpy()
    z_g = (zp[0:2 * n:2] + 1j * zp[1:2 * n:2]).T
    sys_ = oracle.System(J)
    tr = sys_.track(gamma, ids)
    ep_o, _, _ = oracle._classify_endpoints(sys_, tr["z"], tr["t"], tr["status"], oracle.PostOpts())
    ns_g = ep[ids] == 10
    ns_o = ep_o == oracle.EP_NONSINGULAR
    assert np.array_equal(ns_g, ns_o), ids[ns_g != ns_o]
    if ns_g.any():
        scale = np.maximum(1.0, np.max(np.abs(tr["z"][ns_g]), axis=1))
        err = np.max(np.abs(z_g[ns_g] - tr["z"][ns_g]), axis=1) / scale
        assert err.max() < 1e-9, err.max()


def _check_counts(s, N):
    from paper_1104_5497_amd import landscape
    nd = ~s.degenerate
    assert int(nd.sum()) == PAPER["counts"][str(N)]
    assert int(np.sum((-1) ** s.index[nd].astype(np.int64))) == 0
    # the paper's landscape observations: global minimum theta = 0 (V = 0),
    # smallest |det H|^(1/N) at a {0, pi} or twisted configuration
    L = landscape.from_result(s)
    assert L["global_min_kind"] == "zero_pi" and abs(L["global_min_V"]) < 1e-10
    assert np.allclose(L["global_min_theta"], 0.0, atol=1e-9)
    assert L["min_det_kind"] in ("zero_pi", "twisted"), L["min_det_theta"]
    return L


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_paper_ring11(precision):
    print(f"paper ring N=11 {precision}", flush=True)
    J, gamma, s, b, n = _run(11, precision)
    L = _check_counts(s, 11)
    _sampled_paths(J, gamma, b, n, 128, 5)
    if os.path.exists(GOLDEN11):
        g = json.load(open(GOLDEN11))["rings"][0]
        nd = ~s.degenerate
        assert s.histogram.tolist() == g["histogram"]
        match_sets(s.theta[nd], s.index[nd], np.array(g["theta"]), np.array(g["index"]))
        # |det H|^(1/N) from the GPU's eigenvalues against numpy's determinant
        # of the Hessian at the oracle's angles (as multisets)
        dets = np.array([abs(np.linalg.det(oracle.hessian_theta(J, np.array(th))))
                         for th in g["theta"]]) ** (1.0 / 11)
        assert np.allclose(np.sort(L["det_root"]), np.sort(dets), rtol=1e-8)


def test_paper_ring13():
    print("paper ring N=13 fp32", flush=True)
    J, gamma, s, b, n = _run(13, "fp32")
    _check_counts(s, 13)
    _sampled_paths(J, gamma, b, n, 48, 6)
