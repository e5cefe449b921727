"""Per-path parity: every homotopy path is a fixed curve once gamma is fixed,
so the HIP pipeline and the oracle must send each path id to the same
endpoint.  Compared element by element: which paths end at a nonsingular
root (exactly the same id set) and, for those, the refined root (1e-9
relative).  Paths that end elsewhere (infinity, a singular family) may be
labelled differently by the two trackers' stopping rules, so only
"nonsingular or not" is compared for them."""
import functools

import numpy as np
import pytest

import oracle
import workload

pytestmark = pytest.mark.gpu

END_NONSINGULAR = 10


def _gpu_endpoints(J, gamma, precision):
    import torch
    from paper_1104_5497_amd import pipeline
    batch = pipeline.Batch([J], [gamma])
    b = pipeline.run(batch, pipeline.Options(precision=precision))
    torch.cuda.synchronize()
    n = 2 * (J.shape[0] - 1)
    zp = b.z.cpu().numpy()
    z = (zp[0:2 * n:2] + 1j * zp[1:2 * n:2]).T
    return z, b.endpoint.cpu().numpy()


def _compare(z_g, ep_g, z_o, ep_o, ids=None):
    ns_g = ep_g == END_NONSINGULAR
    ns_o = ep_o == oracle.EP_NONSINGULAR
    diff = np.nonzero(ns_g != ns_o)[0]
    assert diff.size == 0, ("nonsingular flags differ", (ids[diff] if ids is not None else diff)[:20])
    both = np.nonzero(ns_g)[0]
    scale = np.maximum(1.0, np.max(np.abs(z_o[both]), axis=1))
    err = np.max(np.abs(z_g[both] - z_o[both]), axis=1) / scale
    assert err.size == 0 or err.max() < 1e-9, (float(err.max()), int(np.argmax(err)))
    return both.size


@functools.lru_cache(maxsize=None)
def _oracle_full(kind, N, p, jseed):
    J = _J(kind, N, p, jseed)
    return oracle.find_all_sps(J, workload.gamma_from_seed(0))


def _J(kind, N, p, jseed=None):
    if kind == "clean":
        return workload.clean_ring_J(N, p)
    if kind == "paper":
        return workload.paper_ring_J(N, p)
    return workload.disordered_ring_J(N, p, np.random.default_rng(jseed))


CASES = [("clean", 6, 1.0, None), ("paper", 7, 0.75, None), ("dis", 7, 1.3, 11)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("case", CASES)
def test_every_path_ends_where_the_oracle_ends(case, precision):
    kind, N, p, js = case
    print(f"per-path {case} {precision}", flush=True)
    J = _J(kind, N, p, js)
    ref = _oracle_full(kind, N, p, js)
    z_g, ep_g = _gpu_endpoints(J, workload.gamma_from_seed(0), precision)
    n_ns = _compare(z_g, ep_g, ref.z, ref.endpoint)
    assert n_ns == int(np.sum(ref.endpoint == oracle.EP_NONSINGULAR))


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_ring10_sampled_paths_match_oracle(precision):
    """The benchmark's workload (N = 10, 262144 paths, default launch), checked
    on 192 random path ids that the oracle tracks one by one."""
    J = workload.clean_ring_J(10, 1.0)
    gamma = workload.gamma_from_seed(0)
    print(f"ring10 sampled {precision}", flush=True)
    z_g, ep_g = _gpu_endpoints(J, gamma, precision)
    ids = np.sort(np.random.default_rng(3).choice(4 ** 9, 192, replace=False))
    sys_ = oracle.System(J)
    tr = sys_.track(gamma, ids)
    ep_o, _, _ = oracle._classify_endpoints(sys_, tr["z"], tr["t"], tr["status"], oracle.PostOpts())
    _compare(z_g[ids], ep_g[ids], tr["z"], ep_o, ids)


@pytest.mark.parametrize("case", CASES)
def test_lane_group_tracker_matches_oracle(case):
    """The float64 tracker with a group of 16 lanes per path (used for the
    last, long paths of a launch and for re-tracks) run on every path from
    t = 0: each path ends at the oracle's root."""
    import torch
    from paper_1104_5497_amd import _lib as L, pipeline
    kind, N, p, js = case
    print(f"lane-group per-path {case}", flush=True)
    J = _J(kind, N, p, js)
    ref = _oracle_full(kind, N, p, js)
    batch = pipeline.Batch([J], [workload.gamma_from_seed(0)])
    to = L.default_track_opts(L.NPHC_FP64).copy(lanes_per_path=16)
    b = pipeline.run(batch, pipeline.Options(precision="fp64", track=to, tail_group=False))
    torch.cuda.synchronize()
    n = 2 * (N - 1)
    zp = b.z.cpu().numpy()
    z = (zp[0:2 * n:2] + 1j * zp[1:2 * n:2]).T
    _compare(z, b.endpoint.cpu().numpy(), ref.z, ref.endpoint)
