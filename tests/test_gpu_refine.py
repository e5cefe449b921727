"""Endpoint refinement and certification (nphc_refine_certify) on their own:
the oracle's nonsingular roots, perturbed at float32 tracking accuracy, must
come back to the roots within float64 rounding, with the certificate
quantities the oracle computes (beta and the residual equal; the Frobenius
forms of cond and alpha inside the bounds that tie them to the 2-norm forms)."""
import ctypes

import numpy as np
import pytest

import oracle
import workload

pytestmark = pytest.mark.gpu


def _refine(J, gamma, zs, lanes=1):
    import torch
    from paper_1104_5497_amd import _lib as L, pipeline
    batch = pipeline.Batch([J], [gamma])
    P, n = batch.num_items, batch.n_max
    K = zs.shape[0]
    zplanes = np.zeros((2 * n, P))
    zplanes[0::2, :K] = zs.real.T
    zplanes[1::2, :K] = zs.imag.T
    dev = batch.device
    z = torch.from_numpy(zplanes).to(dev)
    t = torch.ones(P, dtype=torch.float64, device=dev)
    status = torch.full((P,), L.PATH_DIVERGED, dtype=torch.int32, device=dev)
    status[:K] = L.PATH_REACHED
    ids = torch.arange(K, dtype=torch.int64, device=dev)
    out = {k: torch.zeros(P, dtype=torch.float64, device=dev)
           for k in ("resid", "cond", "beta", "alpha", "alpha_real")}
    endpoint = torch.zeros(P, dtype=torch.int32, device=dev)
    co = L.default_cert_opts().copy(lanes_per_item=lanes)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    L.check(L.lib().nphc_refine_certify(ctypes.byref(batch.c), p(ids), K, None, ctypes.byref(co),
                                        p(z), P, p(t), p(status), p(endpoint), p(out["resid"]),
                                        p(out["cond"]), p(out["beta"]), p(out["alpha"]),
                                        p(out["alpha_real"]), s), "nphc_refine_certify")
    torch.cuda.synchronize()
    zp = z.cpu().numpy()
    zr = (zp[0::2, :K] + 1j * zp[1::2, :K]).T
    return zr, endpoint[:K].cpu().numpy(), {k: v[:K].cpu().numpy() for k, v in out.items()}


@pytest.mark.parametrize("case", [("clean", 6, 1.0), ("dis", 7, 1.3)])
def test_refine_restores_perturbed_roots(case):
    kind, N, p = case
    J = (workload.clean_ring_J(N, p) if kind == "clean"
         else workload.disordered_ring_J(N, p, np.random.default_rng(11)))
    gamma = workload.gamma_from_seed(0)
    ref = oracle.find_all_sps(J, gamma)
    roots = ref.z[ref.endpoint == oracle.EP_NONSINGULAR]
    rng = np.random.default_rng(5)
    scale = np.maximum(1.0, np.abs(roots))
    noise = (rng.standard_normal(roots.shape) + 1j * rng.standard_normal(roots.shape)) * 1e-6 * scale
    print(f"refine {case}: {roots.shape[0]} roots", flush=True)
    z, ep, q = _refine(J, gamma, roots + noise)
    assert np.all(ep == 10), np.bincount(ep)
    sys_ = oracle.System(J)
    beta, ghat, alpha2, cond2, res = oracle.certify(sys_, roots)
    # both sides stop at rounding level: forward error ~ cond * eps
    err = np.max(np.abs(z - roots) / np.maximum(1.0, np.abs(roots)), axis=1)
    bound = np.maximum(1e-13, 1e-14 * cond2)
    assert np.all(err < bound), (float(np.max(err / bound)), float(cond2[np.argmax(err / bound)]))
    n = 2 * (N - 1)
    # beta, the next Newton step, is at rounding level: <~ cond * eps * |z|
    zmax = np.maximum(1.0, np.max(np.abs(roots), axis=1))
    assert np.all(q["beta"] < np.maximum(1e-13, 1e-14 * cond2) * zmax)
    assert np.all(q["resid"] < 1e-12 * np.maximum(1.0, np.max(np.abs(roots), axis=1) ** 2))
    # ||A||_2 ||A^-1||_2 <= ||A||_F ||A^-1||_F <= n ||A||_2 ||A^-1||_2
    assert np.all(q["cond"] >= cond2 * (1 - 1e-8)) and np.all(q["cond"] <= n * cond2 * (1 + 1e-8))
    # alpha = beta ||A^-1|| B: the GPU's Frobenius factor lies within sqrt(n) of the 2-norm one
    ok = q["beta"] > 0
    fro_over_2 = q["alpha"][ok] / q["beta"][ok] / ghat[ok]
    assert np.all(fro_over_2 >= 1 - 1e-8) and np.all(fro_over_2 <= np.sqrt(n) * (1 + 1e-8))
    # the certification decision: alpha is (rounding-level beta) x gamma-hat,
    # so it can only be compared where the oracle's alpha has a wide margin,
    # and where a 1e-6 perturbation is well inside Newton's region of
    # quadratic convergence (moderate condition number)
    clear = ((alpha2 < oracle.ALPHA0 / 100) | (alpha2 > oracle.ALPHA0 * 100)) & (cond2 < 1e6)
    assert clear.mean() > 0.9, clear.mean()
    bad = np.nonzero(clear & ((q["alpha"] < oracle.ALPHA0) != (alpha2 < oracle.ALPHA0)))[0]
    assert bad.size == 0, [(float(q["alpha"][i]), float(alpha2[i]), float(q["beta"][i]), float(beta[i]),
                            float(cond2[i]), float(q["cond"][i]), float(np.max(np.abs(roots[i]))))
                           for i in bad[:5]]


@pytest.mark.parametrize("lanes", [4, 8, 16])
def test_grouped_refinement_matches_one_lane(lanes):
    """lanes_per_item > 1 (Newton on every lane of a group, the certificate's
    2m + 1 solves split over the group) against one lane per endpoint, on
    perturbed oracle roots plus points that fail to converge: the refined
    points and the endpoint classes are identical (same Newton sequence); the
    certificate sums differ only in summation order (1e-13 relative)."""
    J = workload.disordered_ring_J(9, 1.1, np.random.default_rng(4))
    gamma = workload.gamma_from_seed(0)
    ref = oracle.find_all_sps(J, gamma)
    roots = ref.z[ref.endpoint == oracle.EP_NONSINGULAR][:300]
    rng = np.random.default_rng(9)
    noise = (rng.standard_normal(roots.shape) + 1j * rng.standard_normal(roots.shape)) * 1e-5
    junk = rng.standard_normal((37, roots.shape[1])) * 3 + 0j   # ragged tail, mostly not roots
    zs = np.concatenate([roots + noise, junk])
    print(f"grouped refinement lanes={lanes}: {zs.shape[0]} points", flush=True)
    z1, ep1, q1 = _refine(J, gamma, zs, 1)
    zg, epg, qg = _refine(J, gamma, zs, lanes)
    assert np.array_equal(ep1, epg)
    assert np.array_equal(z1, zg, equal_nan=True)
    assert np.array_equal(q1["resid"], qg["resid"], equal_nan=True)
    for k in ("cond", "beta", "alpha", "alpha_real"):
        a, b = q1[k], qg[k]
        fin = np.isfinite(a)
        assert np.array_equal(fin, np.isfinite(b)), k
        assert np.allclose(a[fin], b[fin], rtol=1e-13, atol=0), k


def test_grouped_refinement_rejects_bad_group_size():
    import torch
    from paper_1104_5497_amd import _lib as L, pipeline
    batch = pipeline.Batch([workload.clean_ring_J(5, 1.0)], [workload.gamma_from_seed(0)])
    P, n = batch.num_items, batch.n_max
    dev = batch.device
    z = torch.zeros((2 * n, P), dtype=torch.float64, device=dev)
    t = torch.ones(P, dtype=torch.float64, device=dev)
    st = torch.zeros(P, dtype=torch.int32, device=dev)
    ep = torch.zeros(P, dtype=torch.int32, device=dev)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    for bad in (2, 3, 32):
        co = L.default_cert_opts().copy(lanes_per_item=bad)
        rc = L.lib().nphc_refine_certify(ctypes.byref(batch.c), None, P, None, ctypes.byref(co),
                                         p(z), P, p(t), p(st), p(ep), None, None, None, None, None,
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert rc == L.NPHC_EINVAL
