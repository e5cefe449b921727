"""Write the oracle's results for the large workloads as golden files.

Calls only oracle/ (and the seeded input generators in workload/); nothing
here comes from the HIP path.  Usage:

    python tests/golden/make_golden.py ring10 ring8 batch adjoint9 paper11

Each file holds, per ring: N, sigma, gamma, the number of certified real
nondegenerate stationary points, the Hessian-index histogram, and (unless the
ring is only summarised) their angles (15 significant digits), indices and
energies, sorted lexicographically by angle.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workload  # noqa: E402


def _ring_record(J, gamma, res, full=True, **meta):
    nd = ~res.degenerate
    rec = dict(meta, N=int(J.shape[0]), gamma=[gamma.real, gamma.imag],
               num_real=int(np.sum(nd)), num_degenerate=int(np.sum(res.degenerate)),
               histogram=res.histogram.tolist(), counts=res.info["counts"],
               unresolved_jumps=len(res.info["unresolved_jumps"]),
               max_finite_norm=float(np.max(np.abs(res.z[res.endpoint == oracle.EP_NONSINGULAR]))
                                     if np.any(res.endpoint == oracle.EP_NONSINGULAR) else 0.0))
    if full:
        rec["theta"] = [[float("%.15g" % v) for v in row] for row in res.theta[nd]]
        rec["index"] = res.index[nd].tolist()
        rec["V"] = [float("%.15g" % v) for v in res.V[nd]]
    return rec


def ring10():
    J = workload.clean_ring_J(10, 1.0)
    g = workload.gamma_from_seed(0)
    t0 = time.time()
    res = oracle.find_all_sps(J, g)
    rec = _ring_record(J, g, res, sigma=1.0, gamma_seed=0, seconds=time.time() - t0)
    steps = res.accepted + res.rejected
    rec["mean_steps"] = float(steps.mean())
    return dict(workload="clean XY ring N=10 sigma=1, gamma seed 0", rings=[rec])


def paper11():
    """The paper's N = 11 instance (alpha = 0.75, its normalisation K): the
    paper reports 4774 stationary points."""
    J = workload.paper_ring_J(11, 0.75)
    g = workload.gamma_from_seed(0)
    t0 = time.time()
    res = oracle.find_all_sps(J, g)
    rec = _ring_record(J, g, res, alpha=0.75, gamma_seed=0, seconds=time.time() - t0)
    return dict(workload="paper ring N=11 alpha=0.75, gamma seed 0", rings=[rec])


def ring8():
    rings = []
    for seed, sigma in enumerate((0.5, 1.0, 2.0)):
        J = workload.clean_ring_J(8, sigma)
        g = workload.gamma_from_seed(seed)
        res = oracle.find_all_sps(J, g)
        rings.append(_ring_record(J, g, res, sigma=sigma, gamma_seed=seed))
    return dict(workload="clean XY rings N=8, sigma 0.5/1/2, gamma seeds 0/1/2", rings=rings)


def batch():
    B = workload.batch_rings(0)
    rings = []
    for i, (J, g, s) in enumerate(zip(B.J, B.gamma, B.sigma)):
        res = oracle.find_all_sps(J, g)
        rings.append(_ring_record(J, g, res, full=(i % 16 == 0), sigma=s, ring=i))
    return dict(workload="384 disordered rings (128 each of N=5, 6, 7), batch seed 0", rings=rings)


def adjoint9():
    J = workload.disordered_ring_J(9, 1.0, np.random.default_rng(0))
    g = workload.gamma_from_seed(0)
    res = oracle.find_all_sps(J, g)
    rec = _ring_record(J, g, res, sigma=1.0, J_seed=0, gamma_seed=0)
    E, S, zs = oracle.minima_objectives(res, J)
    mins = np.where((res.index == 0) & ~res.degenerate)[0]
    gmin = int(mins[np.argmin(res.V[mins])])
    zg = res.z[res.real_ids[gmin]].real.astype(complex)
    rec["E_globalmin"] = E
    rec["S_minima"] = S
    rec["dE_dJ"] = oracle.denergy_dJ(J, zg).tolist()
    rec["dS_dJ"] = np.sum([oracle.denergy_dJ(J, z) for z in zs], axis=0).tolist()
    return dict(workload="disordered ring N=9 sigma=1, J seed 0, gamma seed 0", rings=[rec])


JOBS = {"ring10": ring10, "ring8": ring8, "batch": batch, "adjoint9": adjoint9, "paper11": paper11}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(JOBS):
        t0 = time.time()
        data = JOBS[name]()
        data["generator"] = "tests/golden/make_golden.py (oracle only)"
        with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
            json.dump(data, f, separators=(",", ":"))
        print(name, "done in %.1f s" % (time.time() - t0), flush=True)
