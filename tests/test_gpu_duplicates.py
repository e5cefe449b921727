"""The path-jump check (nphc_mark_duplicates) against a brute-force all-pairs
comparison on the CPU: endpoints of a real run with planted coincidences
(exact copies, offsets of 0.4 tol that must be caught, offsets of 3 tol that
must not), in all-pairs mode and in probe mode."""
import ctypes

import numpy as np
import pytest

import workload

pytestmark = pytest.mark.gpu
TOL = 1e-8


def _brute(zp, items, tol):
    """Items (among `items`) with another item within tol in every plane."""
    Z = zp[:, items].T
    marked = set()
    for a in range(len(items)):
        d = np.max(np.abs(Z[a + 1:] - Z[a]), axis=1)
        for b in np.nonzero(d < tol)[0]:
            marked.add(int(items[a]))
            marked.add(int(items[a + 1 + b]))
    return marked


def _setup():
    import torch
    from paper_1104_5497_amd import pipeline
    J = workload.disordered_ring_J(7, 1.3, np.random.default_rng(11))
    batch = pipeline.Batch([J], [workload.gamma_from_seed(0)])
    b = pipeline.run(batch, pipeline.Options(precision="fp64"))
    torch.cuda.synchronize()
    return batch, b


def _plant(b, rng):
    import torch
    from paper_1104_5497_amd import _lib as L
    ep = b.endpoint.cpu().numpy()
    ns = np.nonzero(ep == L.END_NONSINGULAR)[0]
    pick = rng.choice(ns, 24, replace=False)
    src, near, far = pick[:8], pick[8:16], pick[16:24]
    zp = b.z.cpu().numpy().copy()
    n2 = zp.shape[0]
    for i, (a, c) in enumerate(zip(src, near)):
        zp[:, c] = zp[:, a]
        if i % 2:                          # a small offset in one plane
            zp[i % n2, c] += 0.4 * TOL
    for i, (a, c) in enumerate(zip(src, far)):
        if i % 2 == 0:
            zp[:, c] = zp[:, a]
            zp[(i + 1) % n2, c] += 3.0 * TOL  # beyond the tolerance
    b.z.copy_(torch.from_numpy(zp))
    return zp, ns, near


def _run(batch, b, probe=None):
    import torch
    from paper_1104_5497_amd import _lib as L
    dev = b.z.device
    ns_t = torch.nonzero(b.endpoint == L.END_NONSINGULAR).flatten().to(torch.int64)
    ids = torch.zeros(batch.num_items, dtype=torch.int64, device=dev)
    ids[:ns_t.numel()] = ns_t
    cnt = torch.tensor([ns_t.numel(), 0, 0], dtype=torch.int64, device=dev)
    if probe is not None:
        pr = torch.zeros(max(1, len(probe)), dtype=torch.int64, device=dev)  # never a null pointer
        pr[:len(probe)] = torch.from_numpy(np.sort(probe).astype(np.int64)).to(dev)
        cnt[2] = len(probe)
    ws = torch.zeros(int(L.lib().nphc_duplicates_workspace_size(batch.num_items)),
                     dtype=torch.uint8, device=dev)
    p = lambda x: ctypes.c_void_p(x.data_ptr())
    L.check(L.lib().nphc_mark_duplicates(
        ctypes.byref(batch.c), p(ids), batch.num_items, ctypes.c_void_p(cnt.data_ptr()),
        p(pr) if probe is not None else None,
        ctypes.c_void_p(cnt.data_ptr() + 16) if probe is not None else None,
        TOL, p(b.z), batch.num_items, p(b.endpoint), ctypes.c_void_p(cnt.data_ptr() + 8),
        p(ws), ws.numel(), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
        "nphc_mark_duplicates")
    torch.cuda.synchronize()
    ep = b.endpoint.cpu().numpy()
    return set(np.nonzero(ep == L.END_DUPLICATE)[0].tolist()), int(cnt[1])


def test_all_pairs_match_brute_force():
    batch, b = _setup()
    zp, ns, near = _plant(b, np.random.default_rng(1))
    want = _brute(zp, ns, TOL)
    assert len(want) >= 16                    # the 8 planted pairs at least
    got, nmark = _run(batch, b)
    assert got == want
    assert nmark == len(want)


def test_probe_mode_checks_only_probes():
    batch, b = _setup()
    zp, ns, near = _plant(b, np.random.default_rng(2))
    probes = near[:3]
    want = set()
    Z = zp[:, ns].T
    for q in probes:
        d = np.max(np.abs(Z - zp[:, q]), axis=1)
        hits = [int(ns[k]) for k in np.nonzero(d < TOL)[0] if ns[k] != q]
        if hits:
            want.add(int(q))
            want.update(hits)
    assert len(want) >= 6
    got, nmark = _run(batch, b, probe=probes)
    assert got == want and nmark == len(want)


def test_empty_probe_list_does_nothing():
    batch, b = _setup()
    _plant(b, np.random.default_rng(3))
    got, nmark = _run(batch, b, probe=np.zeros(0, np.int64))
    assert got == set() and nmark == 0
