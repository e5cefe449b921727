"""The tracker's per-lane linear solve (xy_lane.hpp: the structured reduction
of the Newton / Davidenko system to an m x m complex system, eliminated with
threshold pivoting in tracking solves), built for the host, against numpy's
dense solve of the oracle's H_z (paper, section "NPHC method": the corrector
solves H_z d = -H, the predictor's tangent H_z dz/dt = -H_t).  Also eval_F
against the oracle's F.  CPU only: the same template code runs in the
kernels."""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "solve_shim.cpp")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = str(tmp_path_factory.mktemp("shim") / "libsolve_shim.so")
    r = subprocess.run([HIPCC, "-O0", "-w", "-std=c++17", "-fPIC", "-shared", "--cuda-host-only",
                        "-o", out, SRC], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    lib = ctypes.CDLL(out)
    vp, dbl = ctypes.c_void_p, ctypes.c_double
    lib.shim_solve.argtypes = [ctypes.c_int, ctypes.c_int, vp, dbl, dbl, dbl, ctypes.c_int, vp, vp,
                               vp, vp]
    lib.shim_solve.restype = ctypes.c_int
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _il(v):
    """complex vector -> interleaved float64"""
    out = np.empty(2 * v.size)
    out[0::2], out[1::2] = v.real, v.imag
    return out


def _solve(shim, prec, J, gamma, t, newton, z, rhs=None):
    m = J.shape[0] - 1
    d = np.zeros(4 * m)
    F = np.zeros(4 * m)
    rc = shim.shim_solve(prec, m, _ptr(np.ascontiguousarray(J)), gamma.real, gamma.imag, t,
                         int(newton), _ptr(_il(z)), _ptr(None if rhs is None else _il(rhs)),
                         _ptr(d), _ptr(F))
    return rc, d[0::2] + 1j * d[1::2], F[0::2] + 1j * F[1::2]


def _cases(seed, count):
    rng = np.random.default_rng(seed)
    for k in range(count):
        N = int(rng.integers(3, 14))
        J = workload.disordered_ring_J(N, float(rng.uniform(0.5, 2.0)), rng) if k % 2 else \
            workload.clean_ring_J(N, float(rng.uniform(0.5, 2.0)))
        m = N - 1
        z = (rng.normal(size=2 * m) + 1j * rng.normal(size=2 * m)) * rng.uniform(0.3, 3.0)
        t = float(rng.uniform(0.02, 0.98))
        yield N, J, z, t


@pytest.mark.parametrize("prec,tol", [(0, 1e-14), (1, 2e-6)])
def test_structured_solve_matches_dense(shim, prec, tol):
    """d from the structured solve equals numpy's solve of the oracle's dense
    H_z: the error relative to |d|, divided by cond(H_z), stays below tol.
    Measured maxima on these cases: 1.9e-16 (float64) and 6.8e-8 (float32,
    about its unit roundoff); the tolerances leave a factor of 30 to 50 for
    the growth that threshold pivoting allows."""
    gamma = workload.gamma_from_seed(0)
    worst = 0.0
    n_cases = 0
    for N, J, z, t in _cases(11 + prec, 120):
        S = oracle.System(J)
        H, Ht, Hz = S.H(gamma, z, t)
        cond = np.linalg.cond(Hz)
        if cond > 1e5:
            continue
        for newton, rhs in ((True, -H), (False, -Ht)):
            rc, d, _ = _solve(shim, prec, J, gamma, t, newton, z)
            assert rc == 0
            want = np.linalg.solve(Hz, rhs)
            err = np.max(np.abs(d - want)) / np.max(np.abs(want)) / cond
            worst = max(worst, err)
            assert err < tol, (N, t, newton, err, cond)
            n_cases += 1
    assert n_cases >= 150


def test_external_rhs_and_target_system(shim):
    """With a given right-hand side b the solve returns H_z^{-1} b; at t = 1
    (H = F) a unit right-hand side gives a column of F_z^{-1}; eval_F equals
    the oracle's F."""
    gamma = workload.gamma_from_seed(0)
    rng = np.random.default_rng(5)
    for N, J, z, t in _cases(7, 60):
        S = oracle.System(J)
        n = 2 * (N - 1)
        b = rng.normal(size=n) + 1j * rng.normal(size=n)
        _, _, Hz = S.H(gamma, z, t)
        if np.linalg.cond(Hz) > 1e5:
            continue
        rc, d, F = _solve(shim, 0, J, gamma, t, True, z, b)
        assert rc == 0
        want = np.linalg.solve(Hz, b)
        assert np.max(np.abs(d - want)) <= 1e-10 * np.max(np.abs(want)) * np.linalg.cond(Hz)
        assert np.allclose(F, S.P(z), rtol=0, atol=1e-12 * max(1.0, np.max(np.abs(z))) ** 2)
        j = int(rng.integers(n))
        e = np.zeros(n, complex)
        e[j] = 1.0
        Fz = S.Pz(z)
        if np.linalg.cond(Fz) > 1e5:
            continue
        rc, col, _ = _solve(shim, 0, J, gamma, 1.0, True, z, e)
        assert rc == 0
        want = np.linalg.solve(Fz, e)
        assert np.max(np.abs(col - want)) <= 1e-10 * np.max(np.abs(want)) * np.linalg.cond(Fz)


def test_singular_system_is_reported(shim):
    """At t = 1 and z = 0 the reduced system vanishes: the solve reports
    failure instead of returning numbers."""
    J = workload.clean_ring_J(6, 1.0)
    z = np.zeros(10, complex)
    for prec in (0, 1):
        rc, d, _ = _solve(shim, prec, J, workload.gamma_from_seed(0), 1.0, True, z)
        assert rc == 1
