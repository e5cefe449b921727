"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: they use the paper's printed
numbers (tests/golden/), closed-form homotopy paths, finite differences,
numpy's library solvers, closed-form stationary points and Hessian spectra,
Morse theory and an independent brute-force search.
"""
import functools
import json
import math
import os

import numpy as np
import pytest

import oracle
import workload
from tests import _bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


@functools.lru_cache(maxsize=None)
def _solve(kind, N, param, gseed=0, jseed=None):
    if kind == "clean":
        J = workload.clean_ring_J(N, param)
    elif kind == "paper":
        J = workload.paper_ring_J(N, param)
    else:
        J = workload.disordered_ring_J(N, param, np.random.default_rng(jseed))
    return J, oracle.find_all_sps(J, workload.gamma_from_seed(gseed))


def _branch_sqrt(w_of_t, ts, start):
    """Continuous branch of sqrt(w(t)) from sqrt(w(0)) = start on a fine grid."""
    grid = np.linspace(0.0, 1.0, 200001)
    w = w_of_t(grid)
    r = np.sqrt(w.astype(np.complex128))
    out = np.empty_like(r)
    cur = start
    for i in range(grid.size):
        c = r[i] if abs(r[i] - cur) <= abs(-r[i] - cur) else -r[i]
        out[i] = c
        cur = c
    return np.interp(ts, grid, out.real) + 1j * np.interp(ts, grid, out.imag)


# ---------------------------------------------------------------------------
# Tracker: closed-form paths
# ---------------------------------------------------------------------------

def test_univariate_paper_example():
    g = _golden("univariate.json")
    s = oracle.System(a=[g["P"]["a"]], c=[g["P"]["c"]])
    gamma = workload.gamma_from_seed(0)
    r = s.track(gamma, [0, 1])
    assert list(r["status"]) == [oracle.ST_REACHED] * 2
    z, _, _ = s.refine(r["z"])
    ends = sorted(z[:, 0].real)
    printed = g["printed_re"]
    assert abs(ends[1] - printed) < 0.5 * 10 ** -g["printed_digits"]
    assert abs(ends[0] + printed) < 0.5 * 10 ** -g["printed_digits"]
    assert np.all(np.abs(z.imag) <= g["printed_im"])
    # start x = +1 ends at +sqrt(5), x = -1 at -sqrt(5)  (x -> -x symmetry of H)
    assert z[0, 0].real > 0 and z[1, 0].real < 0


@pytest.mark.parametrize("predictor", [0, 1])
def test_univariate_path_closed_form(predictor):
    """H = gamma(1-t)(x^2-1) + t(x^2-5) gives x(t)^2 = ((1-t)gamma+5t)/((1-t)gamma+t)."""
    s = oracle.System(a=[1.0], c=[5.0])
    gamma = workload.gamma_from_seed(3)
    w = lambda t: ((1 - t) * gamma + 5 * t) / ((1 - t) * gamma + t)
    ts = np.array([0.1, 0.3, 0.5, 0.7, 0.9, 1.0])
    opts = oracle.TrackOpts(predictor=predictor, hmax=0.01 if predictor else 0.05)
    for pid, start in ((0, 1.0), (1, -1.0)):
        ref = _branch_sqrt(w, ts, start)
        for t_end, zref in zip(ts, ref):
            r = s.track(gamma, [pid], oracle.TrackOpts(**{**opts.__dict__, "t_end": float(t_end)}))
            assert r["status"][0] == oracle.ST_REACHED
            assert r["t"][0] == t_end
            assert abs(r["z"][0, 0] - zref) < 1e-9 * (1 + abs(zref))


def test_separable_paths_closed_form():
    """F_k = a_k z_k^2 - c_k: every coordinate follows its own univariate path,
    so each of the 2^n paths ends at (+-sqrt(c_k/a_k)) with the sign fixed by
    the continuous branch from its start sign."""
    a = np.array([1.0, 2.0, 0.5])
    c = np.array([3.0, -1.0, 2.0])
    s = oracle.System(a=a, c=c)
    gamma = workload.gamma_from_seed(5)
    r = s.track(gamma)
    assert np.all(r["status"] == oracle.ST_REACHED)
    for pid in range(8):
        for k in range(3):
            start = -1.0 if (pid >> k) & 1 else 1.0
            w = lambda t, k=k: ((1 - t) * gamma + t * c[k]) / ((1 - t) * gamma + t * a[k])
            ref = _branch_sqrt(w, np.array([1.0]), start)[0]
            assert abs(r["z"][pid, k] - ref) < 1e-9
    # the 8 endpoints are the 8 distinct roots
    ends = np.round(r["z"], 8)
    assert len({tuple(e) for e in ends}) == 8


def test_separable_divergence():
    """a_k = 0 leaves Q's z_k^2 term alone: z_k^2 = 1 + t c_k / ((1-t) gamma)
    goes to infinity as t -> 1 (a surplus path, section 'NPHC method')."""
    s = oracle.System(a=[1.0, 0.0], c=[2.0, 1.0])
    gamma = workload.gamma_from_seed(1)
    r = s.track(gamma)
    for pid in range(4):
        assert r["status"][pid] in (oracle.ST_DIVERGED, oracle.ST_STALLED, oracle.ST_FAIL_MINSTEP)
        # along the way z_2 follows its closed form
    r2 = s.track(gamma, [0], oracle.TrackOpts(t_end=0.999))
    ref = np.sqrt(1 + 0.999 * 1.0 / ((1 - 0.999) * gamma))
    assert abs(abs(r2["z"][0, 1]) - abs(ref)) < 1e-7 * abs(ref)


# ---------------------------------------------------------------------------
# System evaluation and linear algebra
# ---------------------------------------------------------------------------

def _rand_z(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_jacobian_matches_finite_differences(N):
    rng = np.random.default_rng(N)
    J = workload.disordered_ring_J(N, 1.0, rng)
    s = oracle.System(J)
    z = _rand_z(rng, s.n)
    A = s.Pz(z)
    h = 1e-6
    for j in range(s.n):
        e = np.zeros(s.n, complex)
        e[j] = h
        fd = (s.P(z + e) - s.P(z - e)) / (2 * h)
        assert np.allclose(A[:, j], fd, atol=1e-8, rtol=1e-7)
    gamma = workload.gamma_from_seed(2)
    t = 0.37
    H, Ht, Hz = s.H(gamma, z, t)
    Hp = s.H(gamma, z, t + h)[0]
    Hm = s.H(gamma, z, t - h)[0]
    assert np.allclose(Ht, (Hp - Hm) / (2 * h), atol=1e-8, rtol=1e-7)
    for j in range(s.n):
        e = np.zeros(s.n, complex)
        e[j] = h
        fd = (s.H(gamma, z + e, t)[0] - s.H(gamma, z - e, t)[0]) / (2 * h)
        assert np.allclose(Hz[:, j], fd, atol=1e-8, rtol=1e-7)
    # H at t = 0 is gamma * (z_k^2 - 1), at t = 1 it is P
    assert np.allclose(s.H(gamma, z, 0.0)[0], gamma * (z * z - 1))
    assert np.allclose(s.H(gamma, z, 1.0)[0], s.P(z))


def test_target_system_is_the_angle_gradient():
    """On the real circle points, the gradient rows of P equal dV/dtheta
    computed from finite differences of V (eq. (1) is the stationary
    equation)."""
    rng = np.random.default_rng(11)
    N = 6
    J = workload.disordered_ring_J(N, 0.8, rng)
    s = oracle.System(J)
    th = rng.uniform(-np.pi, np.pi, N - 1)
    z = np.concatenate([np.cos(th), np.sin(th)]).astype(complex)
    F = s.P(z)
    full = lambda t: np.append(t, 0.0)
    iu = np.triu_indices(N, 1)
    V = lambda t: np.sum(J[iu] * (1 - np.cos(full(t)[iu[0]] - full(t)[iu[1]])))
    h = 1e-6
    fd = np.array([(V(th + h * np.eye(N - 1)[k]) - V(th - h * np.eye(N - 1)[k])) / (2 * h)
                   for k in range(N - 1)])
    assert np.allclose(F[: N - 1].real, fd, atol=1e-8)
    assert np.allclose(F[N - 1:], 0, atol=1e-14)


@pytest.mark.parametrize("n", [1, 2, 5, 13, 18, 24])
def test_solve_matches_numpy(n):
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    assert np.allclose(oracle.solve(A, b), np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    # a permuted identity has zeros on the diagonal: needs pivoting
    P = np.eye(n)[rng.permutation(n)].astype(complex)
    assert np.allclose(oracle.solve(P, b), P.T @ b)


def test_solve_rejects_singular():
    with pytest.raises(np.linalg.LinAlgError):
        oracle.solve(np.zeros((3, 3), complex), np.ones(3, complex))


def test_bilinear_bound_dominates_sampled_second_derivative():
    """gamma_hat uses sup ||D^2 P(u,v)/2|| <= sqrt(||Jt||_F^2 + 4m)/2; check the
    bound against D^2 P(u,v)/2 = (P(z+u+v) - P(z+u) - P(z+v) + P(z))/2 for a
    quadratic P, on random unit vectors."""
    rng = np.random.default_rng(4)
    for N in (3, 5, 9):
        J = workload.disordered_ring_J(N, 1.0, rng)
        s = oracle.System(J)
        B = oracle.bilinear_bound(J)
        z = _rand_z(rng, s.n)
        worst = 0.0
        for _ in range(300):
            u = _rand_z(rng, s.n); u /= np.linalg.norm(u)
            v = _rand_z(rng, s.n); v /= np.linalg.norm(v)
            d2 = (s.P(z + u + v) - s.P(z + u) - s.P(z + v) + s.P(z)) / 2
            worst = max(worst, np.linalg.norm(d2))
        # structured directions: u = v = e_{x_1} excites the constraint row
        # alone (value 1); u = e_{y_1}, v = e_{x_2} excites gradient row 1
        # with J_12 / 2 (and row 2 with -J_21 / 2)
        m = N - 1
        e = np.eye(s.n)
        for u, v in ((e[0], e[0]), (e[m], e[1]), (e[m] + e[1], e[m] + e[1])):
            d2 = (s.P(z + u + v) - s.P(z + u) - s.P(z + v) + s.P(z)) / 2
            worst = max(worst, np.linalg.norm(d2) / (np.linalg.norm(u) * np.linalg.norm(v)))
        d2 = (s.P(z + e[m] + e[1]) - s.P(z + e[m]) - s.P(z + e[1]) + s.P(z)) / 2
        assert abs(d2[0] - J[0, 1] / 2) < 1e-12 and abs(d2[1] + J[1, 0] / 2) < 1e-12
        assert worst <= B * (1 + 1e-12)


# ---------------------------------------------------------------------------
# The root set: paper counts, closed forms, brute force, invariants
# ---------------------------------------------------------------------------

def test_N3_closed_form_set():
    """N = 3 (every pair at ring distance 1): the stationary points are the
    {0, pi}^2 configurations and the two twisted states theta_k = 2 pi k n / 3."""
    J, r = _solve("paper", 3, 0.75)
    assert len(r.real_ids) == 6
    expect = [(0, 0), (0, np.pi), (np.pi, 0), (np.pi, np.pi),
              (2 * np.pi / 3, 4 * np.pi / 3), (4 * np.pi / 3, 2 * np.pi / 3)]
    wrap = lambda a: np.mod(np.asarray(a) + np.pi, 2 * np.pi) - np.pi
    got = {tuple(np.round(wrap(t), 9)) for t in r.theta}
    assert got == {tuple(np.round(wrap(e), 9)) for e in expect}
    assert list(r.histogram) == [1, 3, 2]


@pytest.mark.parametrize("N", [3, 5, 7])
def test_paper_counts(N):
    counts = _golden("paper_counts.json")["counts"]
    J, r = _solve("paper", N, 0.75)
    assert len(r.real_ids) == counts[str(N)]
    assert not np.any(r.degenerate)


@pytest.mark.slow
def test_paper_count_N9():
    counts = _golden("paper_counts.json")["counts"]
    J, r = _solve("paper", 9, 0.75)
    assert len(r.real_ids) == counts["9"]


@pytest.mark.parametrize("case", [("clean", 5, 1.0, None), ("clean", 6, 1.0, None),
                                  ("dis", 6, 1.0, 7), ("clean", 7, 2.0, None)])
def test_zero_pi_configurations_and_index(case):
    """Every theta in {0, pi}^m is stationary; its index equals the number of
    negative eigenvalues of the finite-difference Hessian of V."""
    kind, N, p, js = case
    J, r = _solve(kind, N, p, 0, js)
    m = N - 1
    keys = {tuple(np.round(np.abs(t), 7)): (i, t) for i, t in enumerate(r.theta)}
    for bits in range(2 ** m):
        th = np.array([np.pi if (bits >> k) & 1 else 0.0 for k in range(m)])
        i, _ = keys[tuple(np.round(th, 7))]
        ev = np.linalg.eigvalsh(bf.fd_hessian(J, th))
        assert r.index[i] == int(np.sum(ev < -1e-6))


def test_twisted_states_closed_form():
    """Clean ring (circulant J): theta_k = 2 pi k n / N is stationary for every
    n, and the Hessian of the full ring has eigenvalues
    mu(q) = sum_r J(r) cos(2 pi n r/N) (1 - cos(2 pi q r/N)), q = 0..N-1; fixing
    theta_N removes the q = 0 zero mode, so the index is #{q != 0: mu(q) < 0}."""
    N = 7
    J, r = _solve("clean", N, 1.0)
    wrap = lambda a: np.mod(np.asarray(a) + np.pi, 2 * np.pi) - np.pi
    table = {tuple(np.round(wrap(t), 8)): i for i, t in enumerate(r.theta)}
    Jr = J[0]
    for n in range(1, N):
        th = wrap(2 * np.pi * n * np.arange(1, N) / N)
        th[np.isclose(th, -np.pi)] = np.pi
        i = table[tuple(np.round(th, 8))]
        mu = [sum(Jr[rr] * math.cos(2 * math.pi * n * rr / N) * (1 - math.cos(2 * math.pi * q * rr / N))
                  for rr in range(1, N)) for q in range(1, N)]
        assert r.index[i] == sum(1 for x in mu if x < 0)


@pytest.mark.parametrize("case", [("clean", 4, 1.0, None), ("clean", 5, 1.0, None),
                                  ("clean", 6, 1.0, None), ("dis", 5, 1.0, 3),
                                  ("dis", 6, 1.5, 4)])
def test_bruteforce_inclusion(case):
    """Every nondegenerate stationary point that theta-space Newton finds from
    10^5 random real starts is in the homotopy result, with the same index."""
    kind, N, p, js = case
    J, r = _solve(kind, N, p, 0, js)
    th, ev = bf.theta_newton(J, 100000, seed=N)
    nondeg = np.min(np.abs(ev), axis=1) > 1e-6 * np.maximum(1, np.max(np.abs(ev), axis=1))
    ours = r.theta
    for t, e in zip(th[nondeg], ev[nondeg]):
        d = np.abs(np.angle(np.exp(1j * (ours - t[None, :]))))
        hit = np.where(np.max(d, axis=1) < 1e-6)[0]
        assert hit.size == 1, f"brute-force SP {t} missing from the homotopy set"
        assert r.index[hit[0]] == int(np.sum(e < 0))
    # and the brute force found at least the nondegenerate ones we report
    if kind != "clean" or N % 4:
        assert np.sum(nondeg) == len(r.real_ids)


@pytest.mark.parametrize("case", [("clean", 5, 1.0, None), ("clean", 6, 1.0, None),
                                  ("clean", 7, 1.0, None), ("dis", 6, 1.0, 7),
                                  ("paper", 7, 0.75, None)])
def test_invariants(case):
    """Bezout bound, residuals, Morse sum = Euler characteristic of the torus
    (0) when every real stationary point is nondegenerate, mirror closure
    theta -> -theta with equal index, and path accounting."""
    kind, N, p, js = case
    J, r = _solve(kind, N, p, 0, js)
    m = N - 1
    assert len(r.real_ids) <= 4 ** m
    assert r.z.shape[0] == 4 ** m
    ns = r.endpoint == oracle.EP_NONSINGULAR
    assert np.all(r.resid[r.real_ids] < 1e-12)
    if not np.any(r.degenerate):
        assert int(np.sum((-1) ** r.index)) == 0
    table = {tuple(np.round(t, 7)): i for i, t in enumerate(r.theta)}
    for i, t in enumerate(r.theta):
        mt = -t
        mt[np.isclose(mt, -np.pi)] = np.pi
        j = table[tuple(np.round(mt, 7))]
        assert r.index[j] == r.index[i]
    # no two nonsingular endpoints coincide (one path per isolated root)
    zn = np.round(r.z[ns], 6)
    assert len({tuple(v) for v in zn}) == int(np.sum(ns))
    # the whole solution set is closed under complex conjugation
    conj = {tuple(v) for v in np.round(np.conj(r.z[ns]), 6)}
    assert conj == {tuple(v) for v in zn}
    assert r.reality_gap[1] / max(r.reality_gap[0], 1e-300) > 1e4


def test_gamma_independence():
    J, r0 = _solve("dis", 6, 1.0, 0, 7)
    _, r1 = _solve("dis", 6, 1.0, 1, 7)
    assert np.allclose(r0.theta, r1.theta, atol=1e-10)
    assert np.array_equal(r0.index, r1.index)


def test_degenerate_family_for_four_divisible_ring():
    """Clean N = 4: the circle (a, pi, a + pi, 0) of stationary points is not
    isolated; only 6 isolated real points remain, histogram [1, 4, 0, 1]."""
    J, r = _solve("clean", 4, 1.0)
    assert len(r.real_ids) == 6
    assert list(r.histogram) == [1, 4, 0, 1]
    assert r.info["counts"]["singular"] > 0
    # the family is stationary for every a
    a = 0.37
    th = np.array([a, np.pi, a + np.pi])
    s = oracle.System(J)
    z = np.concatenate([np.cos(th), np.sin(th)]).astype(complex)
    assert np.max(np.abs(s.P(z))) < 1e-14


# ---------------------------------------------------------------------------
# Sensitivities (implicit functions)
# ---------------------------------------------------------------------------

def test_energy_sensitivity_envelope_and_fd():
    """dV/dJ_ab at a stationary point equals the partial derivative
    1 - cos(theta_a - theta_b) (the gradient term vanishes), and agrees with
    central differences of V along the re-solved point."""
    J, r = _solve("dis", 6, 1.0, 0, 7)
    N = J.shape[0]
    for k in range(min(6, len(r.real_ids))):
        z = r.z[r.real_ids[k]].real.astype(complex)
        th = np.append(r.theta[k], 0.0)
        G = oracle.denergy_dJ(J, z)
        env = 1 - np.cos(th[:, None] - th[None, :])
        np.fill_diagonal(env, 0)
        assert np.allclose(G, env, atol=1e-12)
        h = 1e-6
        for a, b in [(0, 1), (1, 3), (2, N - 1)]:
            Jp = J.copy(); Jp[a, b] += h; Jp[b, a] += h
            Jm = J.copy(); Jm[a, b] -= h; Jm[b, a] -= h
            Vp = oracle.energy_z(Jp, oracle.resolve_sp(Jp, z)).real
            Vm = oracle.energy_z(Jm, oracle.resolve_sp(Jm, z)).real
            fd = (Vp - Vm) / (2 * h)
            assert abs(fd - G[a, b]) <= 1e-8 * max(1.0, abs(G[a, b])) + 1e-9


def test_coordinate_sensitivity_fd():
    """A non-stationary objective (one coordinate of the stationary point):
    the implicit-function derivative matches central differences."""
    J, r = _solve("dis", 5, 1.0, 0, 3)
    # a non-collinear point ({0, pi} configurations do not move with J)
    far = np.max(np.abs(np.sin(r.theta)), axis=1) > 0.3
    k = int(np.where(far)[0][0])
    z = r.z[r.real_ids[k]].real.astype(complex)
    G = oracle.dcoord_dJ(J, z, 1)
    h = 1e-6
    worst = 0.0
    for a, b in oracle.coupling_pairs(J.shape[0]):
        Jp = J.copy(); Jp[a, b] += h; Jp[b, a] += h
        Jm = J.copy(); Jm[a, b] -= h; Jm[b, a] -= h
        fd = (oracle.resolve_sp(Jp, z)[1] - oracle.resolve_sp(Jm, z)[1]).real / (2 * h)
        worst = max(worst, abs(fd - G[a, b]) / max(1.0, abs(G[a, b])))
    assert worst < 1e-7
    assert np.max(np.abs(G)) > 1e-3
