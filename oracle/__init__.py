"""FP64 CPU oracle for NPHC on the power-law XY ring.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here is shared with the HIP
path (paper_1104_5497_amd/) and neither side imports the other.

The path tracker, the dense linear solves and the Newton refinement are plain
C (nphc_oracle.c, built with gcc); the post-processing below uses numpy's
library routines (solve, SVD, symmetric eigenvalues) as single steps.

Readings of the paper used here (the paper leaves the solver settings open):
  * statuses, tolerances and step control follow DEFAULTS below;
  * an endpoint is NONSINGULAR when the path reached t = 1, Newton on P
    leaves ||P||_inf < res_tol * max(1, ||z||_inf^2) and cond_2(P_z) < 1e10;
  * certification is the alpha-test of Smale's alpha-theory with the exact
    gamma replaced by the upper bound ||P_z^{-1}||_2 * sqrt(||Jt||_F^2 + 4m)/2
    (P is quadratic, so D^3 P = 0 and D^2 P is constant);
  * a root is real when max_k |Im z_k| <= 1e-7 (the paper's reality
    tolerance) and its real projection passes the alpha-test.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import sys
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nphc_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# path outcomes (tracking)
ST_PENDING, ST_REACHED, ST_DIVERGED, ST_FAIL_MINSTEP, ST_FAIL_MAXSTEPS, ST_FAIL_NONFINITE, ST_STALLED = range(7)
# endpoint classes (after refinement)
EP_NONSINGULAR, EP_SINGULAR, EP_DIVERGED, EP_FAIL = 10, 11, 12, 13

ALPHA0 = (13.0 - 3.0 * math.sqrt(17.0)) / 4.0  # Smale's alpha-theory constant


def build(force: bool = False) -> str:
    """Compile nphc_oracle.c into liboracle.so with gcc (-O2, C11, pthreads)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n", ctypes.c_int32), ("N", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("J", ctypes.c_void_p), ("a", ctypes.c_void_p),
                ("c", ctypes.c_void_p)]


class _Opts(ctypes.Structure):
    _fields_ = [("h0", ctypes.c_double), ("hmax", ctypes.c_double), ("hmin", ctypes.c_double),
                ("corr_tol", ctypes.c_double), ("R_inf", ctypes.c_double),
                ("t_stall", ctypes.c_double), ("t_end", ctypes.c_double),
                ("max_corr", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("predictor", ctypes.c_int32), ("pad", ctypes.c_int32)]


@dataclass
class TrackOpts:
    h0: float = 0.01
    hmax: float = 0.05
    hmin: float = 1e-13
    corr_tol: float = 1e-10
    R_inf: float = 1e8
    t_stall: float = 1.0 - 1e-6
    t_end: float = 1.0
    max_corr: int = 3
    max_steps: int = 20000
    predictor: int = 0  # 0 = RK4, 1 = Euler

    def _c(self) -> _Opts:
        return _Opts(self.h0, self.hmax, self.hmin, self.corr_tol, self.R_inf, self.t_stall,
                     self.t_end, self.max_corr, self.max_steps, self.predictor, 0)


@dataclass
class PostOpts:
    refine_iters: int = 20
    refine_tol: float = 1e-15
    res_tol: float = 1e-12        # ||P||_inf < res_tol * max(1, ||z||_inf^2)
    cond_max: float = 1e10        # cond_2(P_z) below this: nonsingular
    sing_res: float = 1e-8        # residual of a singular endpoint
    dup_tol: float = 1e-8         # two nonsingular endpoints closer than this: path jump
    div_norm: float = 1e4         # a path that stops early beyond this norm went to infinity
    real_tol: float = 1e-7        # the paper's reality tolerance
    eig_rel: float = 1e-8         # tau = eig_rel * max(1, max|lambda|)
    retrack_rounds: int = 3


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(build())
        dp, ip, i64p = ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p
        L.oracle_track.argtypes = [ctypes.POINTER(_Sys), ctypes.c_double, ctypes.c_double, i64p,
                                   ctypes.c_int64, ctypes.POINTER(_Opts), dp, dp, ip, ip, ip,
                                   ctypes.c_int]
        L.oracle_refine.argtypes = [ctypes.POINTER(_Sys), dp, ctypes.c_int64, ctypes.c_int,
                                    ctypes.c_double, ip, dp]
        L.oracle_eval_P.argtypes = [ctypes.POINTER(_Sys), dp, dp]
        L.oracle_eval_Pz.argtypes = [ctypes.POINTER(_Sys), dp, dp]
        L.oracle_eval_H.argtypes = [ctypes.POINTER(_Sys), ctypes.c_double, ctypes.c_double, dp,
                                    ctypes.c_double, dp, dp, dp]
        L.oracle_solve.argtypes = [ctypes.c_int, dp, dp, dp]
        for f in ("oracle_track", "oracle_refine", "oracle_eval_P", "oracle_eval_Pz",
                  "oracle_eval_H", "oracle_solve", "oracle_nmax"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class System:
    """A square polynomial system the oracle can track.

    kind "xy": the gauge-fixed XY ring stationary equations, eq. (1), with
    coupling matrix J (N x N); kind "sep": F_k = a_k z_k^2 - c_k."""

    def __init__(self, J: Optional[np.ndarray] = None, a=None, c=None):
        if J is not None:
            self.J = np.ascontiguousarray(J, dtype=np.float64)
            self.N = self.J.shape[0]
            if self.J.shape != (self.N, self.N):
                raise ValueError("J must be square")
            self.kind, self.n = 0, 2 * (self.N - 1)
            self.a = self.c = None
        else:
            self.a = np.ascontiguousarray(a, dtype=np.float64)
            self.c = np.ascontiguousarray(c, dtype=np.float64)
            self.kind, self.n, self.N, self.J = 1, self.a.size, 0, None
        self._s = _Sys(self.kind, self.n, self.N, 0, _ptr(self.J), _ptr(self.a), _ptr(self.c))

    @property
    def m(self) -> int:
        return self.N - 1

    # -- plain evaluations --------------------------------------------------
    def P(self, z) -> np.ndarray:
        z = np.ascontiguousarray(z, dtype=np.complex128)
        out = np.empty(self.n, np.complex128)
        lib().oracle_eval_P(ctypes.byref(self._s), _ptr(z), _ptr(out))
        return out

    def Pz(self, z) -> np.ndarray:
        z = np.ascontiguousarray(z, dtype=np.complex128)
        out = np.empty((self.n, self.n), np.complex128)
        lib().oracle_eval_Pz(ctypes.byref(self._s), _ptr(z), _ptr(out))
        return out

    def H(self, gamma: complex, z, t: float):
        z = np.ascontiguousarray(z, dtype=np.complex128)
        H = np.empty(self.n, np.complex128)
        Ht = np.empty(self.n, np.complex128)
        Hz = np.empty((self.n, self.n), np.complex128)
        lib().oracle_eval_H(ctypes.byref(self._s), gamma.real, gamma.imag, _ptr(z), t,
                            _ptr(H), _ptr(Ht), _ptr(Hz))
        return H, Ht, Hz

    # -- tracking -------------------------------------------------------------
    def track(self, gamma: complex, ids=None, opts: TrackOpts = TrackOpts(), nthreads: int = 0):
        """Track paths; returns dict(z (K,n) complex128, t, status, accepted, rejected)."""
        if ids is None:
            count = 1 << self.n
            ids_arr = None
        else:
            ids_arr = np.ascontiguousarray(ids, dtype=np.int64)
            count = ids_arr.size
        z = np.zeros((count, self.n), np.complex128)
        t = np.zeros(count, np.float64)
        st = np.zeros(count, np.int32)
        acc = np.zeros(count, np.int32)
        rej = np.zeros(count, np.int32)
        nth = nthreads or os.cpu_count() or 1
        o = opts._c()
        rc = lib().oracle_track(ctypes.byref(self._s), gamma.real, gamma.imag, _ptr(ids_arr),
                                count, ctypes.byref(o), _ptr(z), _ptr(t), _ptr(st), _ptr(acc),
                                _ptr(rej), nth)
        if rc != 0:
            raise ValueError("oracle_track rejected its arguments")
        return dict(z=z, t=t, status=st, accepted=acc, rejected=rej)

    def refine(self, z, max_iter: int = 20, tol: float = 1e-15):
        z = np.array(z, dtype=np.complex128, order="C").reshape(-1, self.n)
        it = np.zeros(z.shape[0], np.int32)
        last = np.zeros(z.shape[0], np.float64)
        lib().oracle_refine(ctypes.byref(self._s), _ptr(z), z.shape[0], max_iter, tol, _ptr(it),
                            _ptr(last))
        return z, it, last


def solve(A, b) -> np.ndarray:
    """The oracle's dense Gaussian elimination with partial pivoting."""
    A = np.ascontiguousarray(A, dtype=np.complex128)
    b = np.ascontiguousarray(b, dtype=np.complex128)
    x = np.empty(b.shape, np.complex128)
    rc = lib().oracle_solve(A.shape[0], _ptr(A), _ptr(b), _ptr(x))
    if rc != 0:
        raise np.linalg.LinAlgError("zero pivot")
    return x


# ---------------------------------------------------------------------------
# Post-processing (numpy, fp64)
# ---------------------------------------------------------------------------

def bilinear_bound(J: np.ndarray) -> float:
    """sup ||D^2 P(u,v)/2||_2 over unit u, v is at most sqrt(||Jt||_F^2 + 4m)/2,
    Jt = J restricted to the free spins: each gradient row's quadratic form has
    spectral norm ||Jt_k||_2 / 2 and each constraint row's has norm 1."""
    m = J.shape[0] - 1
    Jt = J[:m, :m]
    return 0.5 * math.sqrt(float(np.sum(Jt * Jt)) + 4.0 * m)


def certify(sys: System, z: np.ndarray):
    """alpha-test per endpoint: returns (beta, gamma_hat, alpha, cond2, resid_inf)."""
    z = np.atleast_2d(z)
    K = z.shape[0]
    beta = np.full(K, np.inf)
    ghat = np.full(K, np.inf)
    cond = np.full(K, np.inf)
    res = np.full(K, np.inf)
    B = bilinear_bound(sys.J)
    for i in range(K):
        F = sys.P(z[i])
        A = sys.Pz(z[i])
        res[i] = np.max(np.abs(F))
        s = np.linalg.svd(A, compute_uv=False)
        if s[-1] <= 0 or not np.all(np.isfinite(s)):
            continue
        cond[i] = s[0] / s[-1]
        beta[i] = np.linalg.norm(np.linalg.solve(A, F))
        ghat[i] = B / s[-1]
    return beta, ghat, beta * ghat, cond, res


def hessian_theta(J: np.ndarray, theta_free: np.ndarray) -> np.ndarray:
    """Hessian of V = sum_{i<k} J_ik (1 - cos(theta_i - theta_k)) in theta_1..theta_m
    (theta_N = 0 fixed): d2V/dth_i^2 = sum_{k != i} J_ik cos(th_i - th_k),
    d2V/dth_i dth_k = -J_ik cos(th_i - th_k)."""
    N = J.shape[0]
    th = np.append(theta_free, 0.0)
    C = np.cos(th[:, None] - th[None, :])
    W = J * C
    np.fill_diagonal(W, 0.0)
    H = -W
    H[np.diag_indices(N)] = np.sum(W, axis=1)
    return H[: N - 1, : N - 1]


def energy(J: np.ndarray, theta_free: np.ndarray) -> float:
    """V = sum_{i<k} J_ik (1 - cos(theta_i - theta_k))."""
    th = np.append(theta_free, 0.0)
    iu = np.triu_indices(J.shape[0], 1)
    return float(np.sum(J[iu] * (1.0 - np.cos(th[iu[0]] - th[iu[1]]))))


def gradient_theta(J: np.ndarray, theta_free: np.ndarray) -> np.ndarray:
    """dV/dtheta_k = sum_j J_kj sin(theta_k - theta_j), k = 1..m."""
    th = np.append(theta_free, 0.0)
    S = np.sin(th[:, None] - th[None, :])
    return np.sum(J * S, axis=1)[:-1]


@dataclass
class Result:
    N: int
    z: np.ndarray                 # (P, n) endpoints after refinement
    t: np.ndarray
    track_status: np.ndarray      # ST_*
    endpoint: np.ndarray          # EP_* per path
    accepted: np.ndarray
    rejected: np.ndarray
    resid: np.ndarray
    cond: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    real_ids: np.ndarray          # path ids of certified real nonsingular SPs, sorted by theta
    theta: np.ndarray             # (R, m)
    index: np.ndarray             # (R,)
    eig: np.ndarray               # (R, m)
    V: np.ndarray                 # (R,)
    degenerate: np.ndarray        # (R,) bool
    retracked: np.ndarray         # path ids re-tracked because of path jumps or failures
    reality_gap: tuple = (0.0, 0.0)
    info: dict = field(default_factory=dict)

    @property
    def histogram(self) -> np.ndarray:
        return np.bincount(self.index[~self.degenerate], minlength=self.N - 1)


def _classify_endpoints(sys: System, z, t, st, po: PostOpts, t_end: float = 1.0):
    """Refine endpoints and sort them into NONSINGULAR / SINGULAR / DIVERGED / FAIL."""
    K = z.shape[0]
    ep = np.full(K, EP_FAIL, np.int32)
    res = np.full(K, np.inf)
    cond = np.full(K, np.inf)
    ep[st == ST_DIVERGED] = EP_DIVERGED
    early = (st == ST_STALLED) | (st == ST_FAIL_MINSTEP) | (st == ST_FAIL_MAXSTEPS)
    with np.errstate(invalid="ignore"):
        big = ~(np.max(np.abs(z), axis=1) <= po.div_norm)
    ep[early & big] = EP_DIVERGED
    cand = np.where((st == ST_REACHED) | ((st == ST_STALLED) & ~big))[0]
    if cand.size:
        zr, _, _ = sys.refine(z[cand], po.refine_iters, po.refine_tol)
        z[cand] = zr
        for j, i in enumerate(cand):
            F = sys.P(z[i])
            res[i] = np.max(np.abs(F))
            if not np.all(np.isfinite(z[i])):
                continue
            s = np.linalg.svd(sys.Pz(z[i]), compute_uv=False)
            cond[i] = s[0] / s[-1] if s[-1] > 0 else np.inf
            zn = np.max(np.abs(z[i]))
            if st[i] == ST_REACHED and t[i] == t_end and res[i] < po.res_tol * max(1.0, zn * zn) \
                    and cond[i] < po.cond_max:
                ep[i] = EP_NONSINGULAR
            elif res[i] < po.sing_res * max(1.0, zn * zn) and cond[i] >= po.cond_max:
                ep[i] = EP_SINGULAR
    return ep, res, cond


def _jump_pairs(z: np.ndarray, ids: np.ndarray, tol: float):
    """Pairs of endpoints closer than tol in the max-norm (brute force over a
    sort on the real part of the first coordinate)."""
    if z.shape[0] < 2:
        return set()
    key = z[:, 0].real
    order = np.argsort(key, kind="stable")
    bad = set()
    for a in range(len(order)):
        i = order[a]
        for b in range(a + 1, len(order)):
            j = order[b]
            if key[j] - key[i] > tol:
                break
            if np.max(np.abs(z[i] - z[j])) < tol:
                bad.add(int(ids[i]))
                bad.add(int(ids[j]))
    return bad


def find_all_sps(J: np.ndarray, gamma: complex, topts: TrackOpts = TrackOpts(),
                 po: PostOpts = PostOpts(), nthreads: int = 0) -> Result:
    """All certified real nondegenerate stationary points of the XY ring with
    couplings J: track every path, refine, resolve path jumps by re-tracking
    with a smaller maximal step, certify, filter the real roots and classify
    them by Hessian index (paper: NPHC method; "A First Application")."""
    sys_ = System(J)
    N, m, n = sys_.N, sys_.m, sys_.n
    tr = sys_.track(gamma, None, topts, nthreads)
    z, t, st = tr["z"], tr["t"], tr["status"]
    acc, rej = tr["accepted"], tr["rejected"]
    ep, res, cond = _classify_endpoints(sys_, z, t, st, po)

    retracked = set()
    # failed paths, then path jumps: re-track with a quarter of the maximal step
    o = topts
    for rnd in range(po.retrack_rounds):
        fails = set(np.where(ep == EP_FAIL)[0].tolist())
        ns = np.where(ep == EP_NONSINGULAR)[0]
        jumps = _jump_pairs(z[ns], ns, po.dup_tol)
        todo = sorted((fails | jumps) - retracked) if rnd == 0 else sorted(fails | jumps)
        if not todo:
            break
        o = replace(o, hmax=o.hmax / 4.0, h0=min(o.h0, o.hmax / 4.0))
        ids = np.array(todo, np.int64)
        r2 = sys_.track(gamma, ids, o, nthreads)
        z[ids], t[ids], st[ids] = r2["z"], r2["t"], r2["status"]
        acc[ids] += r2["accepted"]
        rej[ids] += r2["rejected"]
        e2, r2res, r2cond = _classify_endpoints(sys_, z[ids], t[ids], st[ids], po)
        ep[ids], res[ids], cond[ids] = e2, r2res, r2cond
        retracked |= set(todo)
    ns = np.where(ep == EP_NONSINGULAR)[0]
    still = _jump_pairs(z[ns], ns, po.dup_tol)

    # certification of every nonsingular endpoint
    alpha = np.full(z.shape[0], np.inf)
    beta = np.full(z.shape[0], np.inf)
    if ns.size:
        b, g, a, c, _ = certify(sys_, z[ns])
        alpha[ns], beta[ns] = a, b

    # real filter: |Im z_k| <= real_tol for every k, and the real projection certified
    real = []
    imag_max = np.max(np.abs(z[ns].imag), axis=1) if ns.size else np.zeros(0)
    for i, im in zip(ns, imag_max):
        if im <= po.real_tol:
            _, _, a_re, _, _ = certify(sys_, z[i].real.astype(np.complex128))
            if a_re[0] < ALPHA0:
                real.append(i)
    real = np.array(real, np.int64)
    if ns.size:
        nonreal = imag_max[imag_max > po.real_tol]
        realim = imag_max[imag_max <= po.real_tol]
        gap = (float(realim.max()) if realim.size else 0.0,
               float(nonreal.min()) if nonreal.size else math.inf)
    else:
        gap = (0.0, math.inf)

    # classification of the real stationary points
    theta = np.zeros((real.size, m))
    eig = np.zeros((real.size, m))
    V = np.zeros(real.size)
    for r, i in enumerate(real):
        x, y = z[i, :m].real, z[i, m:].real
        th = np.arctan2(y, x)
        theta[r] = np.where(th <= -np.pi, np.pi, th)  # the paper's range (-pi, pi]
        w = np.linalg.eigvalsh(hessian_theta(sys_.J, theta[r]))
        eig[r] = w
        V[r] = energy(sys_.J, theta[r])
    tau = po.eig_rel * np.maximum(1.0, np.max(np.abs(eig), axis=1)) if real.size else np.zeros(0)
    index = np.sum(eig < -tau[:, None], axis=1).astype(np.int64) if real.size else np.zeros(0, np.int64)
    degenerate = np.min(np.abs(eig), axis=1) <= tau if real.size else np.zeros(0, bool)

    order = np.lexsort(np.round(theta, 9).T[::-1] + 0.0) if real.size else np.zeros(0, np.int64)
    info = dict(unresolved_jumps=sorted(still),
                counts={k: int(np.sum(ep == v)) for k, v in
                        (("nonsingular", EP_NONSINGULAR), ("singular", EP_SINGULAR),
                         ("diverged", EP_DIVERGED), ("fail", EP_FAIL))})
    return Result(N=N, z=z, t=t, track_status=st, endpoint=ep, accepted=acc, rejected=rej,
                  resid=res, cond=cond, alpha=alpha, beta=beta, real_ids=real[order],
                  theta=theta[order], index=index[order], eig=eig[order], V=V[order],
                  degenerate=degenerate[order], retracked=np.array(sorted(retracked), np.int64),
                  reality_gap=gap, info=info)


# ---------------------------------------------------------------------------
# Sensitivities of stationary points to the couplings (implicit functions)
# ---------------------------------------------------------------------------

def coupling_pairs(N: int):
    """Unordered couplings (a, b), a < b, in row-major order."""
    return [(a, b) for a in range(N) for b in range(a + 1, N)]


def _spin(z: np.ndarray, m: int):
    x = np.append(z[:m], 1.0 + 0j)
    y = np.append(z[m:], 0.0 + 0j)
    return x, y


def dP_dJ(N: int, z: np.ndarray, a: int, b: int) -> np.ndarray:
    """dP/dJ_ab for the symmetric coupling J_ab = J_ba: the gradient row of
    spin a gains (y_a x_b - x_a y_b) and that of spin b loses it (the fixed
    spin N-1 has no row)."""
    m = N - 1
    x, y = _spin(z, m)
    v = np.zeros(2 * m, np.complex128)
    w = y[a] * x[b] - x[a] * y[b]
    if a < m:
        v[a] += w
    if b < m:
        v[b] -= w
    return v


def energy_z(J: np.ndarray, z: np.ndarray):
    """V = sum_{i<k} J_ik (1 - x_i x_k - y_i y_k) in the polynomial variables."""
    N = J.shape[0]
    x, y = _spin(z, N - 1)
    iu = np.triu_indices(N, 1)
    return np.sum(J[iu] * (1.0 - x[iu[0]] * x[iu[1]] - y[iu[0]] * y[iu[1]]))


def grad_energy_z(J: np.ndarray, z: np.ndarray) -> np.ndarray:
    """dV/dx_i = -sum_k J_ik x_k, dV/dy_i = -sum_k J_ik y_k for free spins i."""
    N = J.shape[0]
    m = N - 1
    x, y = _spin(z, m)
    Jz = J.copy()
    np.fill_diagonal(Jz, 0.0)
    return np.concatenate([-(Jz @ x)[:m], -(Jz @ y)[:m]])


def sp_sensitivity(J: np.ndarray, z: np.ndarray) -> np.ndarray:
    """dz/dJ_ab = -P_z^{-1} dP/dJ_ab for every coupling (implicit function
    theorem at a nonsingular root); returns (n, #pairs) complex."""
    s = System(J)
    A = s.Pz(z)
    cols = [dP_dJ(s.N, z, a, b) for a, b in coupling_pairs(s.N)]
    return -np.linalg.solve(A, np.stack(cols, axis=1))


def denergy_dJ(J: np.ndarray, z: np.ndarray) -> np.ndarray:
    """Total derivative dV(z*(J); J)/dJ_ab along the stationary point z*(J),
    as an N x N symmetric matrix (entry (a,b) = (b,a) = d/dJ_ab), computed
    forward: partial dV/dJ_ab + grad_z V . dz/dJ_ab."""
    N = J.shape[0]
    x, y = _spin(z, N - 1)
    dz = sp_sensitivity(J, z)
    gz = grad_energy_z(J, z)
    G = np.zeros((N, N))
    for c, (a, b) in enumerate(coupling_pairs(N)):
        d = (1.0 - x[a] * x[b] - y[a] * y[b]) + gz @ dz[:, c]
        G[a, b] = G[b, a] = d.real
    return G


def dcoord_dJ(J: np.ndarray, z: np.ndarray, k: int) -> np.ndarray:
    """d z_k*(J) / dJ_ab (a non-stationary objective), N x N symmetric."""
    N = J.shape[0]
    dz = sp_sensitivity(J, z)
    G = np.zeros((N, N))
    for c, (a, b) in enumerate(coupling_pairs(N)):
        G[a, b] = G[b, a] = dz[k, c].real
    return G


def resolve_sp(J: np.ndarray, z0: np.ndarray, iters: int = 30) -> np.ndarray:
    """Newton on P from z0 (used to follow a stationary point under a small
    change of J)."""
    s = System(J)
    z, _, _ = s.refine(z0.astype(np.complex128), iters, 1e-16)
    return z[0]


def minima_objectives(res: Result, J: np.ndarray):
    """(E_globalmin, sum over certified minima of V) and the minima's endpoints."""
    mins = np.where((res.index == 0) & ~res.degenerate)[0]
    if mins.size == 0:
        return math.inf, 0.0, np.zeros((0, 2 * (J.shape[0] - 1)), np.complex128)
    zs = res.z[res.real_ids[mins]].real.astype(np.complex128)
    return float(np.min(res.V[mins])), float(np.sum(res.V[mins])), zs
