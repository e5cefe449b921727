"""find_all_sps: the NPHC pipeline on one GPU, as a sequence of C-ABI calls.

PyTorch supplies device memory and the stream; every computation is a kernel
of libnphc.so.  The host only marshals pointers and, at the end, copies the
compact results back.

Pipeline (paper, sections "NPHC method" and "A First Application"):
  1. track every total-degree path (float32 or float64 predictor/corrector);
  2. refine the endpoints by Newton on F at t = 1 and certify them (float64);
  3. path-jump check: two nonsingular endpoints of one system at the same
     root are both re-tracked;
  4. re-track failed or duplicated paths in float64 with a quarter of the
     maximal step (repeated a fixed number of rounds, device-side counts);
  5. real filter, angles, energies and Hessian indices of the certified real
     roots (float64).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _p(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Batch:
    """Rings tracked together; systems are kept in the order given, which
    must be sorted by ring size (nondecreasing N)."""

    def __init__(self, Js: Sequence[np.ndarray], gammas: Sequence[complex], device="cuda"):
        if len(Js) != len(gammas) or len(Js) == 0:
            raise ValueError("need one gamma per coupling matrix")
        Ns = [int(np.asarray(J).shape[0]) for J in Js]
        if any(Ns[i] > Ns[i + 1] for i in range(len(Ns) - 1)):
            raise ValueError("systems must be sorted by ring size")
        for J in Js:
            J = np.asarray(J)
            if J.ndim != 2 or J.shape[0] != J.shape[1]:
                raise ValueError("coupling matrices must be square")
        self.device = torch.device(device)
        self.N_host = np.ascontiguousarray(Ns, dtype=np.int32)
        self.path_off_host = np.zeros(len(Ns) + 1, dtype=np.int64)
        self.path_off_host[1:] = np.cumsum([4 ** (n - 1) for n in Ns])
        J_off = np.zeros(len(Ns), dtype=np.int64)
        J_off[1:] = np.cumsum([n * n for n in Ns])[:-1]
        Jcat = np.concatenate([np.asarray(J, dtype=np.float64).ravel() for J in Js])
        g = np.array([[complex(x).real, complex(x).imag] for x in gammas], dtype=np.float64).ravel()
        self.J = torch.from_numpy(Jcat).to(self.device)
        self.J_off = torch.from_numpy(J_off).to(self.device)
        self.gamma = torch.from_numpy(g).to(self.device)
        self.N = torch.from_numpy(self.N_host.copy()).to(self.device)
        self.path_off = torch.from_numpy(self.path_off_host.copy()).to(self.device)
        self.Js = [np.asarray(J, dtype=np.float64) for J in Js]
        self.gammas = [complex(x) for x in gammas]
        self.c = L.Batch_(len(Ns), 0, self.N_host.ctypes.data, self.path_off_host.ctypes.data,
                          self.N.data_ptr(), self.path_off.data_ptr(), self.J.data_ptr(),
                          self.J_off.data_ptr(), self.gamma.data_ptr())

    @property
    def num_systems(self) -> int:
        return len(self.N_host)

    @property
    def num_items(self) -> int:
        return int(self.path_off_host[-1])

    @property
    def n_max(self) -> int:
        return 2 * (int(self.N_host.max()) - 1)

    @property
    def m_max(self) -> int:
        return int(self.N_host.max()) - 1


PREC = {"fp64": L.NPHC_FP64, "fp32": L.NPHC_FP32}


@dataclass
class Buffers:
    """Device arrays of one pipeline run (per item unless noted)."""

    z: torch.Tensor
    t: torch.Tensor
    status: torch.Tensor
    accepted: torch.Tensor
    rejected: torch.Tensor
    solves: torch.Tensor
    h: torch.Tensor
    endpoint: torch.Tensor
    resid: torch.Tensor
    cond: torch.Tensor
    beta: torch.Tensor
    alpha: torch.Tensor
    alpha_real: torch.Tensor
    ids: torch.Tensor          # id list scratch
    ids2: torch.Tensor
    ids3: torch.Tensor         # paths finished by the main launch (overlapped refinement)
    ids4: torch.Tensor         # paths left to the lane-group tail
    ids5: torch.Tensor         # handed-off paths the float64 continuation finished
    counts: torch.Tensor       # small device counters (int64)
    ws: torch.Tensor           # tracker workspace (uint8)
    ws64: torch.Tensor         # tracker workspace for float64 re-tracking
    wsdup: torch.Tensor        # duplicate-check hash table
    wssel: torch.Tensor        # compaction block counts
    # classification outputs, per candidate position
    is_real: torch.Tensor
    theta: torch.Tensor
    energy: torch.Tensor
    index: torch.Tensor
    eig: torch.Tensor
    degenerate: torch.Tensor
    side: Optional[object] = None   # second stream (created on first use)


def allocate(batch: Batch, precision: str) -> Buffers:
    P, n, m = batch.num_items, batch.n_max, batch.m_max
    dev = batch.device
    f64 = dict(dtype=torch.float64, device=dev)
    i32 = dict(dtype=torch.int32, device=dev)
    i64 = dict(dtype=torch.int64, device=dev)
    ws_bytes = L.lib().nphc_track_workspace_size(ctypes.byref(batch.c), PREC[precision])
    ws64_bytes = L.lib().nphc_track_workspace_size(ctypes.byref(batch.c), L.NPHC_FP64)
    return Buffers(
        z=torch.zeros((2 * n, P), **f64), t=torch.zeros(P, **f64),
        status=torch.zeros(P, **i32), accepted=torch.zeros(P, **i32),
        rejected=torch.zeros(P, **i32), solves=torch.zeros(P, **i32), h=torch.zeros(P, **f64),
        endpoint=torch.zeros(P, **i32),
        resid=torch.zeros(P, **f64), cond=torch.zeros(P, **f64), beta=torch.zeros(P, **f64),
        alpha=torch.zeros(P, **f64), alpha_real=torch.zeros(P, **f64),
        ids=torch.zeros(P, **i64), ids2=torch.zeros(P, **i64), ids3=torch.zeros(P, **i64),
        ids4=torch.zeros(P, **i64), ids5=torch.zeros(P, **i64), counts=torch.zeros(16, **i64),
        ws=torch.zeros(max(int(ws_bytes), 256), dtype=torch.uint8, device=dev),
        ws64=torch.zeros(max(int(ws64_bytes), 256), dtype=torch.uint8, device=dev),
        wsdup=torch.zeros(max(int(L.lib().nphc_duplicates_workspace_size(P)), 256),
                          dtype=torch.uint8, device=dev),
        wssel=torch.zeros(max(int(L.lib().nphc_select_workspace_size(P)), 256),
                          dtype=torch.uint8, device=dev),
        is_real=torch.zeros(P, **i32), theta=torch.zeros((m, P), **f64),
        energy=torch.zeros(P, **f64), index=torch.zeros(P, **i32),
        eig=torch.zeros((m, P), **f64), degenerate=torch.zeros(P, **i32))


def _mask(*codes: int) -> int:
    v = 0
    for c in codes:
        v |= 1 << c
    return v


@dataclass
class Options:
    precision: str = "fp32"
    track: Optional[L.TrackOpts_] = None        # defaults per precision
    resume: Optional[L.TrackOpts_] = None       # float64 continuation of handed-off paths
    retrack: Optional[L.TrackOpts_] = None      # float64 re-tracking (see retrack_shrink)
    cert: Optional[L.CertOpts_] = None
    classify: Optional[L.ClassOpts_] = None
    dup_tol: float = 1e-8
    retrack_rounds: int = 2
    # hmax is divided by this in every re-track round.  A quarter per round
    # spent 37 ms at N = 11 on its second round (hmax / 16) for paths that
    # stayed failed; halving recovers as many (N = 11 and 13) at a third of
    # the cost.
    retrack_shrink: float = 2.0
    # Tails: once a launch's queue is empty, its paths in flight get at most
    # this many more steps, then the lane-group tracker (16 lanes per path,
    # float64) finishes them.  None: the default for the precision; 0: off.
    # Which paths are still in flight then depends on scheduling, so such a
    # path may finish in float64 in one run and in float32 in another (its
    # endpoint then differs in the last bits; the certified sets do not).
    # deterministic = True turns the drain hand-off off: every output is then
    # a function of the path id alone.
    drain: Optional[int] = None
    cont_drain: int = 20          # the same for the per-lane float64 continuation
    tail_group: bool = True
    deterministic: bool = False
    # refine the paths the main launch finished on a second stream while the
    # float64 continuation and tail run (they touch disjoint items)
    overlap: bool = True
    # lanes per endpoint for refining the lane-group tail's paths (a short
    # list on the critical path: the certificate's solves split over them)
    tail_refine_lanes: int = 8


DRAIN_DEFAULT = {"fp32": 96, "fp64": 112}
# path statuses that end tracking (everything but PENDING and HANDOFF)
FINISHED = (L.PATH_REACHED, L.PATH_DIVERGED, L.PATH_FAIL_MINSTEP, L.PATH_FAIL_MAXSTEPS,
            L.PATH_FAIL_NONFINITE, L.PATH_STALLED)


def conservative_opts() -> L.TrackOpts_:
    """Re-tracking settings: float64, tight corrector, large divergence
    radius, no end-zone shortcuts (the predictor-error guard stays on); a lane
    group per path, since only a few paths are re-tracked."""
    return L.default_track_opts(L.NPHC_FP64).copy(corr_tol=1e-10, R_inf=1e8, grow_cap=0.0,
                                                   hmin_rel=0.0, lanes_per_path=16)


def run(batch: Batch, opts: Options = Options(), bufs: Optional[Buffers] = None, stream=None,
        events: Optional[Dict] = None) -> Buffers:
    """Enqueue the whole pipeline on the stream (no host synchronisation).
    events: optional dict of torch.cuda.Event, recorded on the pipeline's
    stream around the main tracking launch ("track_begin"/"track_end"), the
    float64 continuation ("resume_begin"/"resume_end") and the lane-group
    tail ("tail_begin"/"tail_end"), and optional callables "after_track" and
    "after_resume", invoked right after those launches are enqueued."""
    lib = L.lib()
    prec = PREC[opts.precision]
    b = bufs or allocate(batch, opts.precision)
    s = _stream(stream)
    main = stream if stream is not None else torch.cuda.current_stream()
    P = batch.num_items
    to = opts.track or L.default_track_opts(prec)
    drain = DRAIN_DEFAULT[opts.precision] if opts.drain is None else opts.drain
    if opts.track is None and opts.tail_group and not opts.deterministic:
        to = to.copy(drain_steps=drain)
    co = opts.cert or L.default_cert_opts()
    clo = opts.classify or L.default_class_opts()
    rt = opts.retrack or conservative_opts()
    B = ctypes.byref(batch.c)
    cnt = b.counts
    c_sel = ctypes.c_void_p(cnt.data_ptr())              # counts[0]: list length
    c_dup = ctypes.c_void_p(cnt.data_ptr() + 8)          # counts[1]: marked duplicates
    stride = P

    events = events or {}
    if "track_begin" in events:
        events["track_begin"].record(main)
    L.check(lib.nphc_track_paths(B, None, P, None, prec, ctypes.byref(to), _p(b.z), stride,
                                 _p(b.t), _p(b.status), _p(b.accepted), _p(b.rejected),
                                 _p(b.solves), _p(b.h), _p(b.ws), b.ws.numel(), s),
            "nphc_track_paths")
    if "track_end" in events:
        events["track_end"].record(main)
    if "after_track" in events:
        events["after_track"]()
    handed_off = (to.handoff_rejects > 0 or to.handoff_norm > 0 or to.handoff_steps > 0 or
                  to.drain_steps > 0)
    c_ho = ctypes.c_void_p(cnt.data_ptr() + 8 * 9)       # counts[9]: handed off
    overlap = handed_off and opts.overlap

    def refine(ids, c_list, strm, o=co):
        L.check(lib.nphc_refine_certify(B, _p(ids), P, c_list, ctypes.byref(o), _p(b.z), stride,
                                        _p(b.t), _p(b.status), _p(b.endpoint), _p(b.resid),
                                        _p(b.cond), _p(b.beta), _p(b.alpha), _p(b.alpha_real),
                                        strm), "nphc_refine_certify")

    if handed_off:
        L.check(lib.nphc_select(_p(b.status), P, _mask(L.PATH_HANDOFF), _p(b.ids), c_ho,
                                _p(b.wssel), b.wssel.numel(), s), "nphc_select")
    if overlap:
        # the paths the main launch finished are refined on a second stream
        c_fin = ctypes.c_void_p(cnt.data_ptr() + 8 * 11)  # counts[11]: finished
        L.check(lib.nphc_select(_p(b.status), P, _mask(*FINISHED), _p(b.ids3), c_fin,
                                _p(b.wssel), b.wssel.numel(), s), "nphc_select")
        if b.side is None:
            b.side = torch.cuda.Stream(device=b.z.device)
        fork = torch.cuda.Event()
        fork.record(main)

    def side_refine_finished():
        # enqueued after the continuation's launch, so that the continuation
        # reaches the hardware first (the refinement then fills its gaps);
        # it depends only on the fork recorded before the continuation
        b.side.wait_event(fork)
        refine(b.ids3, c_fin, ctypes.c_void_p(b.side.cuda_stream))
        ev = torch.cuda.Event()
        ev.record(b.side)
        return ev

    if handed_off and prec == L.NPHC_FP32:
        # float64 continuation of the paths the float32 tracker handed off,
        # one path per lane (its own tail left to the lane groups below)
        ro = opts.resume or L.default_track_opts(L.NPHC_FP64).copy(
            resume=1,
            drain_steps=opts.cont_drain if opts.tail_group and not opts.deterministic else 0)
        if "resume_begin" in events:
            events["resume_begin"].record(main)
        L.check(lib.nphc_track_paths(B, _p(b.ids), P, c_ho, L.NPHC_FP64, ctypes.byref(ro),
                                     _p(b.z), stride, _p(b.t), _p(b.status), _p(b.accepted),
                                     _p(b.rejected), _p(b.solves), _p(b.h), _p(b.ws64),
                                     b.ws64.numel(), s), "nphc_track_paths(resume)")
        if "resume_end" in events:
            events["resume_end"].record(main)
    if overlap:
        join = side_refine_finished()
    if "after_resume" in events:
        events["after_resume"]()
    c_tail = ctypes.c_void_p(cnt.data_ptr() + 8 * 10)      # counts[10]: tail paths
    split = overlap and opts.tail_group and prec == L.NPHC_FP32
    if handed_off and opts.tail_group:
        # the last, long paths: float64, a group of 16 lanes per path
        go = L.default_track_opts(L.NPHC_FP64).copy(resume=1, lanes_per_path=16)
        L.check(lib.nphc_select(_p(b.status), P, _mask(L.PATH_HANDOFF), _p(b.ids4), c_tail,
                                _p(b.wssel), b.wssel.numel(), s), "nphc_select")
        if split:
            # the handed-off paths the continuation finished are refined on
            # the second stream while the lane groups track the rest
            c_cf = ctypes.c_void_p(cnt.data_ptr() + 8 * 12)  # counts[12]
            L.check(lib.nphc_select_list(_p(b.status), _p(b.ids), P, c_ho,
                                         _mask(L.PATH_PENDING, *FINISHED),
                                         _p(b.ids5), c_cf, _p(b.wssel), b.wssel.numel(), s),
                    "nphc_select_list")
            fork2 = torch.cuda.Event()
            fork2.record(main)
            b.side.wait_event(fork2)
            refine(b.ids5, c_cf, ctypes.c_void_p(b.side.cuda_stream))
            join = torch.cuda.Event()      # the second stream runs in order: this
            join.record(b.side)            # also covers its first refinement
        if "tail_begin" in events:
            events["tail_begin"].record(main)
        L.check(lib.nphc_track_paths(B, _p(b.ids4), P, c_tail, L.NPHC_FP64, ctypes.byref(go),
                                     _p(b.z), stride, _p(b.t), _p(b.status), _p(b.accepted),
                                     _p(b.rejected), _p(b.solves), _p(b.h), _p(b.ws64),
                                     b.ws64.numel(), s), "nphc_track_paths(tail)")
        if "tail_end" in events:
            events["tail_end"].record(main)
    if split:
        # the tail's paths; then wait for the second stream
        refine(b.ids4, c_tail, s, co.copy(lanes_per_item=opts.tail_refine_lanes))
        main.wait_event(join)
    elif overlap:
        # the handed-off paths, once finished; then wait for the other half
        refine(b.ids, c_ho, s)
        main.wait_event(join)
    else:
        L.check(lib.nphc_refine_certify(B, None, P, None, ctypes.byref(co), _p(b.z), stride,
                                        _p(b.t), _p(b.status), _p(b.endpoint), _p(b.resid),
                                        _p(b.cond), _p(b.beta), _p(b.alpha), _p(b.alpha_real), s),
                "nphc_refine_certify")

    def dedupe(probe=None, c_probe=None):
        L.check(lib.nphc_select(_p(b.endpoint), P, _mask(L.END_NONSINGULAR), _p(b.ids2), c_sel,
                                _p(b.wssel), b.wssel.numel(), s), "nphc_select")
        L.check(lib.nphc_mark_duplicates(B, _p(b.ids2), P, c_sel, _p(probe), c_probe,
                                         opts.dup_tol, _p(b.z), stride, _p(b.endpoint), c_dup,
                                         _p(b.wsdup), b.wsdup.numel(), s),
                "nphc_mark_duplicates")

    dedupe()
    hmax = rt.hmax
    for r in range(opts.retrack_rounds):
        hmax /= opts.retrack_shrink
        o = rt.copy(h0=min(rt.h0, hmax), hmax=hmax)
        c_rt = ctypes.c_void_p(cnt.data_ptr() + 8 * (2 + r))  # counts[2+r]: re-tracked
        L.check(lib.nphc_select(_p(b.endpoint), P, _mask(L.END_FAIL, L.END_DUPLICATE), _p(b.ids),
                                c_rt, _p(b.wssel), b.wssel.numel(), s), "nphc_select")
        L.check(lib.nphc_track_paths(B, _p(b.ids), P, c_rt, L.NPHC_FP64, ctypes.byref(o), _p(b.z),
                                     stride, _p(b.t), _p(b.status), _p(b.accepted),
                                     _p(b.rejected), None, _p(b.h), _p(b.ws64), b.ws64.numel(), s),
                "nphc_track_paths(retrack)")
        L.check(lib.nphc_refine_certify(B, _p(b.ids), P, c_rt, ctypes.byref(co), _p(b.z), stride,
                                        _p(b.t), _p(b.status), _p(b.endpoint), _p(b.resid),
                                        _p(b.cond), _p(b.beta), _p(b.alpha), _p(b.alpha_real), s),
                "nphc_refine_certify(retrack)")
        # only the re-tracked endpoints can form new coincidences
        dedupe(b.ids, c_rt)
    # classification of every nonsingular endpoint (the real filter is inside)
    c_cls = ctypes.c_void_p(cnt.data_ptr() + 8 * 8)       # counts[8]: nonsingular endpoints
    L.check(lib.nphc_select(_p(b.endpoint), P, _mask(L.END_NONSINGULAR), _p(b.ids2), c_cls,
                            _p(b.wssel), b.wssel.numel(), s), "nphc_select")
    L.check(lib.nphc_classify(B, _p(b.ids2), P, c_cls, ctypes.byref(clo), co.real_tol, _p(b.z),
                              stride, _p(b.endpoint), _p(b.alpha_real), _p(b.is_real),
                              _p(b.theta), _p(b.energy), _p(b.index), _p(b.eig),
                              _p(b.degenerate), s), "nphc_classify")
    return b


@dataclass
class SystemResult:
    N: int
    real_items: np.ndarray     # batch item ids of the certified real stationary points
    theta: np.ndarray          # (R, m), sorted lexicographically
    index: np.ndarray
    eig: np.ndarray
    V: np.ndarray
    degenerate: np.ndarray
    z: np.ndarray              # (R, n) refined coordinates (complex)

    @property
    def histogram(self) -> np.ndarray:
        return np.bincount(self.index[~self.degenerate], minlength=self.N - 1)


def collect(batch: Batch, b: Buffers, retrack_rounds: int = 2) -> Dict:
    """Copy the compact results to the host and split them per system."""
    torch.cuda.synchronize()
    counts = b.counts.cpu().numpy()
    K = int(counts[8])
    ids = b.ids2[:K].cpu().numpy()
    is_real = b.is_real[:K].cpu().numpy().astype(bool)
    m = batch.m_max
    th = b.theta[:, :K].cpu().numpy().T
    eig = b.eig[:, :K].cpu().numpy().T
    V = b.energy[:K].cpu().numpy()
    idx = b.index[:K].cpu().numpy()
    deg = b.degenerate[:K].cpu().numpy().astype(bool)
    rid = ids[is_real]
    zsel = b.z.cpu().numpy()[:, rid]
    endpoint = b.endpoint.cpu().numpy()
    status = b.status.cpu().numpy()
    systems = []
    for s_ in range(batch.num_systems):
        N = int(batch.N_host[s_])
        mm = N - 1
        lo, hi = batch.path_off_host[s_], batch.path_off_host[s_ + 1]
        sel = (ids >= lo) & (ids < hi) & is_real
        t_ = th[sel][:, :mm]
        order = np.lexsort(np.round(t_, 9).T[::-1] + 0.0) if t_.shape[0] else np.zeros(0, np.int64)
        selr = (rid >= lo) & (rid < hi)
        zr = zsel[:, selr]
        zc = (zr[0::2][: 2 * mm] + 1j * zr[1::2][: 2 * mm]).T if zr.size else np.zeros((0, 2 * mm), complex)
        systems.append(SystemResult(
            N=N, real_items=ids[sel][order], theta=t_[order], index=idx[sel][order].astype(np.int64),
            eig=eig[sel][:, :mm][order], V=V[sel][order], degenerate=deg[sel][order],
            z=zc[order] if zc.shape[0] else zc))
    ep_counts = {k: int(np.sum(endpoint == v)) for k, v in
                 (("nonsingular", L.END_NONSINGULAR), ("singular", L.END_SINGULAR),
                  ("diverged", L.END_DIVERGED), ("fail", L.END_FAIL), ("duplicate", L.END_DUPLICATE))}
    return dict(systems=systems, endpoint_counts=ep_counts,
                retracked=[int(c) for c in counts[2:2 + retrack_rounds]],
                handed_off=int(counts[9]),
                duplicates_last=int(counts[1]), nonsingular=K,
                status_counts=np.bincount(status, minlength=8).tolist())


def find_all_sps(Js, gammas, precision: str = "fp32", opts: Optional[Options] = None, device="cuda"):
    """All certified real stationary points of each ring (see module doc)."""
    if isinstance(Js, np.ndarray) and Js.ndim == 2:
        Js, gammas = [Js], [gammas]
    batch = Batch(Js, gammas, device)
    o = opts or Options(precision=precision)
    o.precision = precision if opts is None else o.precision
    b = run(batch, o)
    res = collect(batch, b, o.retrack_rounds)
    res["batch"] = batch
    res["buffers"] = b
    return res
