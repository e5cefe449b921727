#!/usr/bin/env python
"""Benchmark: paths tracked per second on the clean power-law XY ring N=10
(sigma = 1, h = 0, theta_N = 0: 18 complex unknowns, 4^9 = 262144 paths),
float32 tracking with the float64 endgame, against the all-float64 pipeline.

One step = the whole hot path on the GPU for all 262144 paths: track, refine
and certify every endpoint, path-jump check, float64 re-tracking of failed or
duplicated paths, real filter, Hessian-index classification, and the copy of
the compact real stationary points to the host.  Inputs (couplings, gamma)
are resident on the device before the timed region.

--workload paper11 / paper13 time the paper's own alpha = 0.75 rings
(1048576 and 16777216 paths) instead, checked against the stationary-point
counts the paper reports.

Prints one JSON line.  Extra keys: the all-float64 rate and the speed-up, the
tracking kernel's roofline (algorithmic flops per launch over the launch's
duration, timed with HIP events on the launch stream), parity of the real
stationary points with the oracle's stored result, and the CPU oracle timed on
a sample of the same paths.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "paths tracked/s at N=10 (262144 paths), FP32+FP64-endgame vs all-FP64"
GAMMA_SEED = 0
# --workload: the default is the headline configuration; the paper's own
# alpha = 0.75 rings (its reported stationary-point counts are the parity
# check there) are extra measurements.
WORKLOADS = {
    "ring10": dict(N=10, kind="clean", p=1.0, metric=METRIC, golden="oracle_ring10.json",
                   desc="clean XY ring N=10 sigma=1 h=0, 262144 total-degree paths"),
    "paper11": dict(N=11, kind="paper", p=0.75, golden="oracle_paper11.json", paper_count=4774,
                    metric="paths tracked/s on the paper's alpha=0.75 XY ring N=11 (1048576 paths), "
                           "FP32+FP64-endgame vs all-FP64",
                    desc="paper XY ring N=11 alpha=0.75 (paper's K), 1048576 total-degree paths"),
    "paper13": dict(N=13, kind="paper", p=0.75, golden=None, paper_count=24830,
                    metric="paths tracked/s on the paper's alpha=0.75 XY ring N=13 (16777216 paths), "
                           "FP32+FP64-endgame vs all-FP64",
                    desc="paper XY ring N=13 alpha=0.75 (paper's K), 16777216 total-degree paths"),
}
FP32_VECTOR_PEAK = 157.3   # TFLOP/s, MI355X vector fp32 (AMD spec)
FP64_VECTOR_PEAK = 78.6    # TFLOP/s, MI355X vector fp64 (AMD spec)

# HBM traffic of one float32 tracking launch of this workload, from two
# rocprofv3 counter runs of this script (FETCH_SIZE, then WRITE_SIZE, in KiB
# per dispatch), each scaled by what the same counter reads for a plain
# 256 MiB device copy in the same run (--copy-ref 256).  Valid only for the
# tracker sources it was measured on: reported as null once they change.
TRACKER_SOURCES = ("track.hip", "path.hpp", "xy_lane.hpp", "cx.hpp", "common.hpp")
MEASURED_TRAFFIC = dict(
    sources_sha256="c5812fb48ad51f8994bceeb534e7d3dca6a20d6eae8fdf775b531a181c58415e",
    fetch_kib=84158.1875, fetch_scale=1.99967, write_kib=522320.4375, write_scale=1.0)


def fetch_real(b):
    """Compact results to the host: the candidate count, then the classified
    candidates packed into one float64 buffer (one copy; integers and flags
    are exact in float64)."""
    import torch
    K = int(b.counts[8].item())
    m = b.theta.shape[0]
    packed = torch.cat([b.is_real[:K].double(), b.index[:K].double(), b.energy[:K],
                        b.degenerate[:K].double(), b.theta[:, :K].reshape(-1)]).cpu()
    return dict(K=K, is_real=packed[0:K].to(torch.int32), index=packed[K:2 * K].to(torch.int32),
                energy=packed[2 * K:3 * K], degenerate=packed[3 * K:4 * K].to(torch.int32),
                theta=packed[4 * K:].reshape(m, K))


def time_pipeline(pipeline, batch, precision, steps, warmup):
    import torch
    opts = pipeline.Options(precision=precision)
    bufs = pipeline.allocate(batch, precision)
    for _ in range(warmup):
        pipeline.run(batch, opts, bufs)
        fetch_real(bufs)
    torch.cuda.synchronize()
    names = ("track_begin", "track_end", "resume_begin", "resume_end", "tail_begin", "tail_end")
    evs = [{k: torch.cuda.Event(enable_timing=True) for k in names} for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        pipeline.run(batch, opts, bufs, events=evs[k])
        out = fetch_real(bufs)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    def span(a, b):
        out = []
        for e in evs:
            try:
                out.append(e[a].elapsed_time(e[b]))
            except ValueError:      # stage not run in this configuration
                out.append(0.0)
        return out
    track_ms = span("track_begin", "track_end")
    resume_ms = span("resume_begin", "resume_end") if precision == "fp32" else [0.0]
    tail_ms = span("tail_begin", "tail_end")
    return (t1 - t0) / steps, track_ms, resume_ms, tail_ms, bufs, out


def attribute_work(pipeline, batch, bufs, precision, m):
    """Untimed run that splits the linear-solve count between the tracking
    launch, the per-lane float64 continuation and the lane-group tail (the
    counters are cumulative per path: snapshots after each launch)."""
    import torch
    from paper_1104_5497_amd import flops
    snap = {}

    def snapshot(key):
        def f():
            snap[key] = (int(bufs.solves.sum()), int((bufs.accepted + bufs.rejected).sum()))
        return f

    pipeline.run(batch, pipeline.Options(precision=precision), bufs,
                 events={"after_track": snapshot("track"), "after_resume": snapshot("resume")})
    torch.cuda.synchronize()
    s1, st1 = snap["track"]
    s2, st2 = snap["resume"][0] - s1, snap["resume"][1] - st1
    # re-tracked paths restart their step counters and pass no solve counter
    s3 = int(bufs.solves.sum()) - snap["resume"][0]
    st3 = max(0, int((bufs.accepted + bufs.rejected).sum()) - snap["resume"][1])
    return dict(track=flops.kernel_flops(m, s1, st1, wide_residual=(precision == "fp32")),
                track_solves=s1,
                resume=flops.kernel_flops(m, s2, st2), resume_solves=s2,
                tail=flops.kernel_flops(m, s3, st3), tail_solves=s3)


def parity_vs_golden(out, m, golden, paper_count=None):
    """Compare the certified real stationary points with the oracle's stored
    result (same count, same Hessian indices, angles within 1e-10 mod 2 pi)
    and, for the paper's rings, with the count the paper reports."""
    real = out["is_real"].numpy().astype(bool)
    deg = out["degenerate"].numpy().astype(bool)[real]
    th = out["theta"].numpy()[:m].T[real][~deg]
    idx = out["index"].numpy()[real][~deg]
    hist = np.bincount(idx, minlength=m).tolist()
    res = dict(num_real=int(th.shape[0]), histogram=hist,
               morse_sum=int(np.sum((-1) ** idx.astype(np.int64))))
    if paper_count is not None:
        res["paper_count"] = paper_count
        res["matches_paper"] = int(th.shape[0]) == paper_count
    path = os.path.join(ROOT, "tests", "golden", golden) if golden else None
    if path and os.path.exists(path):
        from tests._match import match_sets
        g = json.load(open(path))["rings"][0]
        try:
            err = match_sets(th, idx, np.array(g["theta"]), np.array(g["index"]))
            ok = True
        except AssertionError:
            err, ok = None, False
        res.update(oracle_num_real=g["num_real"], oracle_histogram=g["histogram"], sets_equal=ok,
                   max_theta_err=err)
    return res


def tracker_sources_sha():
    import hashlib
    h = hashlib.sha256()
    for f in TRACKER_SOURCES:
        with open(os.path.join(ROOT, "paper_1104_5497_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """Bytes per float32 tracking launch, or None when not measured for the
    current sources."""
    t = MEASURED_TRAFFIC
    if not t or t["sources_sha256"] != tracker_sources_sha():
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


def cpu_baseline(J, gamma, sample, name, seed=1):
    """The oracle as it stands (track + refine) on a random sample of path ids."""
    import oracle
    threads = min(16, len(os.sched_getaffinity(0)))
    rng = np.random.default_rng(seed)
    P = 4 ** (J.shape[0] - 1)
    sample = min(sample, P)
    ids = np.sort(rng.choice(P, size=sample, replace=False)).astype(np.int64)
    s = oracle.System(J)
    t0 = time.perf_counter()
    r = s.track(gamma, ids, oracle.TrackOpts(), nthreads=threads)
    fin = (r["status"] == oracle.ST_REACHED)
    s.refine(r["z"][fin])
    dt = time.perf_counter() - t0
    return dict(value=sample / dt, unit="paths/s", cores=threads, kind="oracle",
                sample=f"{sample} random path ids of the {name} workload (seed {seed}), "
                       f"tracked and refined with the oracle's FP64 C tracker on {threads} threads; "
                       f"{dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="ring10")
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cpu-sample", type=int, default=65536)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--print-sources-sha", action="store_true")
    ap.add_argument("--copy-ref", type=int, default=0,
                    help="run one plain device copy of this many MiB first (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    a = ap.parse_args()
    if a.print_sources_sha:
        print(tracker_sources_sha())
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the path set would shard by path id across GPUs, "
              "but this build measures a single MI355X", file=sys.stderr)
        sys.exit(2)

    import torch
    import workload
    from paper_1104_5497_amd import flops, pipeline

    if a.copy_ref > 0:
        src = torch.ones(a.copy_ref * 262144, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    W = WORKLOADS[a.workload]
    N = W["N"]
    J = (workload.clean_ring_J(N, W["p"]) if W["kind"] == "clean"
         else workload.paper_ring_J(N, W["p"]))
    gamma = workload.gamma_from_seed(GAMMA_SEED)
    m = N - 1
    P = 4 ** m
    batch = pipeline.Batch([J], [gamma], "cuda")

    sec32, tr32, rs32, tl32, b32, out32 = time_pipeline(pipeline, batch, "fp32", a.steps,
                                                        a.warmup)
    w32 = attribute_work(pipeline, batch, b32, "fp32", m)
    k_track = dict(kernel=f"nphc::track_uniform_kernel<float, {m}>", dtype="f32",
                   launch_ms=float(np.mean(tr32)), flops=w32["track"], solves=w32["track_solves"],
                   peak=FP32_VECTOR_PEAK)
    k_resume = dict(kernel=f"nphc::track_uniform_kernel<double, {m}> (continuation)", dtype="f64",
                    launch_ms=float(np.mean(rs32)), flops=w32["resume"],
                    solves=w32["resume_solves"], peak=FP64_VECTOR_PEAK)
    k_tail = dict(kernel=f"nphc::track_group_uniform_kernel<{m}> (lane-group tail)", dtype="f64",
                  launch_ms=float(np.mean(tl32)), flops=w32["tail"], solves=w32["tail_solves"],
                  peak=FP64_VECTOR_PEAK)
    for k in (k_track, k_resume, k_tail):
        k["achieved"] = k["flops"] / (k["launch_ms"] / 1e3) / 1e12 if k["launch_ms"] > 0 else 0.0
        k["frac"] = k["achieved"] / k["peak"]
    dom = max((k_track, k_resume, k_tail), key=lambda k: k["launch_ms"])
    parity = parity_vs_golden(out32, m, W["golden"], W.get("paper_count"))

    res = dict(metric=W["metric"], value=P / sec32, unit="paths/s", n_gpus=1, steps=a.steps,
               warmup=a.warmup, ms_per_step=sec32 * 1e3, higher_is_better=True, scaling="weak",
               vs_baseline=None, dtype="f32+f64", data="synthetic",
               config=dict(workload=W["desc"] + ", FP32 track + FP64 continuation/endgame/"
                                                 "re-track/certify/classify",
                           N=N, **({"sigma": W["p"]} if W["kind"] == "clean" else {"alpha": W["p"]}),
                           gamma_seed=GAMMA_SEED, paths=P),
               roofline=dict(bound="alu", achieved=dom["achieved"], peak=dom["peak"],
                             unit="TFLOP/s", frac=dom["frac"],
                             traffic=(measured_traffic() if dom is k_track and a.workload == "ring10"
                                      else None),
                             kernel=dom["kernel"], launch_ms=dom["launch_ms"],
                             flops_per_launch=dom["flops"], solve_flops=flops.solve_flops(m),
                             dense_equiv_flops=dom["solves"] * flops.dense_solve_flops(m)),
               kernels=[k_track, k_resume, k_tail],
               track_only_paths_per_s=P / ((k_track["launch_ms"] + k_resume["launch_ms"] +
                                            k_tail["launch_ms"]) / 1e3),
               parity=parity)
    if not a.no_fp64:
        sec64, tr64, _, tl64, b64, out64 = time_pipeline(pipeline, batch, "fp64", a.steps,
                                                         a.warmup)
        w64 = attribute_work(pipeline, batch, b64, "fp64", m)
        ach64 = w64["track"] / (np.mean(tr64) / 1e3) / 1e12
        res["fp64"] = dict(value=P / sec64, ms_per_step=sec64 * 1e3,
                           track_ms=float(np.mean(tr64)), tail_ms=float(np.mean(tl64)),
                           track_only_paths_per_s=P / ((np.mean(tr64) + np.mean(tl64)) / 1e3),
                           achieved_tflops=ach64,
                           frac_of_fp64_peak=ach64 / FP64_VECTOR_PEAK,
                           parity=parity_vs_golden(out64, m, W["golden"], W.get("paper_count")))
        res["speedup_vs_fp64"] = sec64 / sec32
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(J, gamma, a.cpu_sample, a.workload)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
