#!/usr/bin/env python3
"""Benchmark: parallel filter + RTS smoother steps/s at nx = 4, T = 2^20.

One "step" of the benchmark loop is one whole pass of the hot path -- the
parallel Kalman filter (Algorithm 5) and the RTS smoother (Algorithm 6) -- over
one synthetic constant-velocity tracking sequence of T = 2^20 measurements
already resident in HBM.  `value` is time steps (measurements) processed per
second: T * K / wall time of K passes.

Each pass is enqueued stage by stage (kf_prepare, kf_pass_filter,
kf_pass_rts) on the launch stream.  Every --event-every-th pass of the timed
region also records HIP events between its stages; those sampled passes give
the per-kernel durations used for the roofline and the per-pass latency
percentiles.  (An event between stages costs about 5 us of idle GPU time, so
they are not put into every pass.)
The CPU baseline times the FP64 sequential oracle (filter + RTS) on this
machine's host, one core, on the same input.

Other single-GPU workloads of the same model: --T / --log2T set the length
(T = 1000 and T = 2^18 are the small-case and two-filter configurations),
--smoother tf times the two-filter smoother (Algorithm 7) instead of the RTS
pass, --precision selects f32, mixed (FP32 storage, FP64 solves) or f64, and
--scan selects the scan (look-back, or the one-kernel-per-level tree scans).

Prints one JSON line.  --gpus above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_PEAK = 157.3e12      # MI355X vector FP32 (published, packed) FLOP/s
FP64_VALU_PEAK = 78.6e12       # MI355X vector FP64 FLOP/s


def kernel_source_hash() -> str:
    """Hash of the kernel sources and of the compile flags (less the include
    path, which depends on where the repository sits)."""
    from paper_2511_10363_amd import build as kbuild
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2511_10363_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hpp", ".hip")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(fh.read())
    inc = os.path.join(kbuild.ROOT, "include")
    h.update(" ".join(f for f in kbuild.CXXFLAGS if f != inc).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/traffic.json),
    only if the kernel sources and compile flags have not changed since the
    counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get("%s|%s|%s" % (kernel, workload, precision))
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--event-every", type=int, default=4,
                    help="record stage events on every n-th timed pass")
    ap.add_argument("--precision", default=None, choices=["f32", "mixed", "f64"],
                    help="default: mixed for the serving workload, f32 otherwise")
    ap.add_argument("--log2T", type=int, default=20)
    ap.add_argument("--T", type=int, default=0, help="sequence length (overrides --log2T)")
    ap.add_argument("--smoother", default="rts", choices=["rts", "tf"],
                    help="RTS (Algorithm 6) or two-filter (Algorithm 7) backward pass")
    ap.add_argument("--scan", default="lookback",
                    choices=["lookback", "lookback_generic", "blelloch", "hillis_steele",
                             "ladner_fischer", "sengupta_a", "sengupta_b", "sequential"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="approximate CPU time for the oracle baseline (0 = skip)")
    ap.add_argument("--seed", type=int, default=20251110)
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the HIP-graph replay measurement after the timed region")
    ap.add_argument("--workload", default="tracking",
                    choices=["tracking", "batched", "serving", "tv", "speedup", "scans"],
                    help="tracking: one long sequence (the headline); batched: 4096 ragged "
                         "sequences, a random stable model each; serving: Poisson job "
                         "arrivals served in ragged batches; tv: the paper's time-varying "
                         "model with inputs; speedup: the parallel filter against the "
                         "sequential filter on one GPU lane, over a range of T; scans: "
                         "every scan algorithm with each of the three pipelines")
    ap.add_argument("--jobs", type=int, default=2000, help="jobs of the serving workload")
    ap.add_argument("--no-extra-configs", dest="extra_configs", action="store_false",
                    help="skip the T = 1000 FP64 and T = 2^18 two-filter lines after the "
                         "headline")
    ap.add_argument("--nx", type=int, default=16, help="state size of the serving workload")
    ap.add_argument("--arena-rows", type=int, default=1 << 22,
                    help="rows of the serving arena (admission capacity)")
    ap.add_argument("--nseq", type=int, default=4096, help="sequences of the batched workload")
    args = ap.parse_args()

    if args.precision is None:
        args.precision = "mixed" if args.workload == "serving" else "f32"
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import kf_workloads as W
    from paper_2511_10363_amd import kfscan

    kfscan.load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batched":
        return bench_batched(args, np, torch, W, kfscan, dev)
    if args.workload == "serving":
        return bench_serving(args, np, torch, W, kfscan, dev)
    if args.workload == "tv":
        return bench_tv(args, np, torch, W, kfscan, dev)
    if args.workload == "speedup":
        return bench_speedup(args, np, torch, W, kfscan, dev)
    if args.workload == "scans":
        return bench_scans(args, np, torch, W, kfscan, dev)
    T = args.T if args.T > 0 else 1 << args.log2T
    tname = ("T2^%d" % args.log2T) if args.T <= 0 else ("T%d" % T)
    prec = args.precision
    back = "kf_pass_rts" if args.smoother == "rts" else "kf_pass_twofilter"
    kback = "k_rts" if args.smoother == "rts" else "k_twofilter"
    n, m = 4, 2
    w = 8 if prec == "f64" else 4

    model, y_np = W.tracking(T, seed=args.seed)
    dt = kfscan.dtype_for(prec)
    dmodel = kfscan.model_to_device(model.arrays(), prec, dev)
    y = torch.as_tensor(y_np).to(dev, dt).contiguous()
    plan = kfscan.Plan(dmodel, y, precision=prec, scan=args.scan, smoother=True)

    def one_pass(evs=None):
        if evs is not None:
            evs[0].record()
        plan("kf_prepare")
        if evs is not None:
            evs[1].record()
        plan("kf_pass_filter")
        if evs is not None:
            evs[2].record()
        plan(back)
        if evs is not None:
            evs[3].record()

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()

    K = args.steps
    every = max(1, args.event_every)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] if i % every == 0 else None
              for i in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        one_pass(events[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    events = [e for e in events if e is not None]

    # the same pass captured once into a HIP graph and replayed K times (reported
    # beside the headline, which times the passes as enqueued above)
    graph_ms = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                one_pass()
        torch.cuda.current_stream(dev).wait_stream(side)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(K):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - g0) / K * 1e3
        del g

    # device-copy reference: 256 MiB through the library's plain copy kernel,
    # timed with events (also the calibration dispatch of the counter runs)
    nbytes = 256 << 20
    src = torch.empty(nbytes, dtype=torch.uint8, device=dev).fill_(1)
    dst = torch.empty_like(src)
    kfscan.device_copy(dst, src)
    ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ce0.record()
    for _ in range(3):
        kfscan.device_copy(dst, src)
    ce1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * nbytes * 3 / (ce0.elapsed_time(ce1) * 1e-3) / 1e9
    del src, dst

    wall = t1 - t0
    ms_per_step = wall / K * 1e3
    value = T * K / wall
    lat = np.array([e[0].elapsed_time(e[3]) for e in events])          # ms per whole pass
    t_prep = np.array([e[0].elapsed_time(e[1]) for e in events])
    t_filt = np.array([e[1].elapsed_time(e[2]) for e in events])
    t_back = np.array([e[2].elapsed_time(e[3]) for e in events])

    # algorithmic bytes per launch: each kernel's compulsory reads and writes,
    # once each.  The forward pass reads y and writes the filter moments; the
    # RTS pass reads the filter moments and writes the smoothed ones; the
    # two-filter pass also reads y.  The job as a whole moves w (m + 2n + 2n^2)
    # per step (job_hbm_frac).
    bytes_filter = T * w * (m + n + n * n)
    bytes_back = T * w * (2 * (n + n * n) + (m if args.smoother == "tf" else 0))
    kern = {"k_filter": (float(t_filt.mean()), bytes_filter),
            kback: (float(t_back.mean()), bytes_back)}
    dom = max(kern, key=lambda k: kern[k][0])
    dom_ms, dom_bytes = kern[dom]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    traffic = load_traffic(dom, "tracking_%s_%s" % (tname, args.scan), prec)

    # accuracy of this run against the FP64 oracle, and the CPU baseline
    m_f, P_f, m_s, P_s = (t[0].double().cpu().numpy() for t in plan.outputs())
    cpu = None
    errors = None
    if args.cpu_seconds > 0:
        import oracle
        arrs = model.arrays()
        yy = y_np
        if prec != "f64":
            cast = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
            arrs = tuple(cast(a) for a in arrs)
            yy = cast(y_np)
        reps = 0
        c0 = time.perf_counter()
        smooth = oracle.smooth_rts if args.smoother == "rts" else oracle.smooth_twofilter
        while True:
            ref = smooth(*arrs, yy)
            reps += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        c1 = time.perf_counter()
        cpu = {"value": T * reps / (c1 - c0), "unit": "steps/s", "cores": 1, "kind": "oracle",
               "sample": "sequential FP64 filter + %s smoother over the full T=%d input, "
                         "%d repetition(s)" % ({"rts": "RTS", "tf": "two-filter"}[args.smoother],
                                               T, reps)}

        def nw(a, r):
            return float(np.max(np.abs(a - r)) / max(np.max(np.abs(r)), 1e-300))
        z = float(np.max(np.abs(m_s - ref[2]) / np.sqrt(np.einsum("kii->ki", ref[3]))))
        errors = {"m_filt": nw(m_f, ref[0]), "P_filt": nw(P_f, ref[1]),
                  "m_smooth": nw(m_s, ref[2]), "P_smooth": nw(P_s, ref[3]),
                  "z_smooth_max": z}

    out = {
        "metric": "filter+smoother steps/s at nx=4,T=2^20 (% HBM roofline)",
        "value": value,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f32": "f32", "mixed": "f32+f64solve", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "cv_tracking_nx4_ny2_%s" % tname, "T": T, "nx": n, "ny": m,
                   "dt": 0.1, "q": 1.0, "r": 0.25, "sequences": 1,
                   "pipeline": "kf_prepare+kf_pass_filter+" + back,
                   "scan": args.scan, "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": dom},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "kernel_ms": {"k_prepare": float(t_prep.mean()), "k_filter": float(t_filt.mean()),
                      kback: float(t_back.mean())},
        "job_hbm_frac": value * w * (m + 2 * n + 2 * n * n) / (HBM_PEAK_GBS * 1e9),
        "kernel_hbm_frac": {k: b / (t * 1e-3) / 1e9 / HBM_PEAK_GBS for k, (t, b) in kern.items()},
        "copy_GBps": copy_gbps,
        "graph_ms_per_step": graph_ms,
        "errors_vs_oracle": errors,
    }
    if args.extra_configs and args.T <= 0 and args.log2T == 20:
        out["other_configs"] = other_configs(args, np, torch, W, kfscan, dev)
    print(json.dumps(out))
    return 0


def other_configs(args, np, torch, W, kfscan, dev) -> dict:
    """The two other single-sequence configurations of the tracking model, run
    after the headline: T = 1000 in FP64 (filter + RTS), and T = 2^18 with the
    two-filter smoother in FP32 storage with FP64 solves.  Each: event-timed
    passes (prepare + forward + backward, median of 50 after 5 warm-up) and,
    with the CPU-baseline leg on, the errors against the FP64 sequential RTS
    smoother of the oracle.  Then the generic look-back filter and the paper's
    time-varying model at T = 2^20 in FP32."""
    if args.cpu_seconds > 0:
        import oracle

    res = {}
    for name, T, prec, back in (
            ("T1000_f64_filter_rts", 1000, "f64", "kf_pass_rts"),
            ("T2^18_mixed_filter_twofilter", 1 << 18, "mixed", "kf_pass_twofilter")):
        model, y_np = W.tracking(T, seed=args.seed)
        dt = kfscan.dtype_for(prec)
        dmodel = kfscan.model_to_device(model.arrays(), prec, dev)
        y = torch.as_tensor(y_np).to(dev, dt).contiguous()
        plan = kfscan.Plan(dmodel, y, precision=prec, smoother=True)

        def one():
            plan("kf_prepare")
            plan("kf_pass_filter")
            plan(back)
        for _ in range(5):
            one()
        torch.cuda.synchronize()
        ts = []
        for _ in range(50):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            one()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        ms = float(np.median(ts))
        res[name] = {"ms_per_pass": ms, "steps_per_s": T / (ms * 1e-3),
                     "errors_vs_fp64_rts_oracle": None}
        if args.cpu_seconds <= 0:
            continue
        arrs, yy = model.arrays(), y_np
        if prec != "f64":
            cast = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
            arrs, yy = tuple(cast(a) for a in arrs), cast(y_np)
        ref = oracle.smooth_rts(*arrs, yy)
        got = [t[0].double().cpu().numpy() for t in plan.outputs()]
        errs = {k: float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))
                for k, g, r in zip(("m_filt", "P_filt", "m_smooth", "P_smooth"), got, ref)}
        errs["z_smooth_max"] = float(np.max(np.abs(got[2] - ref[2]) /
                                            np.sqrt(np.einsum("kii->ki", ref[3]))))
        res[name]["errors_vs_fp64_rts_oracle"] = errs

    # the generic look-back filter (full Lemma 1 elements, no time-invariant
    # tables) on the headline workload, and the paper's time-varying model
    # (Sec. VI-A, per-step F, Q, H, R, u, d streamed from HBM): T = 2^20, FP32
    def timed(fn, reps=20):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    def rel(got, ref):
        return {k: float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300))
                for k, g, r in zip(("m_filt", "P_filt", "m_smooth", "P_smooth"), got, ref)}

    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    T = 1 << 20
    model, y_np = W.tracking(T, seed=args.seed)
    dmodel = kfscan.model_to_device(model.arrays(), "f32", dev)
    y = torch.as_tensor(y_np).to(dev, torch.float32).contiguous()
    plan = kfscan.Plan(dmodel, y, precision="f32", scan="lookback_generic", smoother=True)
    ms = timed(lambda: (plan("kf_prepare"), plan("kf_pass_filter"), plan("kf_pass_rts")))
    res["T2^20_f32_generic_lookback_filter_rts"] = {"ms_per_pass": ms, "steps_per_s": T / (ms * 1e-3)}
    if args.cpu_seconds > 0:
        ref = oracle.smooth_rts(*(f32(a) for a in model.arrays()), f32(y_np))
        res["T2^20_f32_generic_lookback_filter_rts"]["errors_vs_fp64_rts_oracle"] = rel(
            [t[0].double().cpu().numpy() for t in plan.outputs()], ref)
    del plan, y, dmodel

    rng = np.random.default_rng(args.seed)
    tv = W.paper_tv_model(T, rng, 4, 2)
    ytv = W.simulate(tv, T, rng)
    dv = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev, torch.float32).contiguous()  # noqa: E731
    targs = [dv(a) for a in (tv.F, tv.Q, tv.H, tv.R, tv.u, tv.d, tv.m0, tv.P0, ytv)]
    outs = [None]

    def run_tv():
        outs[0] = kfscan.tv("rts", *targs, precision="f32")
    ms = timed(run_tv)
    res["paper_tv_T2^20_f32_filter_rts"] = {"ms_per_pass": ms, "steps_per_s": T / (ms * 1e-3)}
    if args.cpu_seconds > 0:
        ref = oracle.smooth_rts(*(f32(a) for a in (tv.F, tv.Q, tv.H, tv.R, tv.m0, tv.P0)), f32(ytv),
                                f32(tv.u), f32(tv.d))
        res["paper_tv_T2^20_f32_filter_rts"]["errors_vs_fp64_rts_oracle"] = rel(
            [o.double().cpu().numpy() for o in outs[0]], ref)
    return res


def bench_batched(args, np, torch, W, kfscan, dev) -> int:
    """4096 sequences, T_i = round(2^U) with U ~ U[6, 14], a random stable model
    each (rho = 0.95, Q = 0.1 I, H Gaussian, R = 0.5 I, m0 = 0, P0 = I), nx
    uniform on {2, 4, 8} with ny = nx / 2, filter + RTS smoother.  One
    kf_smooth_rts_batch call per (nx, ny) group per step, each with the scan
    and tile size the package's autotuner picked for its class (measured at
    start-up, before the timed region); value = sum of T_i per second."""
    import concurrent.futures as cf

    from paper_2511_10363_amd import autotune

    prec = args.precision
    dt = kfscan.dtype_for(prec)
    w = 8 if prec == "f64" else 4
    seqs = W.ragged_batch(nseq=args.nseq, nx_choices=(2, 4, 8), seed=args.seed)
    tuner = autotune.Autotuner()
    plans = {}
    groups = {}
    for i, (model, y) in enumerate(seqs):
        groups.setdefault((model.nx, model.ny), []).append(i)
    calls = []
    total_steps = 0
    alg_bytes = 0
    for (nx, ny), idx in sorted(groups.items()):
        lengths = np.array([len(seqs[i][1]) for i in idx], dtype=np.int64)
        offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
        y = np.concatenate([seqs[i][1] for i in idx])
        parts = [np.stack([seqs[i][0].arrays()[j] for i in idx]) for j in range(6)]
        dm = tuple(torch.as_tensor(p).to(dev, dt).contiguous() for p in parts)
        yd = torch.as_tensor(y).to(dev, dt).contiguous()
        Td = torch.as_tensor(lengths).to(dev)
        od = torch.as_tensor(offsets).to(dev)
        plan = tuner.plan("rts", nx, ny, prec, int(lengths.mean()), batched=True)
        plans["%dx%d" % (nx, ny)] = {"scan": plan["scan"], "items": plan["items"]}
        b, keep = kfscan.make_batch(dm, yd, Td, od, prec, scan=plan["scan"], smoother=True,
                                    items=plan["items"])
        ws = torch.empty(max(kfscan.batch_workspace_size(b), 1 << 20), dtype=torch.uint8,
                         device=dev)
        calls.append((b, keep, ws, dm, yd, Td, od, idx, offsets, lengths))
        total_steps += int(lengths.sum())
        alg_bytes += int(lengths.sum()) * w * (ny + 2 * nx + 2 * nx * nx)

    def one_pass():
        for c in calls:
            kfscan.run_batch("kf_smooth_rts_batch", c[0], dev, c[2])

    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    for c in calls:
        if kfscan.workspace_status(c[2]):
            raise RuntimeError("batched workload: a batch entry was refused")
    K = args.steps
    every = max(1, args.event_every)
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(K):
        if i % every == 0:
            e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            e[0].record()
            one_pass()
            e[1].record()
            evs.append(e)
        else:
            one_pass()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = total_steps * K / wall
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    achieved = alg_bytes / (lat.mean() * 1e-3) / 1e9

    # the same pass captured once into a HIP graph and replayed K times
    graph_ms = None
    if not args.no_graph:
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            with torch.cuda.graph(g, stream=side):
                one_pass()
        torch.cuda.current_stream(dev).wait_stream(side)
        for _ in range(3):
            g.replay()
        torch.cuda.synchronize()
        g0 = time.perf_counter()
        for _ in range(K):
            g.replay()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - g0) / K * 1e3
        del g
        for c in calls:
            if kfscan.workspace_status(c[2]):
                raise RuntimeError("batched workload: a batch entry was refused")

    cpu = None
    errors = None
    if args.cpu_seconds > 0:
        import oracle
        cores = len(os.sched_getaffinity(0))
        rng = np.random.default_rng(1)
        cast = (lambda a: a) if prec == "f64" else (
            lambda a: np.asarray(a, dtype=np.float32).astype(np.float64))

        def run_one(i):
            model, y = seqs[i]
            return oracle.smooth_rts(*(cast(a) for a in model.arrays()), cast(y))
        # whole passes over random subsets until the time budget is spent
        done_steps = 0
        c0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=cores) as ex:
            while time.perf_counter() - c0 < args.cpu_seconds:
                pick = rng.choice(len(seqs), size=min(len(seqs), 8 * cores), replace=False)
                list(ex.map(run_one, pick))
                done_steps += sum(len(seqs[i][1]) for i in pick)
        c1 = time.perf_counter()
        cpu = {"value": done_steps / (c1 - c0), "unit": "steps/s", "cores": cores,
               "kind": "oracle",
               "sample": "sequential FP64 filter + RTS smoother over random sequences of the "
                         "batch, one sequence per host thread, %d steps" % done_steps}
        # accuracy on a few sequences of each group
        worst = {"m_filt": 0.0, "P_filt": 0.0, "m_smooth": 0.0, "P_smooth": 0.0}
        for c in calls:
            keep, idx, offsets, lengths = c[1], c[7], c[8], c[9]
            outs = [keep[k].double().cpu().numpy() for k in ("m_filt", "P_filt", "m_smooth",
                                                             "P_smooth")]
            for j in range(0, len(idx), max(1, len(idx) // 16)):
                ref = run_one(idx[j])
                a, b = offsets[j], offsets[j] + lengths[j]
                for name, g, r in zip(worst, outs, ref):
                    e = float(np.max(np.abs(g[a:b] - r)) / max(np.max(np.abs(r)), 1e-300))
                    worst[name] = max(worst[name], e)
        errors = worst

    out = {
        "metric": "batched filter+smoother steps/s (4096 ragged sequences)",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f32": "f32", "mixed": "f32+f64solve", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "ragged_batch_%d_T2^U6-14_nx2,4,8" % args.nseq,
                   "sequences": args.nseq, "total_steps": total_steps,
                   "groups": {"%dx%d" % k: len(v) for k, v in sorted(groups.items())},
                   "pipeline": "kf_smooth_rts_batch per shape group", "seed": args.seed,
                   "autotuned": plans},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "whole pass"},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "graph_ms_per_step": graph_ms,
        "errors_vs_oracle": errors,
    }
    print(json.dumps(out))
    return 0


def bench_serving(args, np, torch, W, kfscan, dev) -> int:
    """Serving through the package's continuous-batching server
    (paper_2511_10363_amd.serving): filter + RTS jobs with nx = 16, ny = 8,
    a random stable model each (rho = 0.98, Q = 0.05 I, H Gaussian,
    R = 0.2 I, m0 = 0, P0 = I), T = round(2^U), U ~ U[10, 16], FP32 storage
    with FP64 solves (--precision, default mixed here).  The measurements of
    every job are resident on the GPU before the timed region; the server
    admits a job when its rows (measurements and outputs) and a model slot fit
    in its device arena, copies the job's data in on the stream that runs it,
    and sends the admitted jobs as ragged batches on two HIP streams.  A job
    is released (its rows and slot freed) as soon as the host sees it done.

    Measured: the saturated rate (every job submitted at t = 0), then Poisson
    arrivals at 0.5, 0.8 and 0.95 of it (latency = the host seeing the job's
    batch done - its arrival), then plain per-sequence FP64 launches
    (kf_smooth_rts, one call per job) on a sample of the jobs, with the
    batched results' distance from them."""
    from paper_2511_10363_amd import serving as S

    prec = args.precision
    dt = kfscan.dtype_for(prec)
    nx, ny = args.nx, args.nx // 2
    rng = np.random.default_rng(args.seed)
    n = args.jobs
    lengths = np.array(W.log_uniform_lengths(n, 10.0, 16.0, rng), dtype=np.int64)
    rows = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    total = int(lengths.sum())
    models = [W.random_stable_model(nx, ny, 0.98, 0.05, 0.2, rng) for _ in range(n)]
    y = np.empty((total, ny))
    for i in range(n):
        y[rows[i]:rows[i] + lengths[i]] = W.simulate(models[i], int(lengths[i]), rng)
    yd = torch.as_tensor(y).to(dev, dt).contiguous()
    ex = S.GpuExecutor(nstreams=2, device=dev)
    dmods = [ex.flat_model(m.arrays(), prec) for m in models]
    job_y = [yd[rows[i]:rows[i] + lengths[i]] for i in range(n)]
    max_batch = 256
    arena_rows = int(min(total, max(4 * int(lengths.max()), args.arena_rows)))
    srv = S.Server(ex, rows_per_class=arena_rows, slots_per_class=1024, max_batch=max_batch)
    key = (nx, ny, prec, "rts")
    sample = set(range(0, n, max(1, n // 8)))
    kept = {}

    def run(arrivals):
        """Submit jobs at their arrival times (host clock), serve until all are
        done, release each job as soon as it is seen done."""
        srv.done.clear()
        t0 = time.perf_counter()
        nxt = 0
        seen = 0
        ids = {}
        while nxt < n or not srv.idle():
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                ids[srv.submit(dmods[nxt], job_y[nxt], "rts", prec, arrival=t0 + arrivals[nxt])] = nxt
                nxt += 1
            srv.step()
            while seen < len(srv.done):
                j = srv.done[seen]
                seen += 1
                i = ids.pop(j.job_id)
                if i in sample and i not in kept:
                    kept[i] = [o.double().cpu().numpy() for o in srv.result(j.job_id)]
                srv.release(j.job_id)
        lat = np.array([(j.finished - j.arrival) * 1e3 for j in srv.done])
        span = max(j.finished for j in srv.done) - t0
        return lat, span

    run(np.zeros(n))                          # warm-up (also fills `kept`)
    torch.cuda.synchronize()
    lat_sat, sat_s = run(np.zeros(n))
    sat_jobs = n / sat_s
    results = []
    for frac in (0.5, 0.8, 0.95):
        arr = W.poisson_arrivals(n, frac * sat_jobs, np.random.default_rng(args.seed + 1))
        arr = arr - arr[0]
        lat, span = run(arr)
        results.append({"load": frac, "rate_jobs_per_s": frac * sat_jobs,
                        "p50_ms": float(np.percentile(lat, 50)),
                        "p99_ms": float(np.percentile(lat, 99)),
                        "steps_per_s": total / span})
    for st in ex.arena[key]["streams"]:
        if kfscan.workspace_status(st["ws"]) & ~kfscan.KF_WS_NUMERIC:
            raise RuntimeError("serving: a batch entry was refused or timed out")

    # plain per-sequence FP64 launches (one kf_smooth_rts call per job) on a sample
    s64 = list(range(0, n, max(1, n // 20)))
    d64 = [[torch.as_tensor(np.ascontiguousarray(a)).to(dev, torch.float64).contiguous()
            for a in models[i].arrays()] for i in s64]
    y64d = [torch.as_tensor(y[rows[i]:rows[i] + lengths[i]]).to(dev, torch.float64).contiguous()
            for i in s64]
    ws64 = torch.empty(256 << 20, dtype=torch.uint8, device=dev)
    for j in range(2):
        kfscan.smooth_rts(d64[j], y64d[j], precision="f64", workspace=ws64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res64 = [kfscan.smooth_rts(d64[j], y64d[j], precision="f64", workspace=ws64)
             for j in range(len(s64))]
    torch.cuda.synchronize()
    t64 = time.perf_counter() - t0
    steps64 = int(sum(lengths[i] for i in s64))
    dist = 0.0
    for j, i in enumerate(s64):
        if i in kept:
            ref = res64[j][2].cpu().numpy()
            dist = max(dist, float(np.max(np.abs(kept[i][2] - ref)) / np.max(np.abs(ref))))
    fp64_plain = {"jobs": len(s64), "steps": steps64, "steps_per_s": steps64 / t64,
                  "batched_steps_per_s": total / sat_s,
                  "batched_m_smooth_rel_diff_sampled": dist}

    errors = None
    if args.cpu_seconds > 0:
        import oracle
        worst = {"m_filt": 0.0, "P_filt": 0.0, "m_smooth": 0.0, "P_smooth": 0.0}
        cast = (lambda a: a) if prec == "f64" else (
            lambda a: np.asarray(a, dtype=np.float32).astype(np.float64))
        for i in sorted(kept)[:4]:
            ref = oracle.smooth_rts(*(cast(a) for a in models[i].arrays()),
                                    cast(y[rows[i]:rows[i] + lengths[i]]))
            for name, g, r in zip(worst, kept[i], ref):
                worst[name] = max(worst[name],
                                  float(np.max(np.abs(g - r)) / max(np.max(np.abs(r)), 1e-300)))
        errors = worst
    w = 8 if prec == "f64" else 4
    step_bytes = w * (ny + 2 * nx + 2 * nx * nx)
    out = {
        "metric": "serving: saturated steps/s and p50/p99 job latency under Poisson arrivals",
        "value": total / sat_s, "unit": "steps/s", "n_gpus": 1, "steps": n,
        "warmup": 1, "ms_per_step": sat_s / n * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f32": "f32", "mixed": "f32+f64solve", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "serving_%d_jobs_T2^U10-16_nx%d_ny%d" % (n, nx, ny), "jobs": n,
                   "total_steps": total, "max_batch": max_batch, "streams": 2,
                   "arena_rows": arena_rows, "arena_bytes": srv.capacity_bytes(key),
                   "seed": args.seed},
        "saturated_jobs_per_s": sat_jobs,
        "saturated_latency_ms": {"p50": float(np.percentile(lat_sat, 50)),
                                 "p99": float(np.percentile(lat_sat, 99))},
        "hbm_frac_saturated": total / sat_s * step_bytes / (HBM_PEAK_GBS * 1e9),
        "poisson": results,
        "fp64_per_sequence": fp64_plain,
        "errors_vs_oracle": errors,
    }
    print(json.dumps(out))
    return 0


def bench_tv(args, np, torch, W, kfscan, dev) -> int:
    """The paper's time-varying model (Sec. VI-A): per step F_k = 0.99 x an
    orthogonal factor, random SPD Q_k, R_k, Gaussian H_k, u_k, d_k; nx = 4,
    ny = 2; filter + RTS smoother (kf_smooth_rts_tv), T = 2^log2T.  The
    per-step model is streamed from HBM: algorithmic bytes per step are
    w (m + 2n^2 + mn + m^2 + n + m + 2n + 2n^2) (y, the step's model, both
    output pairs); the RTS pass reads F, Q, u again, which counts against."""
    prec = args.precision
    dt = kfscan.dtype_for(prec)
    w = 8 if prec == "f64" else 4
    T = args.T if args.T > 0 else 1 << args.log2T
    n, m = 4, 2
    rng = np.random.default_rng(args.seed)
    model = W.paper_tv_model(T, rng, n, m)
    y = W.simulate(model, T, rng)
    dv = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt).contiguous()  # noqa: E731
    F, Q, H, R, u, d = (dv(a) for a in (model.F, model.Q, model.H, model.R, model.u, model.d))
    m0, P0, yd = dv(model.m0), dv(model.P0), dv(y)
    ws = [None]

    def one_pass():
        outs = kfscan.tv("rts", F, Q, H, R, u, d, m0, P0, yd, precision=prec, workspace=ws[0])
        return outs

    outs = one_pass()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        one_pass()
    torch.cuda.synchronize()
    K = args.steps
    every = max(1, args.event_every)
    evs = []
    t0 = time.perf_counter()
    for i in range(K):
        if i % every == 0:
            e = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            e[0].record()
            outs = one_pass()
            e[1].record()
            evs.append(e)
        else:
            outs = one_pass()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = T * K / wall
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    step_bytes = w * (m + 2 * n * n + m * n + m * m + n + m + 2 * n + 2 * n * n)
    achieved = T * step_bytes / (lat.mean() * 1e-3) / 1e9
    cpu = errors = None
    if args.cpu_seconds > 0:
        import oracle
        cast = (lambda a: a) if prec == "f64" else (
            lambda a: np.asarray(a, dtype=np.float32).astype(np.float64))
        arrs = [cast(a) for a in (model.F, model.Q, model.H, model.R, model.m0, model.P0)]
        reps = 0
        c0 = time.perf_counter()
        while True:
            ref = oracle.smooth_rts(*arrs, cast(y), cast(model.u), cast(model.d))
            reps += 1
            if time.perf_counter() - c0 >= args.cpu_seconds:
                break
        cpu = {"value": T * reps / (time.perf_counter() - c0), "unit": "steps/s", "cores": 1,
               "kind": "oracle",
               "sample": "sequential FP64 filter + RTS smoother, time-varying model, T=%d, "
                         "%d repetition(s)" % (T, reps)}
        got = [o.double().cpu().numpy() for o in outs]
        errors = {name: float(np.max(np.abs(g - r)) / np.max(np.abs(r)))
                  for name, g, r in zip(("m_filt", "P_filt", "m_smooth", "P_smooth"), got, ref)}
    out = {
        "metric": "time-varying filter+smoother steps/s (the paper's model, nx=4, ny=2)",
        "value": value, "unit": "steps/s", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": wall / K * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"f32": "f32", "mixed": "f32+f64solve", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "paper_tv_nx4_ny2_T%d" % T, "T": T, "inputs": "u, d",
                   "pipeline": "kf_smooth_rts_tv", "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "whole pass"},
        "cpu_baseline": cpu,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
        "errors_vs_oracle": errors,
    }
    print(json.dumps(out))
    return 0


def bench_speedup(args, np, torch, W, kfscan, dev) -> int:
    """The speedup experiment of Sec. VI (GPU speedup analysis): the parallel
    Kalman filter (Algorithm 5, look-back scan over full elements) against the
    classical sequential filter run by one GPU lane (KF_SCAN_SEQUENTIAL), FP32,
    on the paper's time-varying model (nx = 4, ny = 2, inputs u, d), for
    T = 10^2 .. 10^6 and 2^20.  Both are timed with events around the one-call
    entry point kf_filter_tv (the sequential one once per length after a
    warm-up call, the parallel one as the median of --steps calls).  The model
    and measurements are drawn once at the largest length; each shorter case
    takes their first T steps."""
    prec = args.precision
    dt = kfscan.dtype_for(prec)
    Ts = [100, 1000, 10000, 100000, 1000000, 1 << 20]
    Tmax = max(Ts)
    n, m = 4, 2
    rng = np.random.default_rng(args.seed)
    model = W.paper_tv_model(Tmax, rng, n, m)
    y = W.simulate(model, Tmax, rng)
    dv = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt).contiguous()  # noqa: E731
    full = [dv(a) for a in (model.F, model.Q, model.H, model.R, model.u, model.d)]
    m0, P0, yd = dv(model.m0), dv(model.P0), dv(y)

    def timed(T, scan, reps):
        args_T = [a[:T] for a in full]
        ms = []
        outs = None
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            outs = kfscan.tv("filter", *args_T, m0, P0, yd[:T], precision=prec, scan=scan)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return float(np.median(ms)), outs

    curve = []
    for T in Ts:
        timed(min(T, 1000), "sequential", 1)               # warm-up
        t_seq, seq_out = timed(T, "sequential", 1)
        timed(T, "lookback", max(1, args.warmup))
        t_par, par_out = timed(T, "lookback", max(3, min(args.steps, 50)))
        timed(T, "ladner_fischer", 1)
        t_lf, _ = timed(T, "ladner_fischer", max(3, min(args.steps, 20)))
        diff = float((seq_out[0] - par_out[0]).abs().max() / seq_out[0].abs().max())
        curve.append({"T": T, "sequential_ms": t_seq, "parallel_ms": t_par,
                      "speedup": t_seq / t_par, "ladner_fischer_ms": t_lf,
                      "speedup_ladner_fischer": t_seq / t_lf, "m_filt_rel_diff": diff})
        print("[speedup] T=%d sequential %.3f ms look-back %.4f ms (x%.1f) "
              "Ladner-Fischer %.4f ms (x%.1f)" % (T, t_seq, t_par, t_seq / t_par, t_lf,
                                                   t_seq / t_lf), file=sys.stderr, flush=True)
    top = curve[-1]
    out = {
        "metric": "speedup of the parallel Kalman filter over the sequential filter on one GPU lane",
        "value": top["speedup"], "unit": "x", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": top["parallel_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "mixed": "f32+f64solve", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "paper_tv_nx4_ny2_speedup", "T": Ts, "inputs": "u, d",
                   "pipeline": "kf_filter_tv: look-back scan (value) and in-place "
                               "Ladner-Fischer against the sequential filter",
                   "seed": args.seed},
        "paper": "up to about 750 (Apple M3 Max) and 500 (A100), FP32, in-place Ladner-Fischer",
        "curve": curve,
    }
    print(json.dumps(out))
    return 0


def bench_scans(args, np, torch, W, kfscan, dev) -> int:
    """The paper's comparison of scan algorithms (Sec. VI-B..D): PKF, PRTS and
    PTFS with every scan -- the look-back scan over full elements, the
    one-kernel-per-level Hillis-Steele, Blelloch, in-place Ladner-Fischer,
    Sengupta A and B -- and the sequential recursions, on the paper's
    time-varying model (nx = 4, ny = 2, inputs), FP32, T = 10^3 .. 10^6.
    Each cell is the median of event-timed one-call runs (kf_*_tv).  The model
    and data are drawn once at 10^6 steps; shorter cases take their first T."""
    prec = args.precision
    dt = kfscan.dtype_for(prec)
    Ts = [1000, 10000, 100000, 1000000]
    scans = ["lookback", "hillis_steele", "blelloch", "ladner_fischer", "sengupta_a",
             "sengupta_b", "sequential"]
    n, m = 4, 2
    rng = np.random.default_rng(args.seed)
    model = W.paper_tv_model(max(Ts), rng, n, m)
    y = W.simulate(model, max(Ts), rng)
    dv = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to(dev, dt).contiguous()  # noqa: E731
    full = [dv(a) for a in (model.F, model.Q, model.H, model.R, model.u, model.d)]
    m0, P0, yd = dv(model.m0), dv(model.P0), dv(y)
    table = []
    for T in Ts:
        arrs = [a[:T] for a in full]
        for scan in scans:
            row = {"T": T, "scan": scan}
            for entry in ("filter", "rts", "tf"):
                reps = 1 if scan == "sequential" else max(3, min(args.steps, 10))
                kfscan.tv(entry, *arrs, m0, P0, yd[:T], precision=prec, scan=scan)
                ms = []
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record()
                    kfscan.tv(entry, *arrs, m0, P0, yd[:T], precision=prec, scan=scan)
                    e1.record()
                    torch.cuda.synchronize()
                    ms.append(e0.elapsed_time(e1))
                row[{"filter": "PKF_ms", "rts": "PRTS_ms", "tf": "PTFS_ms"}[entry]] = \
                    float(np.median(ms))
            if scan not in ("lookback", "sequential"):
                row["combines"], row["steps"] = kfscan.scan_counts(scan, T)
            table.append(row)
            print("[scans] T=%d %-15s PKF %.3f  PRTS %.3f  PTFS %.3f ms" %
                  (T, scan, row["PKF_ms"], row["PRTS_ms"], row["PTFS_ms"]), file=sys.stderr,
                  flush=True)
    best = min((r for r in table if r["T"] == max(Ts)), key=lambda r: r["PKF_ms"])
    out = {
        "metric": "time of one PKF / PRTS / PTFS call per scan algorithm (the paper's model)",
        "value": best["PKF_ms"], "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": 1, "ms_per_step": best["PKF_ms"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"f32": "f32", "mixed": "f32+f64solve", "f64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "paper_tv_nx4_ny2_scan_comparison", "T": Ts, "scans": scans,
                   "fastest_PKF_at_1e6": best["scan"], "seed": args.seed},
        "table": table,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
