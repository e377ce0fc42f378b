"""Autotuner of the scan schedule: which scan algorithm and which tile size
(steps per thread, the ``items`` of the C ABI) to use for a workload class.

The paper compares scan algorithms on each GPU and tunes Sengupta's
threshold per platform (Sec. VI): the best schedule depends on the machine,
the state size and the length.  Here a class is (entry, nx, ny, precision,
log2 T rounded, single sequence or ragged batch); ``plan`` times every
candidate schedule on a synthetic problem of that class -- a random stable
model and Gaussian measurements, which is all the kernels' timing depends
on -- keeps the fastest, and caches the plans in a JSON file, so a class is
measured once per machine.  Timing is the median of several event-timed
calls after warm-up on the current HIP stream.
"""
from __future__ import annotations

import json
import math
import os

import numpy as np

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "kfscan", "plans.json")

# (scan, items): items 0 is the library's own choice
NARROW = [("lookback", 0), ("lookback", 2), ("lookback", 4), ("lookback", 8), ("lookback", 16),
          ("lookback_generic", 0), ("lookback_generic", 4), ("sengupta_b", 0),
          ("ladner_fischer", 0)]
NARROW_BATCH = [("lookback", 0), ("lookback", 2), ("lookback", 4), ("lookback", 8),
                ("lookback_generic", 0), ("lookback_generic", 4)]
WIDE = [("lookback", 0)]


def bucket(T: int) -> int:
    return int(round(math.log2(max(int(T), 1))))


def class_key(entry: str, nx: int, ny: int, precision: str, T: int, batched: bool = False) -> str:
    return "%s|nx%d|ny%d|%s|2^%d|%s" % (entry, nx, ny, precision, bucket(T),
                                        "batch" if batched else "single")


def candidates(nx: int, batched: bool):
    if nx > 4:
        return list(WIDE)
    return list(NARROW_BATCH if batched else NARROW)


class Autotuner:
    """Plans per workload class, measured on first use and cached.

    ``measure(entry, nx, ny, precision, T, batched, scan, items) -> ms`` times
    one candidate; the default runs it on the GPU through ``kfscan``.  A
    candidate the library refuses (KF_ERR_UNSUPPORTED) is skipped."""

    def __init__(self, cache_path: str | None = None, measure=None, reps: int = 5,
                 seed: int = 1234):
        self.cache_path = cache_path or os.environ.get("KFSCAN_TUNE_CACHE", DEFAULT_CACHE)
        self.reps = reps
        self.seed = seed
        self.measure = measure or self._measure_gpu
        self.plans = {}
        if self.cache_path and os.path.exists(self.cache_path):
            with open(self.cache_path) as f:
                self.plans = json.load(f)

    def plan(self, entry: str, nx: int, ny: int, precision: str, T: int,
             batched: bool = False) -> dict:
        key = class_key(entry, nx, ny, precision, T, batched)
        p = self.plans.get(key)
        if p is None:
            p = self.tune(entry, nx, ny, precision, T, batched)
        return p

    def tune(self, entry, nx, ny, precision, T, batched=False) -> dict:
        key = class_key(entry, nx, ny, precision, T, batched)
        Tb = 1 << bucket(T)
        times = {}
        for scan, items in candidates(nx, batched):
            try:
                ms = float(self.measure(entry, nx, ny, precision, Tb, batched, scan, items))
            except Exception as e:  # noqa: BLE001 -- an unsupported candidate is skipped
                if type(e).__name__ != "KfScanError":
                    raise
                continue
            times["%s/%d" % (scan, items)] = ms
        if not times:
            raise RuntimeError("no candidate schedule runs for %s" % key)
        best = min(times, key=times.get)
        scan, items = best.split("/")
        p = {"scan": scan, "items": int(items), "ms": times[best], "T": Tb, "times": times}
        self.plans[key] = p
        self.save()
        return p

    def save(self) -> None:
        if not self.cache_path:
            return
        d = os.path.dirname(self.cache_path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = self.cache_path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(self.plans, f, indent=1, sort_keys=True)
        os.replace(tmp, self.cache_path)

    # -- measurement on the GPU ------------------------------------------------
    def _synthetic(self, nx, ny, precision, T, nseq, device):
        import torch

        from . import kfscan

        rng = np.random.default_rng(self.seed + 31 * nx + ny)
        G = rng.standard_normal((nx, nx))
        F = 0.95 * G / max(abs(np.linalg.eigvals(G)))
        H = rng.standard_normal((ny, nx))
        model = (F, 0.1 * np.eye(nx), H, 0.5 * np.eye(ny), np.zeros(nx), np.eye(nx))
        dm = kfscan.model_to_device(model, precision, device)
        y = torch.as_tensor(rng.standard_normal((nseq, T, ny))).to(
            device, kfscan.dtype_for(precision)).contiguous()
        return dm, y

    def _measure_gpu(self, entry, nx, ny, precision, T, batched, scan, items) -> float:
        import torch

        from . import kfscan

        dev = torch.device("cuda", torch.cuda.current_device())
        if batched:
            # 64 sequences of about T steps (0.5 T .. 1.5 T), a shared model
            nseq = 64
            rng = np.random.default_rng(self.seed)
            lens = np.maximum(1, (T * rng.uniform(0.5, 1.5, nseq)).astype(np.int64))
            total = int(lens.sum())
            dm, y = self._synthetic(nx, ny, precision, total, 1, dev)
            y = y[0]
            Td = torch.as_tensor(lens).to(dev)
            off = torch.as_tensor(np.concatenate([[0], np.cumsum(lens)[:-1]])).to(dev)

            def call():
                kfscan.batch(entry, dm, y, Td, off, precision=precision, scan=scan, items=items)
        else:
            dm, y = self._synthetic(nx, ny, precision, T, 1, dev)
            fn = {"filter": kfscan.filter, "rts": kfscan.smooth_rts,
                  "tf": kfscan.smooth_twofilter}[entry]

            def call():
                fn(dm, y, precision=precision, scan=scan, items=items)
        for _ in range(2):
            call()
        torch.cuda.synchronize()
        ts = []
        for _ in range(self.reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            call()
            e1.record()
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))


def tuned(entry: str, model, y, precision: str = "f32", tuner: Autotuner | None = None,
          **kw):
    """Run ``kfscan``'s filter / smoother with the tuned schedule of its class."""
    from . import kfscan

    tuner = tuner or Autotuner()
    F = model[0] if isinstance(model, (tuple, list)) else model.F
    H = model[2] if isinstance(model, (tuple, list)) else model.H
    T = y.shape[-2]
    p = tuner.plan(entry, int(F.shape[-1]), int(H.shape[-2]), precision, int(T))
    fn = {"filter": kfscan.filter, "rts": kfscan.smooth_rts,
          "tf": kfscan.smooth_twofilter}[entry]
    return fn(model, y, precision=precision, scan=p["scan"], items=p["items"], **kw)
