"""Continuous-batching server for filter / smoother jobs on one GPU.

A job is one model (F, Q, H, R, m0, P0) and one measurement sequence y of T
steps; the work is a filter (Algorithm 5), RTS smoother (Algorithm 6) or
two-filter smoother (Algorithm 7) pass over it.  Jobs arrive over time:

* **Admission by HBM footprint.**  Each shape class (nx, ny, precision,
  entry) owns a device arena of rows: a job needs T contiguous rows of
  measurements and outputs plus one model slot, i.e. ``footprint_bytes``.
  A job is admitted (in arrival order) as soon as its rows and a slot are
  free; until then it waits in the queue, which is the server's
  backpressure.  The arena and every per-stream buffer are allocated once,
  when the class is created, so serving allocates no device memory.
* **Device-resident state.**  An admitted job's measurements are copied into
  its rows and its model into its slot, on the stream that will run it; its
  results are written in place and stay there until ``release``.
* **Continuous batching.**  Whenever a stream is idle, the admitted jobs not
  yet launched go out on it as one ragged batch (``kf_*_batch`` with
  ``offset`` = the jobs' arena rows, a model per sequence), up to
  ``max_batch`` jobs.  Jobs that arrive while batches run are admitted as
  rows free up and are sent on the next idle stream, so their work overlaps
  the running batches.
* **Reproducibility.**  A ragged batch takes the same tiles for a sequence
  whatever else it holds, so a job's results are bit-identical alone and in
  any mix.

The device work goes through an executor; ``GpuExecutor`` drives the C ABI
(via ``kfscan``) on HIP streams, and any object with the same three methods
(``launch``, ``done``, ``wait``) can stand in for it, e.g. a simulated one in
tests.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable

import numpy as np

ENTRIES = ("filter", "rts", "tf")


def word_bytes(precision: str) -> int:
    return 8 if precision == "f64" else 4


def row_bytes(nx: int, ny: int, precision: str, entry: str) -> int:
    """HBM bytes per time step of a job: its measurement row and its output rows
    (filter moments, and smoothed moments for the smoothers)."""
    pairs = 1 if entry == "filter" else 2
    return word_bytes(precision) * (ny + pairs * (nx + nx * nx))


def model_bytes(nx: int, ny: int, precision: str) -> int:
    """HBM bytes of one model: F, Q, P0 (nx x nx), H (ny x nx), R (ny x ny), m0."""
    return word_bytes(precision) * (3 * nx * nx + ny * nx + ny * ny + nx)


def footprint_bytes(T: int, nx: int, ny: int, precision: str, entry: str) -> int:
    """Device memory a job holds while admitted: T rows and one model slot."""
    return T * row_bytes(nx, ny, precision, entry) + model_bytes(nx, ny, precision)


# ---------------------------------------------------------------------------
# Row allocator: first fit over [0, nrows), coalescing on free.
# ---------------------------------------------------------------------------
class RowAllocator:
    def __init__(self, nrows: int):
        if nrows < 1:
            raise ValueError("nrows must be positive")
        self.nrows = nrows
        self._free = [(0, nrows)]        # sorted, disjoint (start, length)
        self.used = 0

    def alloc(self, n: int):
        """First row of a free range of n rows, or None if no range fits."""
        if n < 1:
            raise ValueError("n must be positive")
        for i, (s, length) in enumerate(self._free):
            if length >= n:
                if length == n:
                    del self._free[i]
                else:
                    self._free[i] = (s + n, length - n)
                self.used += n
                return s
        return None

    def free(self, start: int, n: int) -> None:
        lo, hi = 0, len(self._free)
        while lo < hi:
            mid = (lo + hi) // 2
            if self._free[mid][0] < start:
                lo = mid + 1
            else:
                hi = mid
        i = lo
        if i > 0:
            ps, pl = self._free[i - 1]
            if ps + pl > start:
                raise ValueError("double free of rows %d..%d" % (start, start + n))
        if i < len(self._free) and start + n > self._free[i][0]:
            raise ValueError("double free of rows %d..%d" % (start, start + n))
        self._free.insert(i, (start, n))
        # coalesce with the neighbours
        if i + 1 < len(self._free) and start + n == self._free[i + 1][0]:
            self._free[i] = (start, n + self._free[i + 1][1])
            del self._free[i + 1]
        if i > 0 and self._free[i - 1][0] + self._free[i - 1][1] == start:
            self._free[i - 1] = (self._free[i - 1][0], self._free[i - 1][1] + self._free[i][1])
            del self._free[i]
        self.used -= n

    def largest_free(self) -> int:
        return max((length for _, length in self._free), default=0)


# ---------------------------------------------------------------------------
# Jobs and batches
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class Job:
    job_id: int
    key: tuple                    # (nx, ny, precision, entry)
    T: int
    model: tuple                  # F, Q, H, R, m0, P0 (host arrays or device tensors)
    y: object                     # [T, ny] host array or device tensor
    arrival: float
    row: int = -1                 # first arena row once admitted
    slot: int = -1                # model slot once admitted
    admitted: float = -1.0
    launched: float = -1.0
    finished: float = -1.0
    batch: int = -1

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class Batch:
    batch_id: int
    key: tuple
    stream: int
    jobs: list
    token: object = None


class ShapeClass:
    """Arena bookkeeping of one (nx, ny, precision, entry): rows and slots."""

    def __init__(self, key, rows: int, slots: int):
        self.key = key
        self.rows = RowAllocator(rows)
        self.nrows = rows
        self.nslots = slots
        self._slots = list(range(slots - 1, -1, -1))

    def admit(self, job: Job) -> bool:
        if not self._slots:
            return False
        row = self.rows.alloc(job.T)
        if row is None:
            return False
        job.row = row
        job.slot = self._slots.pop()
        return True

    def release(self, job: Job) -> None:
        self.rows.free(job.row, job.T)
        self._slots.append(job.slot)
        job.row = job.slot = -1


class Server:
    """The admission / batching loop.  ``submit`` queues a job, ``step`` does one
    round of completion polling, admission and dispatch, ``result`` gives a
    finished job's outputs, ``release`` returns its rows and slot."""

    def __init__(self, executor, rows_per_class: int, slots_per_class: int = 4096,
                 max_batch: int = 256, clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.rows_per_class = rows_per_class
        self.slots_per_class = slots_per_class
        self.max_batch = max_batch
        self.clock = clock
        self.classes: dict = {}
        self.queue: collections.deque = collections.deque()   # waiting for admission
        self.ready: dict = collections.defaultdict(collections.deque)  # admitted, not launched
        self.running: dict = {}                                # stream -> Batch
        self.jobs: dict = {}
        self.done: list = []
        self._next_job = 0
        self._next_batch = 0

    # -- bookkeeping ---------------------------------------------------------
    def shape_class(self, key) -> ShapeClass:
        sc = self.classes.get(key)
        if sc is None:
            sc = ShapeClass(key, self.rows_per_class, self.slots_per_class)
            self.ex.create_class(key, self.rows_per_class, self.slots_per_class, self.max_batch)
            self.classes[key] = sc
        return sc

    def capacity_bytes(self, key) -> int:
        nx, ny, prec, entry = key
        return (self.rows_per_class * row_bytes(nx, ny, prec, entry)
                + self.slots_per_class * model_bytes(nx, ny, prec))

    def submit(self, model, y, entry: str = "rts", precision: str = "f32",
               arrival: float | None = None) -> int:
        if entry not in ENTRIES:
            raise ValueError("entry must be one of %s" % (ENTRIES,))
        T = int(y.shape[0])
        ny = int(y.shape[1])
        if isinstance(model, (tuple, list)):
            nx = int(model[0].shape[-1])
        else:
            # a flat model: 3 nx^2 + ny nx + ny^2 + nx values
            w = int(model.shape[0]) - ny * ny
            nx = int(round((-(ny + 1) + ((ny + 1) ** 2 + 12 * w) ** 0.5) / 6))
            if 3 * nx * nx + ny * nx + nx != w:
                raise ValueError("a flat model must hold F, Q, H, R, m0, P0 back to back")
        if T < 1:
            raise ValueError("a job needs at least one step")
        if T > self.rows_per_class:
            raise ValueError("a job of %d steps can never fit the %d-row arena"
                             % (T, self.rows_per_class))
        job = Job(self._next_job, (nx, ny, precision, entry), T,
                  tuple(model) if isinstance(model, (tuple, list)) else model, y,
                  self.clock() if arrival is None else arrival)
        self._next_job += 1
        self.jobs[job.job_id] = job
        self.shape_class(job.key)
        self.queue.append(job)
        return job.job_id

    # -- the loop --------------------------------------------------------------
    def _complete(self) -> int:
        n = 0
        for s in list(self.running):
            b = self.running[s]
            if self.ex.done(b.token):
                t = self.clock()
                for j in b.jobs:
                    j.finished = t
                    self.done.append(j)
                del self.running[s]
                n += 1
        return n

    def _admit(self) -> int:
        n = 0
        while self.queue:
            job = self.queue[0]
            sc = self.classes[job.key]
            if not sc.admit(job):
                break                         # backpressure: wait for rows or a slot
            self.queue.popleft()
            job.admitted = self.clock()
            self.ready[job.key].append(job)
            n += 1
        return n

    def _dispatch(self) -> int:
        n = 0
        for s in range(self.ex.nstreams):
            if s in self.running:
                continue
            # the class whose oldest admitted job has waited longest
            keys = [k for k, q in self.ready.items() if q]
            if not keys:
                break
            key = min(keys, key=lambda k: self.ready[k][0].arrival)
            q = self.ready[key]
            jobs = [q.popleft() for _ in range(min(self.max_batch, len(q)))]
            b = Batch(self._next_batch, key, s, jobs)
            self._next_batch += 1
            t = self.clock()
            for j in jobs:
                j.launched = t
                j.batch = b.batch_id
            b.token = self.ex.launch(s, key, jobs)
            self.running[s] = b
            n += 1
        return n

    def step(self) -> bool:
        """One round; True if anything changed."""
        c = self._complete()
        a = self._admit()
        d = self._dispatch()
        return bool(c or a or d)

    def idle(self) -> bool:
        return not self.queue and not self.running and not any(self.ready.values())

    def drain(self, poll: Callable[[], None] | None = None) -> None:
        while not self.idle():
            if not self.step() and poll is not None:
                poll()

    def result(self, job_id: int):
        job = self.jobs[job_id]
        if job.finished < 0:
            raise RuntimeError("job %d has not finished" % job_id)
        return self.ex.outputs(job)

    def release(self, job_id: int) -> None:
        job = self.jobs.pop(job_id)
        if job.row >= 0:
            self.classes[job.key].release(job)

    def latency_percentiles(self, qs=(50, 99)) -> dict:
        lat = np.array([j.latency for j in self.done])
        return {"p%d" % q: float(np.percentile(lat, q)) for q in qs} if lat.size else {}


# ---------------------------------------------------------------------------
# The GPU executor: arenas on the device, one workspace and staging set per
# stream, batches through the C ABI.
# ---------------------------------------------------------------------------
class GpuExecutor:
    """Runs batches with ``kfscan`` on ``nstreams`` HIP streams (all at the
    default priority).  Every device buffer is allocated in ``create_class``.

    A job's model may be given as the tuple (F, Q, H, R, m0, P0) or as one
    flat tensor of those values back to back (``flat_model``); either is
    copied into the job's slot of the class's model arena with one copy."""

    def __init__(self, nstreams: int = 2, device="cuda:0"):
        import torch

        from . import kfscan

        self.torch = torch
        self.k = kfscan
        self.k.load_library()
        self.device = torch.device(device)
        self.nstreams = nstreams
        self.streams = [torch.cuda.Stream(self.device) for _ in range(nstreams)]
        self.arena: dict = {}

    @staticmethod
    def model_shapes(nx: int, ny: int):
        return ((nx, nx), (nx, nx), (ny, nx), (ny, ny), (nx,), (nx, nx))

    def flat_model(self, model, precision: str):
        """The model's six arrays back to back as one device tensor."""
        torch = self.torch
        dt = self.k.dtype_for(precision)
        return torch.cat([torch.as_tensor(a).to(self.device, dt).reshape(-1) for a in model])

    def create_class(self, key, rows: int, slots: int, max_batch: int) -> None:
        torch = self.torch
        nx, ny, prec, entry = key
        dt = self.k.dtype_for(prec)
        dev = self.device
        shapes = self.model_shapes(nx, ny)
        sizes = [int(np.prod(sh)) for sh in shapes]
        a = dict(
            y=torch.zeros((rows, ny), dtype=dt, device=dev),
            m_f=torch.zeros((rows, nx), dtype=dt, device=dev),
            P_f=torch.zeros((rows, nx, nx), dtype=dt, device=dev),
            model=torch.zeros((slots, sum(sizes)), dtype=dt, device=dev),
            shapes=shapes, sizes=sizes,
        )
        if entry != "filter":
            a["m_s"] = torch.zeros((rows, nx), dtype=dt, device=dev)
            a["P_s"] = torch.zeros((rows, nx, nx), dtype=dt, device=dev)
        per_stream = []
        for _ in range(self.nstreams):
            st = dict(
                T=torch.zeros(max_batch, dtype=torch.int64, device=dev),
                off=torch.zeros(max_batch, dtype=torch.int64, device=dev),
                slots=torch.zeros(max_batch, dtype=torch.int64, device=dev),
                host=torch.zeros((3, max_batch), dtype=torch.int64).pin_memory(),
                model=[torch.zeros((max_batch,) + sh, dtype=dt, device=dev) for sh in shapes],
                event=torch.cuda.Event(),
            )
            # the workspace for the largest batch over the whole arena
            b, _ = self.k.make_batch(tuple(st["model"]), a["y"], st["T"], st["off"],
                                     precision=prec, smoother=(entry != "filter"),
                                     outputs=self._outs(a, entry))
            need = self.k.batch_workspace_size(b)
            st["ws"] = torch.empty(max(need, 1 << 20), dtype=torch.uint8, device=dev)
            per_stream.append(st)
        a["streams"] = per_stream
        self.arena[key] = a

    @staticmethod
    def _outs(a, entry):
        return (a["m_f"], a["P_f"]) + ((a["m_s"], a["P_s"]) if entry != "filter" else ())

    def launch(self, s: int, key, jobs):
        torch = self.torch
        a = self.arena[key]
        st = a["streams"][s]
        nx, ny, prec, entry = key
        n = len(jobs)
        stream = self.streams[s]
        host = st["host"]
        for i, j in enumerate(jobs):
            host[0, i] = j.T
            host[1, i] = j.row
            host[2, i] = j.slot
        with torch.cuda.stream(stream):
            # the jobs' data into their rows and slots, on this stream
            for j in jobs:
                a["y"][j.row:j.row + j.T].copy_(torch.as_tensor(j.y), non_blocking=True)
                m = j.model
                if isinstance(m, torch.Tensor):
                    a["model"][j.slot].copy_(m, non_blocking=True)
                else:
                    a["model"][j.slot].copy_(self.flat_model(m, prec), non_blocking=True)
            st["T"][:n].copy_(host[0, :n], non_blocking=True)
            st["off"][:n].copy_(host[1, :n], non_blocking=True)
            st["slots"][:n].copy_(host[2, :n], non_blocking=True)
            col = 0
            for dst, size in zip(st["model"], a["sizes"]):
                torch.index_select(a["model"][:, col:col + size], 0, st["slots"][:n],
                                   out=dst[:n].view(n, size))
                col += size
            b, keep = self.k.make_batch(tuple(m[:n] for m in st["model"]), a["y"], st["T"][:n],
                                        st["off"][:n], precision=prec,
                                        smoother=(entry != "filter"),
                                        outputs=self._outs(a, entry))
            name = {"filter": "kf_filter_batch", "rts": "kf_smooth_rts_batch",
                    "tf": "kf_smooth_twofilter_batch"}[entry]
            self.k.run_batch(name, b, self.device, workspace=st["ws"])
            st["event"].record(stream)
        return st["event"]

    def done(self, token) -> bool:
        return token.query()

    def wait(self, token) -> None:
        token.synchronize()

    def outputs(self, job):
        a = self.arena[job.key]
        sl = slice(job.row, job.row + job.T)
        outs = [a["m_f"][sl], a["P_f"][sl]]
        if job.key[3] != "filter":
            outs += [a["m_s"][sl], a["P_s"][sl]]
        return outs
