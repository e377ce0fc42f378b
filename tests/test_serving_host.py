"""Host logic of the continuous-batching server (paper_2511_10363_amd.serving)
with a simulated executor: admission by HBM footprint, backpressure, batching
of jobs that arrive while others run, completion, release.  No GPU."""
import numpy as np
import pytest

from paper_2511_10363_amd import serving as S


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Batches take `cost(jobs)` seconds of simulated time on their stream."""

    def __init__(self, clock, nstreams=2, cost=lambda jobs: 1e-3 + 1e-6 * sum(j.T for j in jobs)):
        self.clock = clock
        self.nstreams = nstreams
        self.cost = cost
        self.classes = []
        self.launched = []

    def create_class(self, key, rows, slots, max_batch):
        self.classes.append((key, rows, slots, max_batch))

    def launch(self, s, key, jobs):
        self.launched.append((s, key, [j.job_id for j in jobs]))
        return self.clock() + self.cost(jobs)

    def done(self, token):
        return self.clock() >= token

    def wait(self, token):
        self.clock.t = max(self.clock.t, token)

    def outputs(self, job):
        return ("rows", job.row, job.T)


def _model(nx=4, ny=2):
    return (np.eye(nx), np.eye(nx), np.ones((ny, nx)), np.eye(ny), np.zeros(nx), np.eye(nx))


def _y(T, ny=2):
    return np.zeros((T, ny))


def test_footprint_counts_rows_and_model():
    assert S.row_bytes(4, 2, "f32", "rts") == 4 * (2 + 2 * (4 + 16))
    assert S.row_bytes(4, 2, "f64", "filter") == 8 * (2 + 4 + 16)
    assert S.model_bytes(16, 8, "f32") == 4 * (3 * 256 + 128 + 64 + 16)
    assert S.footprint_bytes(1000, 16, 8, "f32", "rts") == \
        1000 * 4 * (8 + 2 * (16 + 256)) + S.model_bytes(16, 8, "f32")


def test_row_allocator_first_fit_and_coalescing():
    a = S.RowAllocator(100)
    r1, r2, r3 = a.alloc(30), a.alloc(30), a.alloc(30)
    assert (r1, r2, r3) == (0, 30, 60)
    assert a.alloc(20) is None
    a.free(r2, 30)
    assert a.largest_free() == 30
    assert a.alloc(25) == 30
    a.free(30, 25)
    a.free(r1, 30)
    a.free(r3, 30)
    assert a.largest_free() == 100 and a.used == 0
    with pytest.raises(ValueError):
        a.free(0, 10)


def test_admission_waits_for_rows_backpressure():
    clock = FakeClock()
    ex = FakeExecutor(clock, nstreams=1)
    srv = S.Server(ex, rows_per_class=1000, slots_per_class=8, max_batch=8, clock=clock)
    a = srv.submit(_model(), _y(600))
    b = srv.submit(_model(), _y(600))      # does not fit beside a
    c = srv.submit(_model(), _y(300))      # would fit, but waits behind b (arrival order)
    srv.step()
    assert srv.jobs[a].row == 0 and srv.jobs[b].row == -1 and srv.jobs[c].row == -1
    assert len(srv.queue) == 2
    clock.t = 1.0
    srv.step()                              # a finishes; its rows stay held until release
    assert srv.jobs[a].finished == 1.0
    assert srv.jobs[b].row == -1
    srv.release(a)
    srv.step()                              # now b and c are admitted and batched together
    assert srv.jobs[b].row >= 0 and srv.jobs[c].row >= 0
    assert srv.jobs[b].batch == srv.jobs[c].batch
    assert srv.classes[(4, 2, "f32", "rts")].rows.used == 900


def test_slots_limit_admission():
    clock = FakeClock()
    ex = FakeExecutor(clock, nstreams=1)
    srv = S.Server(ex, rows_per_class=10000, slots_per_class=2, max_batch=8, clock=clock)
    ids = [srv.submit(_model(), _y(10)) for _ in range(3)]
    srv.step()
    assert [srv.jobs[i].row >= 0 for i in ids] == [True, True, False]


def test_continuous_batching_overlaps_on_two_streams():
    clock = FakeClock()
    ex = FakeExecutor(clock, nstreams=2, cost=lambda jobs: 1.0)
    srv = S.Server(ex, rows_per_class=100000, slots_per_class=64, max_batch=4, clock=clock)
    first = [srv.submit(_model(), _y(100)) for _ in range(3)]
    srv.step()                              # one batch of 3 on stream 0
    assert len(ex.launched) == 1 and ex.launched[0][0] == 0
    clock.t = 0.5
    late = [srv.submit(_model(), _y(100)) for _ in range(2)]
    srv.step()                              # arrived while the first runs: stream 1 at once
    assert len(ex.launched) == 2 and ex.launched[1][0] == 1
    assert ex.launched[1][2] == late
    clock.t = 1.0
    srv.step()
    assert all(srv.jobs[i].finished == 1.0 for i in first)
    assert all(srv.jobs[i].finished < 0 for i in late)
    clock.t = 1.5
    srv.step()
    assert all(srv.jobs[i].finished == 1.5 for i in late)
    p = srv.latency_percentiles()
    assert p["p50"] == 1.0 and p["p99"] > 0.99


def test_max_batch_and_classes():
    clock = FakeClock()
    ex = FakeExecutor(clock, nstreams=1)
    srv = S.Server(ex, rows_per_class=100000, slots_per_class=64, max_batch=3, clock=clock)
    for _ in range(4):
        srv.submit(_model(), _y(50))
    srv.submit(_model(8, 4), _y(50, 4), precision="mixed")
    srv.step()
    assert len(ex.launched[0][2]) == 3
    assert len(ex.classes) == 2
    srv.drain(poll=lambda: setattr(clock, "t", clock.t + 0.01))
    assert len(srv.done) == 5
    keys = {k for _, k, _ in ex.launched}
    assert keys == {(4, 2, "f32", "rts"), (8, 4, "mixed", "rts")}


def test_rejects_jobs_that_never_fit():
    clock = FakeClock()
    srv = S.Server(FakeExecutor(clock), rows_per_class=100, clock=clock)
    with pytest.raises(ValueError):
        srv.submit(_model(), _y(101))
    with pytest.raises(ValueError):
        srv.submit(_model(), _y(10), entry="kalman")
