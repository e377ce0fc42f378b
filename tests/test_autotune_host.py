"""Host logic of the schedule autotuner with a stand-in timer (no GPU): the
class key buckets T by powers of two, the fastest runnable candidate wins,
refused candidates are skipped, and plans are cached on disk."""
import json

import pytest

from paper_2511_10363_amd import autotune as A
from paper_2511_10363_amd import kfscan


def test_class_key_buckets_lengths():
    assert A.class_key("rts", 4, 2, "f32", 1 << 20) == A.class_key("rts", 4, 2, "f32", 1_100_000)
    assert A.class_key("rts", 4, 2, "f32", 1 << 20) != A.class_key("rts", 4, 2, "f32", 1 << 18)
    assert A.class_key("rts", 4, 2, "f32", 1000, batched=True) != \
        A.class_key("rts", 4, 2, "f32", 1000)


def test_candidates_by_class():
    assert A.candidates(16, False) == [("lookback", 0)]
    assert all(s.startswith("lookback") for s, _ in A.candidates(4, True))
    assert ("sengupta_b", 0) in A.candidates(4, False)


def test_picks_fastest_skips_refused_and_caches(tmp_path):
    calls = []

    def measure(entry, nx, ny, prec, T, batched, scan, items):
        calls.append((scan, items, T))
        if scan == "ladner_fischer":
            raise kfscan.KfScanError("unsupported")
        return {"lookback": 1.0 + 0.1 * items, "lookback_generic": 3.0}.get(scan, 2.0)

    path = str(tmp_path / "plans.json")
    t = A.Autotuner(cache_path=path, measure=measure)
    p = t.plan("rts", 4, 2, "f32", 1000)
    assert (p["scan"], p["items"]) == ("lookback", 0)
    assert p["T"] == 1024 and "ladner_fischer/0" not in p["times"]
    n = len(calls)
    t.plan("rts", 4, 2, "f32", 1100)          # same bucket: cached, nothing measured
    assert len(calls) == n
    saved = json.load(open(path))
    assert A.class_key("rts", 4, 2, "f32", 1000) in saved
    t2 = A.Autotuner(cache_path=path, measure=lambda *a: pytest.fail("measured again"))
    assert t2.plan("rts", 4, 2, "f32", 1000)["scan"] == "lookback"


def test_other_errors_propagate(tmp_path):
    def measure(*a):
        raise ZeroDivisionError
    t = A.Autotuner(cache_path=str(tmp_path / "p.json"), measure=measure)
    with pytest.raises(ZeroDivisionError):
        t.plan("filter", 2, 1, "f64", 64)
