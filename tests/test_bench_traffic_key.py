"""Host checks of the key under which bench.py keeps rocprofv3 traffic: stored
counter bytes are reported only for the kernel sources and compile flags they
were measured on."""
import json
import os

import bench
from paper_2511_10363_amd import build as kbuild


def test_hash_follows_compile_flags(monkeypatch):
    h0 = bench.kernel_source_hash()
    monkeypatch.setattr(kbuild, "CXXFLAGS", kbuild.CXXFLAGS + ["-DKF_EXTRA_FLAG"])
    assert bench.kernel_source_hash() != h0


def test_hash_ignores_where_the_repository_sits(monkeypatch):
    h0 = bench.kernel_source_hash()
    inc = os.path.join(kbuild.ROOT, "include")
    moved = "/elsewhere/repo"
    flags = [os.path.join(moved, "include") if f == inc else f for f in kbuild.CXXFLAGS]
    monkeypatch.setattr(kbuild, "ROOT", moved)
    monkeypatch.setattr(kbuild, "CXXFLAGS", flags)
    assert bench.kernel_source_hash() == h0


def test_stale_traffic_is_not_reported(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    key = "k_rts|tracking_T2^20_lookback|f32"
    h = bench.kernel_source_hash()
    rec = {"bytes_per_launch": 1.0e8, "source_hash": h}
    (prof / "traffic.json").write_text(json.dumps({key: rec}))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.load_traffic("k_rts", "tracking_T2^20_lookback", "f32") == 1.0e8
    rec["source_hash"] = "0" * 16
    (prof / "traffic.json").write_text(json.dumps({key: rec}))
    assert bench.load_traffic("k_rts", "tracking_T2^20_lookback", "f32") is None
