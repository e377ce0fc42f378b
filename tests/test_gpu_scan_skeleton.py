"""Bit-exact GPU test of the look-back scan skeleton (kf_selftest_scan): the
tile driver shared by the filter, RTS and two-filter passes, run with exact
affine maps mod p, forward (all-prefix-sums) and reversed (reversed
all-prefix-sums, Sec. II-B), against exact host scans."""
import sys

import numpy as np
import pytest

from tests import affine_scan as S
from tests.gpu_common import gpu_available, kfscan, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(e, prec, reverse, items, group=1):
    k = kfscan()
    dt = torch.float64 if prec == "f64" else torch.float32
    ed = torch.as_tensor(e).to("cuda", dt).contiguous()
    out = k.selftest_scan(ed, reverse=reverse, items=items, group=group)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("items", [2, 8, 16])
@pytest.mark.parametrize("T", [1, 2, 255, 511, 512, 513, 4097, 70001])
def test_scan_skeleton_exact(prec, reverse, items, T):
    p = kfscan().AFFINE_MODULUS[prec]
    rng = np.random.default_rng(T * 31 + items)
    nseq = 3
    e = S.random_elements(rng, nseq, T, p, reverse=reverse)
    _say("skeleton", prec, "reverse" if reverse else "forward", "L=%d T=%d nseq=%d" % (items, T, nseq))
    got = _run(e, prec, reverse, items)
    want = S.doubling(e, p, reverse=reverse)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("reverse", [False, True])
def test_scan_skeleton_anchors(prec, reverse):
    """Elements with A = 0 scattered at random: wavefront totals, thread
    aggregates and tile aggregates that are anchors take the early-publication
    and restart paths."""
    p = kfscan().AFFINE_MODULUS[prec]
    rng = np.random.default_rng(5)
    for rate in (0.001, 0.02, 0.3):
        e = S.random_elements(rng, 2, 300001, p, anchor_rate=rate, reverse=reverse)
        _say("skeleton anchors", prec, reverse, rate)
        got = _run(e, prec, reverse, 4)
        assert np.array_equal(got, S.doubling(e, p, reverse=reverse))


@pytest.mark.parametrize("reverse", [False, True])
def test_scan_skeleton_many_tiles(reverse):
    """2^21 + 12345 steps in 512-step tiles (4121 tiles): look-back windows of
    1024 tiles, several of them for a tile that finds no published prefix."""
    p = kfscan().AFFINE_MODULUS["f64"]
    rng = np.random.default_rng(21)
    T = (1 << 21) + 12345
    e = S.random_elements(rng, 1, T, p, reverse=reverse)
    _say("skeleton many tiles", reverse, T)
    got = _run(e, "f64", reverse, 2)
    assert np.array_equal(got, S.doubling(e, p, reverse=reverse))


# ---------------------------------------------------------------------------
# The group driver of the wide-state scans (groups of 8 lanes in 256-thread
# workgroups, 16 lanes in one-wavefront ones): tiles of 32 x items and
# 4 x items steps, look-back windows of 32 x 16 and 4 x 16 tiles.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("group,items", [(8, 2), (8, 16), (16, 2), (16, 16)])
@pytest.mark.parametrize("T", [1, 2, 127, 128, 129, 513, 4097, 30001])
def test_group_skeleton_exact(prec, reverse, group, items, T):
    p = kfscan().AFFINE_MODULUS[prec]
    rng = np.random.default_rng(T * 7 + items + group)
    e = S.random_elements(rng, 2, T, p, reverse=reverse)
    _say("group skeleton", prec, "reverse" if reverse else "forward",
         "G=%d L=%d T=%d" % (group, items, T))
    got = _run(e, prec, reverse, items, group)
    assert np.array_equal(got, S.doubling(e, p, reverse=reverse))


@pytest.mark.parametrize("reverse", [False, True])
@pytest.mark.parametrize("group", [8, 16])
def test_group_skeleton_many_windows(reverse, group):
    """100003 steps in tiles of 8 (G = 16) or 64 (G = 8) steps: 12501 or 1563
    tiles, against windows of 64 or 512 tiles, so a tile that finds no
    published prefix nearby folds several windows."""
    p = kfscan().AFFINE_MODULUS["f64"]
    rng = np.random.default_rng(group)
    T = 100003
    e = S.random_elements(rng, 1, T, p, reverse=reverse)
    _say("group skeleton many windows", group, reverse, T)
    got = _run(e, "f64", reverse, 2, group)
    assert np.array_equal(got, S.doubling(e, p, reverse=reverse))


@pytest.mark.parametrize("group", [8, 16])
def test_group_skeleton_anchors(group):
    p = kfscan().AFFINE_MODULUS["f32"]
    rng = np.random.default_rng(55)
    for rate in (0.002, 0.05):
        e = S.random_elements(rng, 3, 50001, p, anchor_rate=rate)
        _say("group skeleton anchors", group, rate)
        got = _run(e, "f32", False, 4, group)
        assert np.array_equal(got, S.doubling(e, p))
