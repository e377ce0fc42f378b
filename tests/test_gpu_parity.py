"""GPU parity: every C-ABI entry point against the CPU FP64 oracle, element by
element on the same seeded inputs (tolerances in tests/gpu_common.TOL)."""
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import (TOL, TOL_COMPONENT, TOL_Z, componentwise, gpu_available, kfscan,
                              normwise, oracle_inputs_for, to_dev, y_dev, zscore, torch)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

PRECS = ["f64", "f32", "mixed"]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(entry, model, y, prec, scan="auto"):
    k = kfscan()
    dev_model = to_dev(model, prec)
    yd = y_dev(y, prec)
    fn = {"filter": k.filter, "rts": k.smooth_rts, "tf": k.smooth_twofilter}[entry]
    out = fn(dev_model, yd, precision=prec, scan=scan)
    torch.cuda.synchronize()
    return [o.double().cpu().numpy() for o in out]


def _reference(entry, model, y, prec):
    arrs, yy = oracle_inputs_for(model, y, prec)
    if entry == "filter":
        m_f, P_f, _, _ = oracle.kf_filter(*arrs, yy)
        return [m_f, P_f]
    if entry == "rts":
        return list(oracle.smooth_rts(*arrs, yy))
    return list(oracle.smooth_twofilter(*arrs, yy))


def _check(entry, model, y, prec, tol=None, scan="auto"):
    tol = TOL[prec] if tol is None else tol
    _say(entry, prec, scan, "nx=%d ny=%d T=%d" % (model.nx, model.ny, y.shape[0]))
    got = _run(entry, model, y, prec, scan)
    ref = _reference(entry, model, y, prec)
    names = ["m_filt", "P_filt", "m_smooth", "P_smooth"]
    errs = {}
    for name, g, r in zip(names, got, ref):
        assert g.shape == r.shape, (name, g.shape, r.shape)
        assert np.all(np.isfinite(g)), name
        errs[name] = normwise(g, r)
    for name, e in errs.items():
        assert e <= tol, (entry, prec, name, errs)
    # FP64: every component and covariance entry on its own scale, and the
    # means to a small fraction of a posterior standard deviation
    if prec == "f64" and tol == TOL["f64"]:
        for name, g, r in zip(names, got, ref):
            c = componentwise(g, r)
            assert c <= TOL_COMPONENT["f64"], (entry, name, "componentwise", c)
        for i in range(0, len(got), 2):
            z = zscore(got[i], ref[i], ref[i + 1])
            assert z <= TOL_Z["f64"], (entry, names[i], "zscore", z)
    # covariances are exactly symmetric
    for g in got[1::2]:
        assert np.array_equal(g, np.swapaxes(g, -1, -2))
    return errs


SCAN_KINDS = ["lookback", "lookback_generic"]
TREE_KINDS = ["blelloch", "hillis_steele", "ladner_fischer", "sengupta_a",
              "sengupta_b"]             # one kernel per tree level (Algorithms 1-4)
ALL_KINDS = SCAN_KINDS + TREE_KINDS


@pytest.mark.parametrize("scan", ALL_KINDS)
@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_tracking_T1000(entry, prec, scan):
    """Constant-velocity tracking, T = 1000."""
    model, y = W.tracking(1000, seed=1)
    _check(entry, model, y, prec, scan=scan)


@pytest.mark.parametrize("scan", ALL_KINDS)
@pytest.mark.parametrize("T", [1, 2, 3, 7, 63, 64, 65, 511, 512, 513, 1000, 1023, 1024, 1025,
                               1500, 2047, 2048, 2049, 4095, 4096, 4097, 6000, 8193, 12289])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_ragged_lengths_f64(entry, T, scan):
    """Empty-tail tiles, single steps and tile boundaries.  A tile is 256 * L
    steps: the time-invariant filter takes L = 2 (512-step tiles) at all these
    lengths; the full-element scans take the longest L that still gives 4
    tiles: L = 2 up to 2048 steps, 4 up to 8192, then 8 (2048-step tiles)."""
    model, y = W.tracking(T, seed=T)
    _check(entry, model, y, "f64", scan=scan)


@pytest.mark.parametrize("scan", ALL_KINDS)
@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 4)])
@pytest.mark.parametrize("prec", ["f64", "mixed"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_shapes_stable_models(entry, prec, nx, ny, scan):
    rng = np.random.default_rng(100 * nx + ny)
    model = W.random_stable_model(nx, ny, 0.95, 0.1, 0.5, rng)
    y = W.simulate(model, 9000, rng)
    _check(entry, model, y, prec, scan=scan)


@pytest.mark.parametrize("scan", ALL_KINDS)
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_batch_of_sequences(entry, scan):
    """nseq sequences sharing the model in one launch equal separate runs."""
    _say("batch", entry, scan)
    model = W.cv_model()
    rng = np.random.default_rng(4)
    ys = np.stack([W.simulate(model, 3000, rng) for _ in range(3)])
    k = kfscan()
    out = {"filter": k.filter, "rts": k.smooth_rts, "tf": k.smooth_twofilter}[entry](
        to_dev(model, "f64"), y_dev(ys, "f64"), precision="f64", scan=scan)
    torch.cuda.synchronize()
    for s in range(3):
        ref = _reference(entry, model, ys[s], "f64")
        for g, r in zip(out, ref):
            assert normwise(g[s].double().cpu().numpy(), r) <= TOL["f64"]


def test_workspace_reuse_is_deterministic():
    """The workspace is left clean: repeated calls give bit-identical output."""
    model, y = W.tracking(20000, seed=2)
    a = _run("rts", model, y, "f32")
    b = _run("rts", model, y, "f32")
    c = _run("tf", model, y, "f32")
    d = _run("rts", model, y, "f32")
    for x, z in zip(a, d):
        assert np.array_equal(x, z)
    del b, c


@pytest.mark.parametrize("scan", SCAN_KINDS)
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
def test_full_size_T_2_20(prec, scan):
    """The benchmark workload: tracking model, T = 2^20, filter + RTS smoother,
    every output compared with the oracle."""
    T = 1 << 20
    model, y = W.tracking(T, seed=20251110)
    errs = _check("rts", model, y, prec, scan=scan)
    _say("errors", errs)


@pytest.mark.parametrize("scan", TREE_KINDS)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_size_tree_scans_T_2_20(prec, scan):
    """The benchmark workload through the one-kernel-per-level scans."""
    T = 1 << 20
    model, y = W.tracking(T, seed=20251110)
    errs = _check("rts", model, y, prec, scan=scan)
    _say("errors", errs)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("entry", ["rts", "tf"])
def test_intermediate_tile_sizes(entry, prec):
    """T = 2^19 + 12345 selects L = 8 for the time-invariant filter (2^20 selects
    16, 2^18 selects 4, short sequences 2), so with the ragged-length and
    full-size tests every compiled L of the nx = 4 kernels is compared with the
    oracle."""
    T = (1 << 19) + 12345
    model, y = W.tracking(T, seed=19)
    _check(entry, model, y, prec)


@pytest.mark.parametrize("scan", TREE_KINDS)
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_tree_scans_past_the_sengupta_threshold(entry, scan):
    """T = 100000 pads to 2^17: Sengupta B reduces three levels down to its
    16384-position top level before Hillis-Steele, and every other tree scan
    runs many levels over a ragged tail of identity padding."""
    model, y = W.tracking(100000, seed=17)
    _check(entry, model, y, "f64", scan=scan)


def test_full_size_twofilter_T_2_18():
    model, y = W.tracking(1 << 18, seed=18)
    _check("tf", model, y, "mixed")


def test_unsupported_and_bad_arguments():
    k = kfscan()
    model = W.random_stable_model(5, 2, 0.9, 0.1, 0.5, np.random.default_rng(0))
    y = np.zeros((10, 2))
    with pytest.raises(k.KfScanError):
        k.filter(to_dev(model, "f32"), y_dev(y, "f32"), precision="f32")
    m4, y4 = W.tracking(10)
    with pytest.raises(ValueError):
        k.filter(to_dev(m4, "f32"), y_dev(y4, "f64"), precision="f32")
    with pytest.raises(k.KfScanError):
        k.filter(to_dev(m4, "f32"), torch.zeros((10, 2)), precision="f32")


def test_one_workspace_across_precisions_and_shapes():
    """One workspace serves calls of different precisions and shapes in turn
    (each call re-initialises the control words its layout uses)."""
    k = kfscan()
    ws = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    model, y = W.tracking(1000, seed=3)
    rng = np.random.default_rng(8)
    m2 = W.random_stable_model(2, 1, 0.9, 0.1, 0.5, rng)
    y2 = W.simulate(m2, 7000, rng)
    for prec, mdl, yy, fn in [("f32", model, y, k.filter), ("f64", model, y, k.smooth_rts),
                              ("mixed", m2, y2, k.smooth_twofilter), ("f64", model, y, k.smooth_rts),
                              ("f32", m2, y2, k.smooth_rts)]:
        _say("shared workspace", prec, mdl.nx, yy.shape[0])
        out = fn(to_dev(mdl, prec), y_dev(yy, prec), precision=prec, workspace=ws)
        torch.cuda.synchronize()
        ref = _reference("filter" if fn is k.filter else ("tf" if fn is k.smooth_twofilter else "rts"),
                         mdl, yy, prec)
        for g, r in zip(out, ref):
            assert normwise(g.double().cpu().numpy(), r) <= TOL[prec]


@pytest.mark.parametrize("scan", ["lookback", "lookback_generic", "sequential", "ladner_fischer",
                                  "sengupta_b"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_many_short_equal_sequences(entry, scan):
    """3000 sequences of 37 steps share the model in one kf_problem: one tile
    per sequence for the look-back scans (the ticket -> sequence map), 47
    blocks of 64 lanes for the sequential recursions, 3000 grid rows for the
    tree scans.  Sampled sequences, including the first and the last, are
    compared with the oracle."""
    _say("many sequences", entry, scan)
    rng = np.random.default_rng(37)
    model = W.random_stable_model(4, 2, 0.95, 0.1, 0.5, rng)
    nseq, T = 3000, 37
    ys = np.stack([W.simulate(model, T, rng) for _ in range(nseq)])
    k = kfscan()
    out = {"filter": k.filter, "rts": k.smooth_rts, "tf": k.smooth_twofilter}[entry](
        to_dev(model, "f64"), y_dev(ys, "f64"), precision="f64", scan=scan)
    torch.cuda.synchronize()
    out = [o.double().cpu().numpy() for o in out]
    for s in (0, 1, 63, 64, 1500, 2998, 2999):
        ref = _reference(entry, model, ys[s], "f64")
        for g, r in zip(out, ref):
            assert normwise(g[s], r) <= TOL["f64"], (entry, scan, s)
