"""GPU parity of the wide-state scans (nx = 8, ny = 4 and nx = 16, ny = 8):
elements spread over groups of nx lanes (kf_wide.hpp), for the filter (Lemma
1), the RTS smoother (Lemma 2) and the two-filter smoother, against the CPU
FP64 oracle, at lengths around the tile sizes (512 steps at nx = 8, 64 at
nx = 16) and inside ragged batches with a model per sequence."""
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import TOL, gpu_available, kfscan, normwise, oracle_inputs_for, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

SHAPES = [(8, 4), (16, 8)]
PRECS = ["f64", "f32", "mixed"]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _reference(entry, model, y, prec):
    arrs, yy = oracle_inputs_for(model, y, prec)
    if entry == "filter":
        return list(oracle.kf_filter(*arrs, yy)[:2])
    if entry == "rts":
        return list(oracle.smooth_rts(*arrs, yy))
    return list(oracle.smooth_twofilter(*arrs, yy))


def _model(nx, ny, seed):
    rng = np.random.default_rng(seed)
    rho, q, r = (0.95, 0.1, 0.5) if nx == 8 else (0.98, 0.05, 0.2)
    return W.random_stable_model(nx, ny, rho, q, r, rng), rng


def test_wide_shapes_supported():
    k = kfscan()
    for nx, ny in SHAPES:
        for prec in PRECS:
            assert k.supported(nx, ny, prec)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_wide_plain(nx, ny, entry, prec):
    k = kfscan()
    model, rng = _model(nx, ny, 10 * nx + ny)
    lengths = [1, 2, 7, 127, 128, 129, 511, 512, 513, 1000, 2600]
    dm = k.model_to_device(model.arrays(), prec)
    fn = {"filter": k.filter, "rts": k.smooth_rts, "tf": k.smooth_twofilter}[entry]
    for T in lengths:
        y = W.simulate(model, T, rng)
        _say("wide", entry, prec, "nx=%d ny=%d T=%d" % (nx, ny, T))
        yd = torch.as_tensor(y).to("cuda", k.dtype_for(prec)).contiguous()
        out = fn(dm, yd, precision=prec)
        torch.cuda.synchronize()
        got = [o.double().cpu().numpy() for o in out]
        ref = _reference(entry, model, y, prec)
        for g, r in zip(got, ref):
            assert g.shape == r.shape
            assert np.all(np.isfinite(g))
            assert normwise(g, r) <= TOL[prec], (T, normwise(g, r))
        for g in got[1::2]:
            assert np.array_equal(g, np.swapaxes(g, -1, -2))


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
@pytest.mark.parametrize("nx,ny", SHAPES)
def test_wide_batch(nx, ny, entry, prec):
    """Ragged batch, one model per sequence, shuffled packing with gaps."""
    k = kfscan()
    rng = np.random.default_rng(77 + nx)
    lengths = [1, 2, 127, 128, 129, 511, 512, 513, 1500, 4097]
    rho, q, r = (0.95, 0.1, 0.5) if nx == 8 else (0.98, 0.05, 0.2)
    models = [W.random_stable_model(nx, ny, rho, q, r, rng) for _ in lengths]
    ys = [W.simulate(m, T, rng) for m, T in zip(models, lengths)]
    order = rng.permutation(len(lengths))
    offsets = np.zeros(len(lengths), dtype=np.int64)
    row = 0
    for i in order:
        row += int(rng.integers(0, 4))
        offsets[i] = row
        row += lengths[i]
    total = row + 2
    dt = k.dtype_for(prec)
    parts = [np.stack([m.arrays()[j] for m in models]) for j in range(6)]
    dm = tuple(torch.as_tensor(np.ascontiguousarray(p)).to("cuda", dt).contiguous() for p in parts)
    y = np.zeros((total, ny))
    for i, yi in enumerate(ys):
        y[offsets[i]:offsets[i] + len(yi)] = yi
    yd = torch.as_tensor(y).to("cuda", dt).contiguous()
    T = torch.as_tensor(np.array(lengths, dtype=np.int64)).cuda()
    off = torch.as_tensor(offsets).cuda()
    _say("wide batch", entry, prec, "nx=%d ny=%d nseq=%d" % (nx, ny, len(lengths)))
    outs, ws = k.batch(entry, dm, yd, T, off, precision=prec)
    torch.cuda.synchronize()
    assert k.workspace_status(ws) == 0
    got = [o.double().cpu().numpy() for o in outs]
    for i in range(len(lengths)):
        ref = _reference(entry, models[i], ys[i], prec)
        a, b = offsets[i], offsets[i] + lengths[i]
        for g, rr in zip(got, ref):
            assert normwise(g[a:b], rr) <= TOL[prec], (i, lengths[i], normwise(g[a:b], rr))


@pytest.mark.parametrize("nx,ny,T,prec", [(8, 4, 1 << 16, "f32"), (16, 8, 20000, "mixed"),
                                          (16, 8, 9000, "f64"), (16, 8, 65536, "f32")])
def test_wide_long(nx, ny, T, prec):
    """Many tiles per sequence (RTS, which runs the filter first): 128 tiles of
    512 steps at nx = 8 (one look-back window of 32 groups x 4 tiles); 141 to
    1024 tiles of 64 steps at nx = 16, over windows of 4 groups x 16 tiles."""
    k = kfscan()
    model, rng = _model(nx, ny, 5)
    y = W.simulate(model, T, rng)
    _say("wide long", prec, "nx=%d T=%d" % (nx, T))
    dm = k.model_to_device(model.arrays(), prec)
    yd = torch.as_tensor(y).to("cuda", k.dtype_for(prec)).contiguous()
    out = k.smooth_rts(dm, yd, precision=prec)
    torch.cuda.synchronize()
    got = [o.double().cpu().numpy() for o in out]
    ref = _reference("rts", model, y, prec)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= TOL[prec], normwise(g, r)


def test_wide_refuses_other_scans():
    k = kfscan()
    model, rng = _model(8, 4, 1)
    dm = k.model_to_device(model.arrays(), "f32")
    yd = torch.as_tensor(W.simulate(model, 100, rng)).to("cuda", torch.float32).contiguous()
    for scan in ("blelloch", "sequential", "sengupta_b"):
        with pytest.raises(k.KfScanError):
            k.smooth_rts(dm, yd, precision="f32", scan=scan)
