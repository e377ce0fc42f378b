"""GPU parity of the ragged-batch entry points (kf_filter_batch,
kf_smooth_rts_batch, kf_smooth_twofilter_batch) against the CPU FP64 oracle run
on every sequence separately.  Sequences are packed in a shuffled order with
unused rows between them; models are shared or one per sequence."""
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import TOL, gpu_available, kfscan, normwise, oracle_inputs_for, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

LENGTHS = [1, 2, 7, 63, 511, 512, 513, 1000, 2048, 2049, 5000, 20000]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _case(lengths, nx, ny, per_model, seed):
    """Models, sequences, a shuffled packing with gaps: (models, ys, offsets, total)."""
    rng = np.random.default_rng(seed)
    n = len(lengths)
    if per_model:
        models = [W.random_stable_model(nx, ny, 0.95, 0.1, 0.5, rng) for _ in range(n)]
    else:
        models = [W.random_stable_model(nx, ny, 0.95, 0.1, 0.5, rng)] * n
    ys = [W.simulate(models[i], lengths[i], rng) for i in range(n)]
    order = rng.permutation(n)
    offsets = np.zeros(n, dtype=np.int64)
    row = 0
    for i in order:
        row += int(rng.integers(0, 5))          # unused rows between sequences
        offsets[i] = row
        row += lengths[i]
    return models, ys, offsets, row + 3


def _device_batch(models, ys, offsets, total, per_model, prec):
    k = kfscan()
    dt = k.dtype_for(prec)
    if per_model:
        parts = [np.stack([m.arrays()[j] for m in models]) for j in range(6)]
    else:
        parts = list(models[0].arrays())
    dm = tuple(torch.as_tensor(np.ascontiguousarray(p)).to("cuda", dt).contiguous() for p in parts)
    ny = ys[0].shape[1]
    y = np.zeros((total, ny))
    for i, yi in enumerate(ys):
        y[offsets[i]:offsets[i] + len(yi)] = yi
    yd = torch.as_tensor(y).to("cuda", dt).contiguous()
    T = torch.as_tensor(np.array([len(v) for v in ys], dtype=np.int64)).cuda()
    off = torch.as_tensor(offsets).cuda()
    return dm, yd, T, off


def _reference(entry, model, y, prec):
    arrs, yy = oracle_inputs_for(model, y, prec)
    if entry == "filter":
        return list(oracle.kf_filter(*arrs, yy)[:2])
    if entry == "rts":
        return list(oracle.smooth_rts(*arrs, yy))
    return list(oracle.smooth_twofilter(*arrs, yy))


def _check_batch(entry, lengths, nx, ny, per_model, prec, scan, seed):
    _say("batch", entry, prec, scan, "per_model" if per_model else "shared",
         "nx=%d ny=%d nseq=%d" % (nx, ny, len(lengths)))
    k = kfscan()
    models, ys, offsets, total = _case(lengths, nx, ny, per_model, seed)
    dm, yd, T, off = _device_batch(models, ys, offsets, total, per_model, prec)
    outs, ws = k.batch(entry, dm, yd, T, off, precision=prec, scan=scan)
    torch.cuda.synchronize()
    assert k.workspace_status(ws) == 0
    got = [o.double().cpu().numpy() for o in outs]
    for i in range(len(lengths)):
        ref = _reference(entry, models[i], ys[i], prec)
        a, b = offsets[i], offsets[i] + lengths[i]
        for g, r in zip(got, ref):
            assert g[a:b].shape == r.shape
            assert normwise(g[a:b], r) <= TOL[prec], (i, lengths[i])
        for g in got[1::2]:
            assert np.array_equal(g[a:b], np.swapaxes(g[a:b], -1, -2))


@pytest.mark.parametrize("scan", ["lookback", "lookback_generic"])
@pytest.mark.parametrize("per_model", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_ragged_batch(entry, prec, per_model, scan):
    _check_batch(entry, LENGTHS, 4, 2, per_model, prec, scan, seed=7)


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (3, 2), (4, 4)])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_ragged_batch_shapes(entry, nx, ny):
    _check_batch(entry, [3, 700, 1500, 4097], nx, ny, True, "f64", "auto", seed=nx * 10 + ny)


@pytest.mark.parametrize("entry", ["rts", "tf"])
def test_many_short_sequences(entry):
    """600 sequences of lengths 2^U, U ~ U[6, 12], one model each (the shape of
    the batched workload): the tile map spans several thousand tickets."""
    rng = np.random.default_rng(3)
    lengths = [int(round(2 ** u)) for u in rng.uniform(6, 12, size=600)]
    _check_batch(entry, lengths, 4, 2, True, "f32", "auto", seed=11)


def test_invalid_entries_are_skipped_and_reported():
    """A zero length, a negative offset and rows past the end are refused on the
    device: status bit 1 is raised, those rows are left untouched, and the
    valid sequences are still right."""
    k = kfscan()
    lengths = [700, 900, 1200, 300]
    models, ys, offsets, total = _case(lengths, 4, 2, False, seed=5)
    dm, yd, T, off = _device_batch(models, ys, offsets, total, False, "f64")
    bad_T = T.clone()
    bad_off = off.clone()
    bad_T[1] = 0                      # no steps
    bad_off[2] = -5                   # before the first row
    bad_off[3] = total - 10           # runs past the last row
    b, keep = k.make_batch(dm, yd, bad_T, bad_off, precision="f64", smoother=True)
    for name in ("m_filt", "P_filt", "m_smooth", "P_smooth"):
        keep[name].fill_(12345.0)
    ws = k.run_batch("kf_smooth_rts_batch", b, yd.device)
    torch.cuda.synchronize()
    assert k.workspace_status(ws) & 2
    got = [keep[n].double().cpu().numpy() for n in ("m_filt", "P_filt", "m_smooth", "P_smooth")]
    ref = _reference("rts", models[0], ys[0], "f64")
    a, b_ = offsets[0], offsets[0] + lengths[0]
    for g, r in zip(got, ref):
        assert normwise(g[a:b_], r) <= TOL["f64"]
    for i in (1, 2):                  # skipped sequences keep the sentinel
        a, b_ = offsets[i], offsets[i] + lengths[i]
        for g in got:
            assert np.all(g[a:b_] == 12345.0)
    # the same workspace then serves a valid call and reports no error
    outs, ws = k.batch("rts", dm, yd, T, off, precision="f64", workspace=ws)
    torch.cuda.synchronize()
    assert k.workspace_status(ws) == 0


@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_results_do_not_depend_on_the_rest_of_the_batch(entry):
    """A sequence's outputs are bit-identical whether it is processed alone or
    packed with others (different lengths, models and positions): batches
    always take the longest tiles, and each sequence's look-back depends only
    on its own tiles."""
    k = kfscan()
    lengths = [5000, 300, 70000, 1, 2500, 9000]
    models, ys, offsets, total = _case(lengths, 4, 2, True, seed=21)
    dm, yd, T, off = _device_batch(models, ys, offsets, total, True, "f32")
    mixed, _ = k.batch(entry, dm, yd, T, off, precision="f32")
    for i in (0, 2, 3):
        one_m = tuple(t[i:i + 1].contiguous() for t in dm)
        y1 = yd[offsets[i]:offsets[i] + lengths[i]].contiguous()
        alone, _ = k.batch(entry, one_m, y1, T[i:i + 1].contiguous(),
                           torch.zeros(1, dtype=torch.int64, device="cuda"), precision="f32")
        torch.cuda.synchronize()
        for a, b in zip(alone, mixed):
            assert torch.equal(a, b[offsets[i]:offsets[i] + lengths[i]]), (entry, i)


def test_one_sequence_batch_equals_plain_call():
    """A batch of one sequence gives bit-identical results to kf_smooth_rts at a
    length where both take the longest tiles."""
    k = kfscan()
    model, y = W.tracking(1 << 20, seed=9)
    dm = k.model_to_device(model.arrays(), "f32")
    yd = torch.as_tensor(y).to("cuda", torch.float32).contiguous()
    plain = k.smooth_rts(dm, yd, precision="f32")
    T = torch.tensor([len(y)], dtype=torch.int64, device="cuda")
    off = torch.zeros(1, dtype=torch.int64, device="cuda")
    outs, _ = k.batch("rts", dm, yd, T, off, precision="f32")
    torch.cuda.synchronize()
    for a, b in zip(plain, outs):
        assert torch.equal(a, b)
