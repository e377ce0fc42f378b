"""Numeric failures at the boundary: the optional per-sequence status array.

A ragged batch in which one sequence has a NaN measurement and another a
model whose R is not positive definite (so S_k of Sec. III-A has no Cholesky
factor): those two sequences get KF_SEQ_NONFINITE and NaN in every output
row, an invalid entry gets KF_SEQ_INVALID with its rows untouched, and every
other sequence still matches the CPU FP64 oracle."""
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import TOL, gpu_available, kfscan, normwise, oracle_inputs_for, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


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


LENGTHS = [700, 5000, 1, 2049, 333, 12000, 64]
NAN_SEQ, BAD_R_SEQ, INVALID_SEQ = 1, 3, 4


@pytest.mark.parametrize("scan", ["lookback", "lookback_generic", "sequential"])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_batch_status(entry, prec, scan):
    k = kfscan()
    _say("status batch", entry, prec, scan)
    rng = np.random.default_rng(99)
    n = len(LENGTHS)
    models = [W.random_stable_model(4, 2, 0.95, 0.1, 0.5, rng) for _ in range(n)]
    ys = [W.simulate(models[i], LENGTHS[i], rng) for i in range(n)]
    ys[NAN_SEQ] = ys[NAN_SEQ].copy()
    ys[NAN_SEQ][LENGTHS[NAN_SEQ] // 2, 1] = np.nan
    models[BAD_R_SEQ] = W.Model(*models[BAD_R_SEQ].arrays()[:3], -10.0 * np.eye(2),
                                *models[BAD_R_SEQ].arrays()[4:])
    offsets = np.cumsum([0] + LENGTHS[:-1]).astype(np.int64)
    total = int(sum(LENGTHS))
    dt = k.dtype_for(prec)
    parts = [np.stack([m.arrays()[j] for m in models]) for j in range(6)]
    dm = tuple(torch.as_tensor(np.ascontiguousarray(p)).to("cuda", dt).contiguous() for p in parts)
    y = np.concatenate(ys)
    yd = torch.as_tensor(y).to("cuda", dt).contiguous()
    lens = np.array(LENGTHS, dtype=np.int64)
    lens[INVALID_SEQ] = 0                      # an invalid entry: skipped
    T = torch.as_tensor(lens).cuda()
    off = torch.as_tensor(offsets).cuda()
    status = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    b, keep = k.make_batch(dm, yd, T, off, precision=prec, scan=scan,
                           smoother=(entry != "filter"), status=status)
    names = ["m_filt", "P_filt", "m_smooth", "P_smooth"][:2 if entry == "filter" else 4]
    sentinel = 12345.0
    for nm in names:
        keep[nm].fill_(sentinel)
    name = {"filter": "kf_filter_batch", "rts": "kf_smooth_rts_batch",
            "tf": "kf_smooth_twofilter_batch"}[entry]
    ws = k.run_batch(name, b, yd.device)
    torch.cuda.synchronize()
    bits = k.workspace_status(ws)
    assert bits & k.KF_WS_NUMERIC
    assert bits & k.KF_WS_INVALID
    st = status.cpu().numpy()
    want = np.zeros(n, dtype=np.int32)
    want[NAN_SEQ] = want[BAD_R_SEQ] = k.KF_SEQ_NONFINITE
    want[INVALID_SEQ] = k.KF_SEQ_INVALID
    assert st.tolist() == want.tolist()
    got = [keep[nm].double().cpu().numpy() for nm in names]
    for i in range(n):
        a, e = offsets[i], offsets[i] + LENGTHS[i]
        if i in (NAN_SEQ, BAD_R_SEQ):
            for g in got:
                assert np.all(np.isnan(g[a:e])), (i, "rows must be NaN")
        elif i == INVALID_SEQ:
            for g in got:
                assert np.all(g[a:e] == sentinel), (i, "rows must be untouched")
        else:
            ref = _reference(entry, models[i], ys[i], prec)
            for g, r in zip(got, ref):
                assert normwise(g[a:e], r) <= TOL[prec], (i, LENGTHS[i])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_plain_status(prec):
    """Equal-length sequences sharing a model: a NaN measurement in one of
    three sequences marks that one only."""
    k = kfscan()
    _say("status plain", prec)
    model, y0 = W.tracking(3000, seed=5)
    ys = np.stack([y0, y0[::-1].copy(), y0 * 0.5])
    ys[2, 1700, 0] = np.inf
    dt = k.dtype_for(prec)
    dm = k.model_to_device(model.arrays(), prec)
    yd = torch.as_tensor(ys).to("cuda", dt).contiguous()
    status = torch.zeros(3, dtype=torch.int32, device="cuda")
    out = k.smooth_rts(dm, yd, precision=prec, status=status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, 0, k.KF_SEQ_NONFINITE]
    got = [o.double().cpu().numpy() for o in out]
    for g in got:
        assert np.all(np.isnan(g[2]))
        assert np.all(np.isfinite(g[:2]))
    arrs, _ = oracle_inputs_for(model, y0, prec)
    for i in range(2):
        _, yy = oracle_inputs_for(model, ys[i], prec)
        ref = oracle.smooth_rts(*arrs, yy)
        for g, r in zip(got, ref):
            assert normwise(g[i], r) <= TOL[prec]


def test_status_clean_call_is_zero():
    """A call with nothing wrong writes 0 into every status word and leaves
    the workspace's numeric bit clear."""
    k = kfscan()
    model, y = W.tracking(5000, seed=2)
    dm = k.model_to_device(model.arrays(), "f32")
    yd = torch.as_tensor(y).to("cuda", torch.float32).contiguous()
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    k.smooth_twofilter(dm, yd, precision="f32", status=status)
    torch.cuda.synchronize()
    assert status.item() == 0
