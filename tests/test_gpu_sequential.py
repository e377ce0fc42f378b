"""GPU parity of KF_SCAN_SEQUENTIAL, the sequential recursions of Sec. III run
by one GPU lane per sequence (the baseline of the speedup experiment of
Sec. VI), against the CPU FP64 oracle: plain, time-varying and ragged-batch
entry points, every precision, the stage entry points, and agreement with the
parallel scans on the same inputs."""
import numpy as np
import pytest

import kf_workloads as W
from tests.gpu_common import TOL, gpu_available, kfscan, normwise, to_dev, y_dev, torch
from tests.test_gpu_batch import _check_batch
from tests.test_gpu_parity import _check, _reference, _say
from tests.test_gpu_tv import _check_tv

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

SEQ = "sequential"


@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_tracking_T1000(entry, prec):
    model, y = W.tracking(1000, seed=1)
    _check(entry, model, y, prec, scan=SEQ)


@pytest.mark.parametrize("T", [1, 2, 3, 64, 1025])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_lengths_f64(entry, T):
    model, y = W.tracking(T, seed=T)
    _check(entry, model, y, "f64", scan=SEQ)


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (2, 2), (3, 1), (3, 2), (4, 1), (4, 4)])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_shapes_stable_models(entry, nx, ny):
    rng = np.random.default_rng(100 * nx + ny)
    model = W.random_stable_model(nx, ny, 0.95, 0.1, 0.5, rng)
    y = W.simulate(model, 3000, rng)
    _check(entry, model, y, "f64", scan=SEQ)


@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_sequences_share_the_model(entry):
    """nseq = 70 sequences: two 64-lane blocks, the second partly idle."""
    _say("sequential nseq=70", entry)
    model = W.cv_model()
    rng = np.random.default_rng(4)
    ys = np.stack([W.simulate(model, 300, rng) for _ in range(70)])
    k = kfscan()
    out = {"filter": k.filter, "rts": k.smooth_rts, "tf": k.smooth_twofilter}[entry](
        to_dev(model, "f64"), y_dev(ys, "f64"), precision="f64", scan=SEQ)
    torch.cuda.synchronize()
    out = [o.double().cpu().numpy() for o in out]
    for s in (0, 1, 63, 64, 69):
        ref = _reference(entry, model, ys[s], "f64")
        for g, r in zip(out, ref):
            assert normwise(g[s], r) <= TOL["f64"], s


@pytest.mark.parametrize("entry,prec", [("filter", "f64"), ("filter", "f32"), ("filter", "mixed"),
                                        ("rts", "f64"), ("rts", "f32"), ("rts", "mixed"),
                                        ("tf", "f64"), ("tf", "mixed")])
def test_paper_time_varying_model(entry, prec):
    _check_tv(entry, 3000, prec, True, seed=3, scan=SEQ)


def test_time_varying_twofilter_f32_needs_conditioned_noise():
    """The sequential backward information filter inverts R_k and I + J Q_k
    alone.  On the paper's model some R_k and Q_k have condition numbers of
    1e7..1e9, beyond FP32, so the FP32 recursion is only compared on the same
    model with Q_k + I, R_k + I (condition numbers below about 30); the
    parallel form factorises H Q H^T + R instead and needs no such change
    (FP32 solves in KF_PREC_F32, FP64 in KF_PREC_F32_F64SOLVE pass on the
    unmodified model)."""
    _check_tv("tf", 3000, "f32", True, seed=3, scan=SEQ, ridge=1.0)


@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_time_varying_no_inputs_and_sequences(entry):
    _check_tv(entry, 700, "f64", False, seed=8, nseq=3, scan=SEQ)


@pytest.mark.parametrize("nx,ny", [(1, 1), (3, 2), (4, 4)])
def test_time_varying_shapes(nx, ny):
    _check_tv("tf", 900, "f64", True, seed=nx * 7 + ny, nx=nx, ny=ny, scan=SEQ)


@pytest.mark.parametrize("per_model", [False, True])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_ragged_batch(entry, prec, per_model):
    _check_batch(entry, [1, 2, 7, 63, 511, 1000, 2049, 5000], 4, 2, per_model, prec, SEQ, seed=7)


def test_ragged_batch_skips_invalid_entries():
    """Entries with no steps or rows outside the buffer are skipped one by one
    and reported in status bit 1; the valid ones are still right."""
    from tests.test_gpu_batch import _case, _device_batch
    k = kfscan()
    lengths = [700, 900, 1200, 300]
    models, ys, offsets, total = _case(lengths, 4, 2, False, seed=5)
    dm, yd, T, off = _device_batch(models, ys, offsets, total, False, "f64")
    bad_T = T.clone()
    bad_T[1] = 0
    bad_off = off.clone()
    bad_off[2] = total - 10
    b, keep = k.make_batch(dm, yd, bad_T, bad_off, precision="f64", scan=SEQ, smoother=True)
    for name in ("m_filt", "P_filt", "m_smooth", "P_smooth"):
        keep[name].fill_(12345.0)
    ws = k.run_batch("kf_smooth_rts_batch", b, yd.device)
    torch.cuda.synchronize()
    assert k.workspace_status(ws) & 2
    got = [keep[n].double().cpu().numpy() for n in ("m_filt", "P_filt", "m_smooth", "P_smooth")]
    for i in (0, 3):
        ref = _reference("rts", models[i], ys[i], "f64")
        a, e = offsets[i], offsets[i] + lengths[i]
        for g, r in zip(got, ref):
            assert normwise(g[a:e], r) <= TOL["f64"]
    for i in (1, 2):
        a, e = offsets[i], offsets[i] + lengths[i]
        for g in got:
            assert np.all(g[a:e] == 12345.0)


def test_stage_entry_points():
    """kf_prepare + kf_pass_filter + kf_pass_rts / kf_pass_twofilter with the
    sequential recursions give the one-call results bit for bit."""
    k = kfscan()
    model, y = W.tracking(4000, seed=6)
    plan = k.Plan(to_dev(model, "f32"), y_dev(y, "f32"), precision="f32", scan=SEQ)
    for entry, one in (("kf_pass_rts", "rts"), ("kf_pass_twofilter", "tf")):
        plan("kf_prepare")
        plan("kf_pass_filter")
        plan(entry)
        torch.cuda.synchronize()
        staged = [o.clone() for o in plan.outputs()]
        fn = k.smooth_rts if one == "rts" else k.smooth_twofilter
        full = fn(to_dev(model, "f32"), y_dev(y, "f32"), precision="f32", scan=SEQ)
        torch.cuda.synchronize()
        for a, b in zip(staged, full):
            assert torch.equal(a.reshape(b.shape), b), entry


@pytest.mark.parametrize("entry", ["rts", "tf"])
def test_sequential_agrees_with_the_parallel_scan(entry):
    """On the same FP64 inputs the sequential recursion and the look-back scan
    are two orderings of the same exact computation."""
    model, y = W.tracking(50000, seed=12)
    k = kfscan()
    fn = k.smooth_rts if entry == "rts" else k.smooth_twofilter
    a = fn(to_dev(model, "f64"), y_dev(y, "f64"), precision="f64", scan=SEQ)
    b = fn(to_dev(model, "f64"), y_dev(y, "f64"), precision="f64", scan="lookback")
    torch.cuda.synchronize()
    for x, z in zip(a, b):
        assert normwise(x.cpu().numpy(), z.cpu().numpy()) <= TOL["f64"]
