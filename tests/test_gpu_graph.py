"""HIP-graph capture of whole passes.

The entry points enqueue kernels only (the control words are cleared by a
kernel, never by a memset), so a pass can be captured once and replayed.  Each
test captures the stage entry points of one pass into a graph, replays it
several times with the program's own eager work and synchronisations in
between, and checks every replay against the eager result bit for bit (the
same kernels on the same inputs)."""
import sys

import numpy as np
import pytest

import kf_workloads as W
from tests.gpu_common import gpu_available, kfscan, to_dev, y_dev, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("scan", ["lookback", "lookback_generic", "ladner_fischer", "sequential"])
@pytest.mark.parametrize("backward", ["kf_pass_rts", "kf_pass_twofilter"])
def test_captured_pass_replays_match_eager(backward, scan):
    _say("graph", backward, scan)
    k = kfscan()
    model, y = W.tracking(300000, seed=31)
    other_model, other_y = W.tracking(5000, seed=32)
    plan = k.Plan(to_dev(model, "f32"), y_dev(y, "f32"), precision="f32", scan=scan)
    # eager reference
    for entry in ("kf_prepare", "kf_pass_filter", backward):
        plan(entry)
    torch.cuda.synchronize()
    ref = [o.clone() for o in plan.outputs()]
    for o in plan.outputs():
        o.fill_(float("nan"))
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for entry in ("kf_prepare", "kf_pass_filter", backward):
                plan(entry)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in plan.outputs():
            o.fill_(float("nan"))
        # eager work of the program between replays
        k.smooth_rts(to_dev(other_model, "f32"), y_dev(other_y, "f32"), precision="f32")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(plan.outputs(), ref):
            assert torch.equal(a, b), (backward, scan, rep)


def test_captured_ragged_batch_replays_match_eager():
    """kf_smooth_rts_batch (prepare of one model per sequence, the device-side
    tile map, both scans) captured once and replayed."""
    import ctypes

    from tests.test_gpu_batch import _case, _device_batch
    _say("graph batch")
    k = kfscan()
    lib = k.load_library()
    lengths = [5000, 300, 70000, 1, 2500, 9000, 777]
    models, ys, offsets, total = _case(lengths, 4, 2, True, seed=41)
    dm, yd, T, off = _device_batch(models, ys, offsets, total, True, "f32")
    b, keep = k.make_batch(dm, yd, T, off, precision="f32", smoother=True)
    ws = torch.empty(k.batch_workspace_size(b), dtype=torch.uint8, device="cuda")
    outs = [keep[n] for n in ("m_filt", "P_filt", "m_smooth", "P_smooth")]

    def call():
        stream = torch.cuda.current_stream().cuda_stream
        rc = lib.kf_smooth_rts_batch(ctypes.byref(b), ws.data_ptr(), ws.numel(), stream)
        assert rc == 0

    call()
    torch.cuda.synchronize()
    assert k.workspace_status(ws) == 0
    ref = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    for rep in range(3):
        for o in outs:
            o.fill_(float("nan"))
        k.batch("filter", dm, yd, T, off, precision="f32")   # eager work in between
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert k.workspace_status(ws) == 0
        for a, r in zip(outs, ref):
            # rows outside every sequence are not written by either run
            a_n, r_n = a.cpu().numpy(), r.cpu().numpy()
            for i, L in enumerate(lengths):
                sl = slice(offsets[i], offsets[i] + L)
                assert np.array_equal(a_n[sl], r_n[sl]), (rep, i)
