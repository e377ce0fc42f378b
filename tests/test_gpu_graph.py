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
