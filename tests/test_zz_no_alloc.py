"""kf_smooth_rts_noalloc (the entry point that allocates nothing: its
workspace is a static device array of KF_NOALLOC_SCRATCH_BYTES) against
kf_smooth_rts with a caller workspace: two calls in a row, the second on a
smaller input, must agree bit for bit; a problem whose workspace exceeds the
array is refused with KF_ERR_WORKSPACE before anything is launched."""
import ctypes
import sys

import numpy as np
import pytest

import kf_workloads as W
from tests.gpu_common import gpu_available, kfscan, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

SCRATCH_BYTES = 16 << 20


def _noalloc(k, p, stream):
    lib = k.load_library()
    fn = lib.kf_smooth_rts_noalloc
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.POINTER(k.KfProblem), ctypes.c_void_p]
    return fn(ctypes.byref(p), stream)


def _case(k, T, prec, seed, nseq=1):
    print("[case] noalloc", prec, "T=%d nseq=%d" % (T, nseq), flush=True)
    sys.stdout.flush()
    model, _ = W.tracking(8, seed=seed)
    rng = np.random.default_rng(seed)
    ys = np.stack([W.simulate(model, T, rng) for _ in range(nseq)])
    dt = k.dtype_for(prec)
    dm = k.model_to_device(model.arrays(), prec)
    yd = torch.as_tensor(ys).to("cuda", dt).contiguous()
    want = k.smooth_rts(dm, yd, precision=prec)
    nx = model.nx
    m_s = torch.empty((nseq, T, nx), dtype=dt, device="cuda")
    P_s = torch.empty((nseq, T, nx, nx), dtype=dt, device="cuda")
    p, keep = k.make_problem(dm, yd, prec, "auto", m_smooth=m_s, P_smooth=P_s)
    assert k.workspace_size(p) <= SCRATCH_BYTES
    stream = torch.cuda.current_stream().cuda_stream
    assert _noalloc(k, p, stream) == k.KF_OK
    torch.cuda.synchronize()
    got = (keep["m_filt"], keep["P_filt"], m_s, P_s)
    for g, w in zip(got, want):
        assert torch.equal(g, w)


@pytest.mark.parametrize("prec", ["f32", "f64", "mixed"])
def test_noalloc_matches_workspace_entry_point(prec):
    k = kfscan()
    _case(k, 1 << 20, prec, seed=3)       # first call: the full tracking length
    _case(k, 3001, prec, seed=4, nseq=2)  # second call, smaller: the array keeps the last contents


def test_noalloc_refuses_oversized_problems():
    k = kfscan()
    model, y = W.tracking(16, seed=1)
    dm = k.model_to_device(model.arrays(), "f64")
    yd = torch.as_tensor(y).to("cuda", torch.float64).contiguous()
    p, keep = k.make_problem(dm, yd, "f64", "auto")
    p.T = 1 << 27                         # sizes only: nothing is launched
    p.nseq = 4
    assert k.workspace_size(p) > SCRATCH_BYTES
    assert _noalloc(k, p, torch.cuda.current_stream().cuda_stream) == k.KF_ERR_WORKSPACE
