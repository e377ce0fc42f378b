"""GPU parity of the time-varying entry points (kf_filter_tv, kf_smooth_rts_tv,
kf_smooth_twofilter_tv) against the CPU FP64 oracle on the paper's
time-varying model (Sec. VI-A): per-step F_k = 0.99 x orthogonal, random SPD
Q_k and R_k, Gaussian H_k, inputs u_k, d_k."""
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import TOL, gpu_available, kfscan, normwise, torch

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _cast(a, prec):
    return a if prec == "f64" else np.asarray(a, dtype=np.float32).astype(np.float64)


def _check_tv(entry, T, prec, inputs, seed, nx=4, ny=2, nseq=1, scan="auto", ridge=0.0):
    _say("tv", entry, prec, scan, "T=%d" % T, "inputs" if inputs else "no inputs",
         "nseq=%d" % nseq)
    k = kfscan()
    rng = np.random.default_rng(seed)
    model = W.paper_tv_model(T, rng, nx, ny)
    if ridge:
        # better-conditioned noise covariances: Q_k + ridge I, R_k + ridge I
        model.Q = model.Q + ridge * np.eye(nx)
        model.R = model.R + ridge * np.eye(ny)
    if not inputs:
        model.u = np.zeros((T, nx))
        model.d = np.zeros((T, ny))
    ys = np.stack([W.simulate(model, T, rng) for _ in range(nseq)])
    dt = k.dtype_for(prec)
    dev = lambda a: torch.as_tensor(np.ascontiguousarray(a)).to("cuda", dt).contiguous()  # noqa: E731
    u = dev(model.u) if inputs else None
    d = dev(model.d) if inputs else None
    got = k.tv(entry, dev(model.F), dev(model.Q), dev(model.H), dev(model.R), u, d,
               dev(model.m0), dev(model.P0), dev(ys), precision=prec, scan=scan)
    torch.cuda.synchronize()
    got = [g.double().cpu().numpy() for g in got]
    arrs = [_cast(a, prec) for a in (model.F, model.Q, model.H, model.R, model.m0, model.P0)]
    uu = _cast(model.u, prec) if inputs else None
    dd = _cast(model.d, prec) if inputs else None
    for s in range(nseq):
        yy = _cast(ys[s], prec)
        if entry == "filter":
            ref = list(oracle.kf_filter(*arrs, yy, uu, dd)[:2])
        elif entry == "rts":
            ref = list(oracle.smooth_rts(*arrs, yy, uu, dd))
        else:
            ref = list(oracle.smooth_twofilter(*arrs, yy, uu, dd))
        tols = [TOL[prec]] * len(ref)
        if entry == "tf":
            # The backward information filter is ill-conditioned on this model
            # (random SPD Q_k, R_k reach condition numbers ~1e8): the oracle's
            # own parallel form of Algorithm 7 (the paper's elements, folded)
            # and its sequential two-filter recursion differ by up to ~1e-8 in
            # FP64.  The GPU may differ from the sequential oracle by at most 4x
            # that disagreement of two exact formulations (never less than TOL).
            par = oracle.ptfs(*arrs, yy, uu, dd)
            for i in (2, 3):
                tols[i] = max(tols[i], 4.0 * normwise(par[i], ref[i]))
        for g, r, tol in zip(got, ref, tols):
            assert normwise(g[s], r) <= tol, (entry, prec, T, normwise(g[s], r), tol)
        for g in got[1::2]:
            assert np.array_equal(g[s], np.swapaxes(g[s], -1, -2))


@pytest.mark.parametrize("inputs", [True, False])
@pytest.mark.parametrize("prec", ["f64", "f32", "mixed"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_paper_time_varying_model(entry, prec, inputs):
    _check_tv(entry, 5000, prec, inputs, seed=3)


@pytest.mark.parametrize("T", [1, 2, 7, 513, 2048, 2049, 8193, 30000])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_time_varying_lengths_f64(entry, T):
    _check_tv(entry, T, "f64", True, seed=T)


@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_time_varying_batch_of_sequences(entry):
    """Several sequences share the per-step model."""
    _check_tv(entry, 3000, "f64", True, seed=5, nseq=3)


@pytest.mark.parametrize("scan", ["blelloch", "hillis_steele", "ladner_fischer", "sengupta_a",
                                  "sengupta_b"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_time_varying_tree_scans(entry, scan):
    """The one-kernel-per-level scans over the per-step elements, at a length
    past Sengupta B's threshold (T = 40000 pads to 2^16)."""
    _check_tv(entry, 40000, "f64", True, seed=9, scan=scan)


@pytest.mark.parametrize("entry", ["filter", "rts"])
def test_time_varying_ladner_fischer_f32(entry):
    """The configuration of the paper's speedup experiment: FP32, in-place
    Ladner-Fischer, the time-varying model with inputs."""
    _check_tv(entry, 20000, "f32", True, seed=10, scan="ladner_fischer")


@pytest.mark.parametrize("nx,ny", [(1, 1), (2, 1), (3, 2), (4, 4)])
def test_time_varying_shapes(nx, ny):
    _check_tv("rts", 2500, "f64", True, seed=nx * 7 + ny, nx=nx, ny=ny)
