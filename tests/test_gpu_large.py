"""GPU parity at large sizes, against the CPU FP64 oracle on every output.

* A slowly mixing scalar random walk (F = H = 1, q = 1e-6, r = 1): the
  steady-state decay per step is 0.999, so no wave, tile or window aggregate
  decays to an exact anchor.  At T = 2^23 + 12345 each scan has over 2000
  tiles of 4096 steps, more than one look-back window (4 x 256 tiles) covers,
  so look-backs walk over many published aggregates and across windows.
* The benchmark model at T = 2^24 (16 x the benchmark length) in FP32:
  16.7M steps, 8192 tiles per reverse scan.
"""
import functools
import sys

import numpy as np
import pytest

import oracle
import kf_workloads as W
from tests.gpu_common import (TOL, TOL_COMPONENT, TOL_Z, componentwise, gpu_available, kfscan,
                              normwise, oracle_inputs_for, zscore, torch)

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@functools.lru_cache(maxsize=2)
def _slow_walk(T, seed):
    model = W.Model(F=np.eye(1), Q=np.array([[1e-6]]), H=np.eye(1), R=np.eye(1),
                    m0=np.zeros(1), P0=np.eye(1), name="slow_walk")
    return model, W.simulate(model, T, np.random.default_rng(seed))


def _compare(entry, model, y, prec, scan="auto"):
    k = kfscan()
    dm = k.model_to_device(model.arrays(), prec)
    yd = torch.as_tensor(y).to("cuda", k.dtype_for(prec)).contiguous()
    fn = {"filter": k.filter, "rts": k.smooth_rts, "tf": k.smooth_twofilter}[entry]
    got = fn(dm, yd, precision=prec, scan=scan)
    torch.cuda.synchronize()
    got = [g.double().cpu().numpy() for g in got]
    del yd
    arrs, yy = oracle_inputs_for(model, y, prec)
    if entry == "filter":
        ref = list(oracle.kf_filter(*arrs, yy)[:2])
    elif entry == "rts":
        ref = list(oracle.smooth_rts(*arrs, yy))
    else:
        ref = list(oracle.smooth_twofilter(*arrs, yy))
    errs = [normwise(g, r) for g, r in zip(got, ref)]
    comp = [componentwise(g, r) for g, r in zip(got, ref)]
    zs = [zscore(got[i], ref[i], ref[i + 1]) for i in range(0, len(got), 2)]
    _say(entry, prec, scan, "T=%d" % len(y), "errors", errs, "componentwise", comp, "z", zs)
    if prec == "f64":
        assert max(comp) <= TOL_COMPONENT["f64"], comp
        assert max(zs) <= TOL_Z["f64"], zs
    return errs


@pytest.mark.parametrize("scan", ["lookback", "lookback_generic"])
@pytest.mark.parametrize("entry", ["filter", "rts", "tf"])
def test_slow_mixing_walk_multi_window_lookback(entry, scan):
    model, y = _slow_walk((1 << 23) + 12345, seed=23)
    for e in _compare(entry, model, y, "f64", scan):
        assert e <= TOL["f64"]


@pytest.mark.parametrize("prec", ["f32", "mixed"])
@pytest.mark.parametrize("entry", ["filter", "rts"])
def test_slow_mixing_walk_fp32(entry, prec):
    """Means to the FP32 bound.  The smoothed covariance P_s = P + G (P_s' - P^-)
    G^T with G = 0.999 at steady state loses about log10(1 / (1 - G)) = 3
    digits to cancellation in FP32 storage, so its bound is 4 x FP32 epsilon
    x 1 / (1 - G) (4.8e-4) rather than the 1e-4 kept for well-conditioned
    models."""
    model, y = _slow_walk((1 << 23) + 12345, seed=23)
    errs = _compare(entry, model, y, prec)
    q, r = 1e-6, 1.0
    pm = (q + np.sqrt(q * q + 4 * q * r)) / 2          # steady predicted variance
    g = (pm - q) / pm                                  # steady RTS gain P / P^-
    tol_cov = 4 * np.finfo(np.float32).eps / (1 - g)
    for i, e in enumerate(errs):
        assert e <= (tol_cov if i == 3 else TOL[prec]), (i, e)


def test_benchmark_model_T_2_24_fp32():
    model, y = W.tracking(1 << 24, seed=24)
    for e in _compare("rts", model, y, "f32"):
        assert e <= TOL["f32"]
