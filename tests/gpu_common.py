"""Shared helpers for the GPU parity tests (GPU path vs the CPU FP64 oracle)."""
from __future__ import annotations

import numpy as np
import pytest

torch = pytest.importorskip("torch")

# Tolerances (normwise, see the design notes): FP64 paths must match the FP64
# oracle to 1e-9; FP32 storage paths to 1e-4 on means and covariances.
TOL = {"f64": 1e-9, "f32": 1e-4, "mixed": 1e-4}


def gpu_available() -> bool:
    return torch.cuda.is_available()


def kfscan():
    from paper_2511_10363_amd import kfscan as k
    k.load_library()
    return k


def normwise(a, ref) -> float:
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    if scale == 0:
        scale = 1.0
    return float(np.max(np.abs(a - ref)) / scale)


# Per-component bounds (FP64 only): every state component of a mean, and every
# covariance entry, against its own scale (componentwise), and the error of
# the means in posterior standard deviations (zscore).
TOL_COMPONENT = {"f64": 1e-9}
TOL_Z = {"f64": 1e-6}


def componentwise(a, ref) -> float:
    """Largest error of one state component or covariance entry, each scaled by
    its own size: a mean's component i by max_k |ref[k, i]|, a covariance
    entry (i, j) by sqrt(max_k ref[k, i, i] * max_k ref[k, j, j]).  Unlike
    normwise, large components (positions of about 1e7 on long tracks) do
    not hide the errors of small ones (velocities)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    err = np.abs(a - ref)
    lead = tuple(range(ref.ndim - (2 if ref.ndim >= 3 else 1)))
    if ref.ndim >= 3 and ref.shape[-1] == ref.shape[-2]:
        d = np.max(np.abs(np.diagonal(ref, axis1=-2, axis2=-1)), axis=lead)
        scale = np.sqrt(np.outer(d, d))
        e = np.max(err, axis=lead)
    else:
        scale = np.max(np.abs(ref), axis=lead)
        e = np.max(err, axis=lead)
    glob = np.max(np.abs(ref)) if ref.size else 1.0
    scale = np.where(scale > 0, scale, glob if glob > 0 else 1.0)
    return float(np.max(e / scale)) if e.size else 0.0


def zscore(m, m_ref, P_ref) -> float:
    """max_{k,i} |m - m_ref| / sqrt(P_ref[k, i, i]): the error of the means in
    posterior standard deviations."""
    m = np.asarray(m, dtype=np.float64)
    m_ref = np.asarray(m_ref, dtype=np.float64)
    sd = np.sqrt(np.diagonal(np.asarray(P_ref, dtype=np.float64), axis1=-2, axis2=-1))
    return float(np.max(np.abs(m - m_ref) / sd)) if m.size else 0.0


def to_dev(model, precision):
    k = kfscan()
    return k.model_to_device(model.arrays(), precision)


def y_dev(y, precision):
    k = kfscan()
    return torch.as_tensor(np.ascontiguousarray(y)).to("cuda", k.dtype_for(precision)).contiguous()


def oracle_inputs_for(model, y, precision):
    """Rounded copies of the inputs as the GPU sees them (FP32 storage rounds
    the model and data; the oracle then runs in FP64 on the same values)."""
    if precision == "f64":
        return model.arrays(), y
    cast = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    return tuple(cast(a) for a in model.arrays()), cast(y)
