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
