"""MI355X-native parallel-in-time Kalman filter and smoothers (arXiv 2511.10363).

The computation lives in libkfscan.so (HIP kernels for gfx950 behind the C ABI
of include/kfscan.h); ``kfscan`` is its Python binding.
"""
from . import kfscan  # noqa: F401
from .kfscan import (filter, smooth_rts, smooth_twofilter, supported,  # noqa: F401
                     model_to_device, KfScanError)

__all__ = ["kfscan", "filter", "smooth_rts", "smooth_twofilter", "supported",
           "model_to_device", "KfScanError"]
