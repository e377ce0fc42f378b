"""Python binding of the C ABI in include/kfscan.h (argument marshalling only).

PyTorch supplies device memory and the current HIP stream; every step of the
filter and smoothers runs in the HIP kernels of libkfscan.so.  There is no
CPU path: if the library is missing, or a tensor is not on a GPU, the call
raises.

    m_f, P_f = filter(model, y)
    m_f, P_f, m_s, P_s = smooth_rts(model, y)
    m_f, P_f, m_s, P_s = smooth_twofilter(model, y)

``model`` is any object with tensor attributes F, Q, H, R, m0, P0 (or a tuple
in that order); ``y`` is ``[T, ny]`` or ``[nseq, T, ny]``.  ``precision`` is
"f64", "f32" or "mixed" (FP32 storage with FP64 solves, KF_PREC_F32_F64SOLVE).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkfscan.so")

(KF_OK, KF_ERR_INVALID_ARG, KF_ERR_UNSUPPORTED, KF_ERR_WORKSPACE, KF_ERR_DEVICE,
 KF_ERR_NUMERIC) = range(6)
# per-sequence status bits (the optional ``status`` tensor of a call) and the
# workspace error bits of workspace_status()
KF_SEQ_NONFINITE, KF_SEQ_INVALID = 1, 2
KF_WS_TIMEOUT, KF_WS_INVALID, KF_WS_NUMERIC = 1, 2, 4
PRECISIONS = {"f64": 0, "f32": 1, "mixed": 2}
SCANS = {"auto": 0, "lookback": 1, "blelloch": 2, "hillis_steele": 3, "lookback_generic": 4,
         "sequential": 5, "ladner_fischer": 6, "sengupta_a": 7, "sengupta_b": 8}
_VOIDP = ctypes.c_void_p


class KfProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("scan", ctypes.c_int32),
                ("T", ctypes.c_int64), ("nseq", ctypes.c_int64),
                ("F", _VOIDP), ("Q", _VOIDP), ("H", _VOIDP), ("R", _VOIDP),
                ("m0", _VOIDP), ("P0", _VOIDP), ("y", _VOIDP),
                ("m_filt", _VOIDP), ("P_filt", _VOIDP),
                ("m_smooth", _VOIDP), ("P_smooth", _VOIDP), ("status", _VOIDP),
                ("items", ctypes.c_int32)]


class KfBatch(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("scan", ctypes.c_int32),
                ("nseq", ctypes.c_int64), ("nmodels", ctypes.c_int64),
                ("total_steps", ctypes.c_int64), ("T", _VOIDP), ("offset", _VOIDP),
                ("F", _VOIDP), ("Q", _VOIDP), ("H", _VOIDP), ("R", _VOIDP),
                ("m0", _VOIDP), ("P0", _VOIDP), ("y", _VOIDP),
                ("m_filt", _VOIDP), ("P_filt", _VOIDP),
                ("m_smooth", _VOIDP), ("P_smooth", _VOIDP), ("status", _VOIDP),
                ("items", ctypes.c_int32)]


class KfTvProblem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("scan", ctypes.c_int32),
                ("T", ctypes.c_int64), ("nseq", ctypes.c_int64),
                ("F", _VOIDP), ("Q", _VOIDP), ("H", _VOIDP), ("R", _VOIDP),
                ("u", _VOIDP), ("d", _VOIDP), ("m0", _VOIDP), ("P0", _VOIDP), ("y", _VOIDP),
                ("m_filt", _VOIDP), ("P_filt", _VOIDP),
                ("m_smooth", _VOIDP), ("P_smooth", _VOIDP), ("status", _VOIDP),
                ("items", ctypes.c_int32)]


class KfScanError(RuntimeError):
    pass


_lib = None
_lock = threading.Lock()
EXPORTS = ("kf_abi_version", "kf_status_string", "kf_supported", "kf_workspace_size",
           "kf_workspace_clear", "kf_workspace_timed_out", "kf_device_copy", "kf_filter", "kf_smooth_rts",
           "kf_smooth_twofilter", "kf_prepare", "kf_pass_filter", "kf_pass_rts",
           "kf_pass_twofilter", "kf_batch_workspace_size", "kf_filter_batch",
           "kf_smooth_rts_batch", "kf_smooth_twofilter_batch", "kf_workspace_status",
           "kf_tv_workspace_size", "kf_filter_tv", "kf_smooth_rts_tv", "kf_smooth_twofilter_tv",
           "kf_scan_counts", "kf_selftest_scan_workspace", "kf_selftest_scan")
STAGES = ("kf_prepare", "kf_pass_filter", "kf_pass_rts", "kf_pass_twofilter")
# When set (the tests set it), every call synchronises and checks the
# workspace's look-back timeout flag.
CHECK = os.environ.get("KFSCAN_CHECK", "0") == "1"


def load_library(path: str = LIB_PATH):
    """Load libkfscan.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(path):
            raise KfScanError("%s is not built; run paper_2511_10363_amd.build.build()" % path)
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(KfProblem)
        lib.kf_abi_version.restype = ctypes.c_int
        lib.kf_status_string.restype = ctypes.c_char_p
        lib.kf_status_string.argtypes = [ctypes.c_int]
        lib.kf_supported.restype = ctypes.c_int
        lib.kf_supported.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        lib.kf_workspace_size.restype = ctypes.c_int
        lib.kf_workspace_size.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
        lib.kf_workspace_clear.restype = ctypes.c_int
        lib.kf_workspace_clear.argtypes = [_VOIDP, ctypes.c_size_t, _VOIDP]
        B = ctypes.POINTER(KfBatch)
        lib.kf_batch_workspace_size.restype = ctypes.c_int
        lib.kf_batch_workspace_size.argtypes = [B, ctypes.POINTER(ctypes.c_size_t)]
        for name in ("kf_filter_batch", "kf_smooth_rts_batch", "kf_smooth_twofilter_batch"):
            getattr(lib, name).restype = ctypes.c_int
            getattr(lib, name).argtypes = [B, _VOIDP, ctypes.c_size_t, _VOIDP]
        V = ctypes.POINTER(KfTvProblem)
        lib.kf_tv_workspace_size.restype = ctypes.c_int
        lib.kf_tv_workspace_size.argtypes = [V, ctypes.POINTER(ctypes.c_size_t)]
        for name in ("kf_filter_tv", "kf_smooth_rts_tv", "kf_smooth_twofilter_tv"):
            getattr(lib, name).restype = ctypes.c_int
            getattr(lib, name).argtypes = [V, _VOIDP, ctypes.c_size_t, _VOIDP]
        lib.kf_workspace_status.restype = ctypes.c_int
        lib.kf_workspace_status.argtypes = [_VOIDP, ctypes.c_size_t, ctypes.POINTER(ctypes.c_uint32),
                                            _VOIDP]
        lib.kf_scan_counts.restype = ctypes.c_int
        lib.kf_scan_counts.argtypes = [ctypes.c_int32, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        lib.kf_selftest_scan_workspace.restype = ctypes.c_int
        lib.kf_selftest_scan_workspace.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.c_int64, ctypes.c_int64,
                                                   ctypes.POINTER(ctypes.c_size_t)]
        lib.kf_selftest_scan.restype = ctypes.c_int
        lib.kf_selftest_scan.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, _VOIDP,
                                         _VOIDP, _VOIDP, ctypes.c_size_t, _VOIDP]
        lib.kf_device_copy.restype = ctypes.c_int
        lib.kf_device_copy.argtypes = [_VOIDP, _VOIDP, ctypes.c_size_t, _VOIDP]
        lib.kf_workspace_timed_out.restype = ctypes.c_int
        lib.kf_workspace_timed_out.argtypes = [P, _VOIDP, ctypes.c_size_t,
                                               ctypes.POINTER(ctypes.c_int32), _VOIDP]
        for name in ("kf_filter", "kf_smooth_rts", "kf_smooth_twofilter") + STAGES:
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [P, _VOIDP, ctypes.c_size_t, _VOIDP]
        _lib = lib
        return lib


def status_string(code: int) -> str:
    return load_library().kf_status_string(code).decode()


def _check(code: int, what: str):
    if code != KF_OK:
        raise KfScanError("%s: %s (status %d)" % (what, status_string(code), code))


def dtype_for(precision: str) -> torch.dtype:
    return torch.float64 if precision == "f64" else torch.float32


def _model_tensors(model):
    if isinstance(model, (tuple, list)):
        return tuple(model[:6])
    return (model.F, model.Q, model.H, model.R, model.m0, model.P0)


class Workspace:
    """Device workspace, grown on demand, one per (device, stream).  Calls on
    one stream run in order, and each call re-initialises the control words it
    uses, so reuse needs no clearing."""

    _cache: dict = {}

    @classmethod
    def get(cls, device: torch.device, stream: int, nbytes: int) -> torch.Tensor:
        key = (device.index, stream)
        buf = cls._cache.get(key)
        if buf is None or buf.numel() < nbytes:
            buf = torch.empty(max(nbytes, 1 << 20), dtype=torch.uint8, device=device)
            cls._cache[key] = buf
        return buf


def _status_ptr(status, nseq, dev):
    """Device pointer of an optional per-sequence status tensor (int32 [nseq])."""
    if status is None:
        return None
    if (status.dtype != torch.int32 or tuple(status.shape) != (nseq,) or status.device != dev
            or not status.is_contiguous()):
        raise ValueError("status must be a contiguous int32 [%d] tensor on %s" % (nseq, dev))
    return status.data_ptr()


def make_problem(model, y, precision="f32", scan="auto", m_filt=None, P_filt=None,
                 m_smooth=None, P_smooth=None, status=None, items=0):
    """Validate tensors and fill a KfProblem.  Returns (problem, keepalive).
    ``status`` is an optional int32 [nseq] GPU tensor that receives each
    sequence's KF_SEQ_* bits (non-finite results are then replaced by NaN)."""
    if precision not in PRECISIONS:
        raise ValueError("precision must be one of %s" % list(PRECISIONS))
    if scan not in SCANS:
        raise ValueError("scan must be one of %s" % list(SCANS))
    dt = dtype_for(precision)
    F, Q, H, R, m0, P0 = _model_tensors(model)
    if y.dim() == 2:
        y = y.unsqueeze(0)
    if y.dim() != 3:
        raise ValueError("y must be [T, ny] or [nseq, T, ny]")
    nseq, T, ny = y.shape
    nx = F.shape[-1]
    dev = y.device
    if dev.type != "cuda":
        raise KfScanError("kfscan runs on the GPU only; y is on %s" % dev)
    shapes = {"F": (F, (nx, nx)), "Q": (Q, (nx, nx)), "H": (H, (ny, nx)), "R": (R, (ny, ny)),
              "m0": (m0, (nx,)), "P0": (P0, (nx, nx))}
    for name, (t, shp) in shapes.items():
        if tuple(t.shape) != shp:
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shp))
        if t.device != dev or t.dtype != dt or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dt, dev))
    if y.dtype != dt or not y.is_contiguous():
        raise ValueError("y must be a contiguous %s tensor" % dt)
    if m_filt is None:
        m_filt = torch.empty((nseq, T, nx), dtype=dt, device=dev)
    if P_filt is None:
        P_filt = torch.empty((nseq, T, nx, nx), dtype=dt, device=dev)
    p = KfProblem()
    p.nx, p.ny, p.precision, p.scan = nx, ny, PRECISIONS[precision], SCANS[scan]
    p.T, p.nseq = T, nseq
    p.F, p.Q, p.H, p.R = F.data_ptr(), Q.data_ptr(), H.data_ptr(), R.data_ptr()
    p.m0, p.P0, p.y = m0.data_ptr(), P0.data_ptr(), y.data_ptr()
    p.m_filt, p.P_filt = m_filt.data_ptr(), P_filt.data_ptr()
    if m_smooth is not None:
        p.m_smooth, p.P_smooth = m_smooth.data_ptr(), P_smooth.data_ptr()
    p.status = _status_ptr(status, nseq, dev)
    p.items = int(items)
    keep = dict(y=y, m_filt=m_filt, P_filt=P_filt, m_smooth=m_smooth, P_smooth=P_smooth,
                status=status)
    return p, keep


def workspace_size(p: KfProblem) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().kf_workspace_size(ctypes.byref(p), ctypes.byref(n)), "kf_workspace_size")
    return n.value


def _call(entry: str, p: KfProblem, device: torch.device, workspace=None):
    lib = load_library()
    stream = torch.cuda.current_stream(device).cuda_stream
    need = workspace_size(p)
    ws = workspace if workspace is not None else Workspace.get(device, stream, need)
    if ws.numel() * ws.element_size() < need:
        raise KfScanError("workspace of %d bytes is smaller than the %d needed"
                          % (ws.numel() * ws.element_size(), need))
    nbytes = ws.numel() * ws.element_size()
    _check(getattr(lib, entry)(ctypes.byref(p), ws.data_ptr(), nbytes, stream), entry)
    if CHECK:
        flag = ctypes.c_int32(0)
        _check(lib.kf_workspace_timed_out(ctypes.byref(p), ws.data_ptr(), nbytes,
                                          ctypes.byref(flag), stream), "kf_workspace_timed_out")
        if flag.value:
            raise KfScanError("%s: a look-back wait timed out; outputs are invalid" % entry)


def _squeeze(x, was2d):
    return x[0] if was2d else x


def filter(model, y, precision="f32", scan="auto", workspace=None, status=None,  # noqa: A001
           items=0):
    """Algorithm 5.  Returns (x_{k|k}, P_{k|k})."""
    was2d = y.dim() == 2
    p, keep = make_problem(model, y, precision, scan, status=status, items=items)
    _call("kf_filter", p, y.device, workspace)
    return _squeeze(keep["m_filt"], was2d), _squeeze(keep["P_filt"], was2d)


def _smoother(entry, model, y, precision, scan, workspace, status=None, items=0):
    was2d = y.dim() == 2
    yy = y.unsqueeze(0) if was2d else y
    nseq, T, _ = yy.shape
    nx = _model_tensors(model)[0].shape[-1]
    dt = dtype_for(precision)
    m_s = torch.empty((nseq, T, nx), dtype=dt, device=y.device)
    P_s = torch.empty((nseq, T, nx, nx), dtype=dt, device=y.device)
    p, keep = make_problem(model, yy, precision, scan, m_smooth=m_s, P_smooth=P_s,
                           status=status, items=items)
    _call(entry, p, y.device, workspace)
    return tuple(_squeeze(keep[k], was2d) for k in ("m_filt", "P_filt", "m_smooth", "P_smooth"))


def smooth_rts(model, y, precision="f32", scan="auto", workspace=None, status=None, items=0):
    """Algorithm 6.  Returns (x_{k|k}, P_{k|k}, x_{k|T}, P_{k|T})."""
    return _smoother("kf_smooth_rts", model, y, precision, scan, workspace, status, items)


def smooth_twofilter(model, y, precision="f32", scan="auto", workspace=None, status=None,
                     items=0):
    """Algorithm 7.  Returns (x_{k|k}, P_{k|k}, x_{k|T}, P_{k|T})."""
    return _smoother("kf_smooth_twofilter", model, y, precision, scan, workspace, status, items)


def make_batch(models, y, T, offset, precision="f32", scan="auto", smoother=False, status=None,
               items=0, outputs=None):
    """Fill a KfBatch for a ragged batch.  ``models`` holds F, Q, H, R, m0, P0 of
    one shared model, or each with a leading [nseq] dimension (one model per
    sequence); ``y`` is the packed [total_steps, ny] measurements; ``T`` and
    ``offset`` are int64 GPU tensors [nseq] (length and first row of each
    sequence).  Returns (batch, keepalive) with the outputs in keepalive."""
    if precision not in PRECISIONS:
        raise ValueError("precision must be one of %s" % list(PRECISIONS))
    if scan not in SCANS:
        raise ValueError("scan must be one of %s" % list(SCANS))
    dt = dtype_for(precision)
    F, Q, H, R, m0, P0 = _model_tensors(models)
    if y.dim() != 2:
        raise ValueError("y must be packed as [total_steps, ny]")
    dev = y.device
    if dev.type != "cuda":
        raise KfScanError("kfscan runs on the GPU only; y is on %s" % dev)
    total, ny = y.shape
    nx = F.shape[-1]
    nseq = T.shape[0]
    nmodels = F.shape[0] if F.dim() == 3 else 1
    lead = (nmodels,) if F.dim() == 3 else ()
    shapes = {"F": (F, (nx, nx)), "Q": (Q, (nx, nx)), "H": (H, (ny, nx)), "R": (R, (ny, ny)),
              "m0": (m0, (nx,)), "P0": (P0, (nx, nx))}
    for name, (t, shp) in shapes.items():
        if tuple(t.shape) != lead + shp:
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), lead + shp))
        if t.device != dev or t.dtype != dt or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dt, dev))
    for name, t in (("T", T), ("offset", offset)):
        if t.shape != (nseq,) or t.dtype != torch.int64 or t.device != dev or not t.is_contiguous():
            raise ValueError("%s must be a contiguous int64 [nseq] tensor on %s" % (name, dev))
    if y.dtype != dt or not y.is_contiguous():
        raise ValueError("y must be a contiguous %s tensor" % dt)
    if outputs is not None:
        # caller-owned output arrays (m_filt, P_filt[, m_smooth, P_smooth]) of
        # [total_steps, nx] / [total_steps, nx, nx]
        outs = list(outputs) + [None] * (4 - len(outputs))
        for t, shp in zip(outs, [(total, nx), (total, nx, nx)] * 2):
            if t is not None and (tuple(t.shape) != shp or t.dtype != dt or t.device != dev
                                  or not t.is_contiguous()):
                raise ValueError("output arrays must be contiguous %s tensors of shape %s"
                                 % (dt, shp))
        keep = dict(y=y, T=T, offset=offset, m_filt=outs[0], P_filt=outs[1],
                    m_smooth=outs[2], P_smooth=outs[3])
        if smoother and outs[2] is None:
            raise ValueError("a smoother needs m_smooth and P_smooth outputs")
    else:
        keep = dict(y=y, T=T, offset=offset,
                    m_filt=torch.empty((total, nx), dtype=dt, device=dev),
                    P_filt=torch.empty((total, nx, nx), dtype=dt, device=dev),
                    m_smooth=None, P_smooth=None)
        if smoother:
            keep["m_smooth"] = torch.empty((total, nx), dtype=dt, device=dev)
            keep["P_smooth"] = torch.empty((total, nx, nx), dtype=dt, device=dev)
    b = KfBatch()
    b.nx, b.ny, b.precision, b.scan = nx, ny, PRECISIONS[precision], SCANS[scan]
    b.nseq, b.nmodels, b.total_steps = nseq, nmodels, total
    b.T, b.offset = T.data_ptr(), offset.data_ptr()
    b.F, b.Q, b.H, b.R = F.data_ptr(), Q.data_ptr(), H.data_ptr(), R.data_ptr()
    b.m0, b.P0, b.y = m0.data_ptr(), P0.data_ptr(), y.data_ptr()
    b.m_filt, b.P_filt = keep["m_filt"].data_ptr(), keep["P_filt"].data_ptr()
    if smoother:
        b.m_smooth, b.P_smooth = keep["m_smooth"].data_ptr(), keep["P_smooth"].data_ptr()
    b.status = _status_ptr(status, nseq, dev)
    b.items = int(items)
    keep["status"] = status
    return b, keep


def batch_workspace_size(b: KfBatch) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().kf_batch_workspace_size(ctypes.byref(b), ctypes.byref(n)),
           "kf_batch_workspace_size")
    return n.value


def workspace_status(ws: torch.Tensor) -> int:
    """Error bits of the last call on this workspace (synchronises the current
    stream): KF_WS_TIMEOUT = a look-back wait gave up, KF_WS_INVALID = invalid
    ragged-batch entries, KF_WS_NUMERIC = a sequence's outputs held non-finite
    values (calls with a status tensor only)."""
    flag = ctypes.c_uint32(0)
    stream = torch.cuda.current_stream(ws.device).cuda_stream
    rc = load_library().kf_workspace_status(ws.data_ptr(), ws.numel() * ws.element_size(),
                                            ctypes.byref(flag), stream)
    if rc != KF_ERR_NUMERIC:
        _check(rc, "kf_workspace_status")
    return flag.value


def run_batch(entry, b: KfBatch, device, workspace=None):
    """Enqueue kf_filter_batch / kf_smooth_rts_batch / kf_smooth_twofilter_batch."""
    lib = load_library()
    stream = torch.cuda.current_stream(device).cuda_stream
    need = batch_workspace_size(b)
    ws = workspace if workspace is not None else Workspace.get(device, stream, need)
    nbytes = ws.numel() * ws.element_size()
    if nbytes < need:
        raise KfScanError("workspace of %d bytes is smaller than the %d needed" % (nbytes, need))
    _check(getattr(lib, entry)(ctypes.byref(b), ws.data_ptr(), nbytes, stream), entry)
    if CHECK and workspace_status(ws) & 1:
        raise KfScanError("%s: a look-back wait timed out; outputs are invalid" % entry)
    return ws


def batch(entry, models, y, T, offset, precision="f32", scan="auto", workspace=None,
          status=None, items=0):
    """One ragged-batch call; entry is "filter", "rts" or "tf".  Returns the
    packed outputs (m_filt, P_filt[, m_smooth, P_smooth]) and the workspace."""
    name = {"filter": "kf_filter_batch", "rts": "kf_smooth_rts_batch",
            "tf": "kf_smooth_twofilter_batch"}[entry]
    b, keep = make_batch(models, y, T, offset, precision, scan, smoother=(entry != "filter"),
                         status=status, items=items)
    ws = run_batch(name, b, y.device, workspace)
    outs = (keep["m_filt"], keep["P_filt"])
    if entry != "filter":
        outs += (keep["m_smooth"], keep["P_smooth"])
    return outs, ws


def tv(entry, F, Q, H, R, u, d, m0, P0, y, precision="f32", scan="auto", workspace=None,
       status=None):
    """A time-varying model (kf_*_tv): F, Q [T, nx, nx], H [T, ny, nx], R [T, ny, ny],
    u [T, nx] or None, d [T, ny] or None (row j belongs to step j+1), prior m0,
    P0, measurements y [T, ny] or [nseq, T, ny].  entry is "filter", "rts" or
    "tf".  Returns (x_{k|k}, P_{k|k}[, x_{k|T}, P_{k|T}])."""
    if precision not in PRECISIONS:
        raise ValueError("precision must be one of %s" % list(PRECISIONS))
    dt = dtype_for(precision)
    was2d = y.dim() == 2
    yy = y.unsqueeze(0) if was2d else y
    nseq, T, ny = yy.shape
    nx = F.shape[-1]
    dev = y.device
    if dev.type != "cuda":
        raise KfScanError("kfscan runs on the GPU only; y is on %s" % dev)
    shapes = {"F": (F, (T, nx, nx)), "Q": (Q, (T, nx, nx)), "H": (H, (T, ny, nx)),
              "R": (R, (T, ny, ny)), "m0": (m0, (nx,)), "P0": (P0, (nx, nx))}
    if u is not None:
        shapes["u"] = (u, (T, nx))
    if d is not None:
        shapes["d"] = (d, (T, ny))
    for name, (t, shp) in shapes.items():
        if tuple(t.shape) != shp:
            raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), shp))
        if t.device != dev or t.dtype != dt or not t.is_contiguous():
            raise ValueError("%s must be a contiguous %s tensor on %s" % (name, dt, dev))
    if yy.dtype != dt or not yy.is_contiguous():
        raise ValueError("y must be a contiguous %s tensor" % dt)
    outs = [torch.empty((nseq, T, nx), dtype=dt, device=dev),
            torch.empty((nseq, T, nx, nx), dtype=dt, device=dev)]
    if entry != "filter":
        outs += [torch.empty((nseq, T, nx), dtype=dt, device=dev),
                 torch.empty((nseq, T, nx, nx), dtype=dt, device=dev)]
    p = KfTvProblem()
    p.nx, p.ny, p.precision, p.scan = nx, ny, PRECISIONS[precision], SCANS[scan]
    p.T, p.nseq = T, nseq
    p.F, p.Q, p.H, p.R = F.data_ptr(), Q.data_ptr(), H.data_ptr(), R.data_ptr()
    p.u = u.data_ptr() if u is not None else None
    p.d = d.data_ptr() if d is not None else None
    p.m0, p.P0, p.y = m0.data_ptr(), P0.data_ptr(), yy.data_ptr()
    p.m_filt, p.P_filt = outs[0].data_ptr(), outs[1].data_ptr()
    if entry != "filter":
        p.m_smooth, p.P_smooth = outs[2].data_ptr(), outs[3].data_ptr()
    p.status = _status_ptr(status, nseq, dev)
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.kf_tv_workspace_size(ctypes.byref(p), ctypes.byref(n)), "kf_tv_workspace_size")
    stream = torch.cuda.current_stream(dev).cuda_stream
    ws = workspace if workspace is not None else Workspace.get(dev, stream, n.value)
    nbytes = ws.numel() * ws.element_size()
    name = {"filter": "kf_filter_tv", "rts": "kf_smooth_rts_tv", "tf": "kf_smooth_twofilter_tv"}[entry]
    _check(getattr(lib, name)(ctypes.byref(p), ws.data_ptr(), nbytes, stream), name)
    if CHECK and workspace_status(ws) & 1:
        raise KfScanError("%s: a look-back wait timed out; outputs are invalid" % name)
    return tuple(_squeeze(o, was2d) for o in outs)


class Plan:
    """A problem bound to preallocated device buffers, for repeated calls and
    for stage-by-stage launches (kf_prepare, kf_pass_*), e.g. to time each
    kernel with events on the current stream."""

    def __init__(self, model, y, precision="f32", scan="auto", smoother=True, workspace=None,
                 items=0):
        was2d = y.dim() == 2
        yy = y.unsqueeze(0) if was2d else y
        nseq, T, _ = yy.shape
        nx = _model_tensors(model)[0].shape[-1]
        dt = dtype_for(precision)
        self.model = model
        self.m_s = self.P_s = None
        if smoother:
            self.m_s = torch.empty((nseq, T, nx), dtype=dt, device=y.device)
            self.P_s = torch.empty((nseq, T, nx, nx), dtype=dt, device=y.device)
        self.p, self.keep = make_problem(model, yy, precision, scan, m_smooth=self.m_s,
                                         P_smooth=self.P_s, items=items)
        self.device = y.device
        self.need = workspace_size(self.p)
        self.ws = workspace if workspace is not None else torch.empty(
            max(self.need, 1 << 20), dtype=torch.uint8, device=y.device)
        self.lib = load_library()

    def __call__(self, entry: str):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(getattr(self.lib, entry)(ctypes.byref(self.p), self.ws.data_ptr(),
                                        self.ws.numel(), stream), entry)

    def outputs(self):
        return (self.keep["m_filt"], self.keep["P_filt"], self.m_s, self.P_s)


def device_copy(dst: torch.Tensor, src: torch.Tensor) -> None:
    """dst[:] = src[:] (same byte size, contiguous, on one GPU) with the library's
    plain streaming copy kernel, on the current stream."""
    if not (dst.is_cuda and src.is_cuda and dst.is_contiguous() and src.is_contiguous()):
        raise KfScanError("device_copy needs contiguous GPU tensors")
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("device_copy: size mismatch")
    stream = torch.cuda.current_stream(src.device).cuda_stream
    _check(load_library().kf_device_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream),
           "kf_device_copy")


def scan_counts(scan: str, T: int) -> tuple[int, int]:
    """(operator applications, parallel steps that apply it) of one scan of
    kind ``scan`` over T elements (kf_scan_counts)."""
    c, n = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(load_library().kf_scan_counts(SCANS[scan], T, ctypes.byref(c), ctypes.byref(n)),
           "kf_scan_counts")
    return c.value, n.value


AFFINE_MODULUS = {"f64": 33554393, "f32": 2039}


def selftest_scan(elems: torch.Tensor, reverse: bool = False, items: int = 8,
                  group: int = 1) -> torch.Tensor:
    """Run a look-back scan skeleton with the exact affine operator of
    kf_selftest_scan over ``elems`` [nseq, T, 10] (float64 or float32 integers
    below AFFINE_MODULUS); returns the composed maps' (b, C) [nseq, T, 6].
    group 1 is the thread driver, 8 or 16 the group driver of the wide scans."""
    if elems.dim() != 3 or elems.shape[-1] != 10 or not elems.is_contiguous():
        raise ValueError("elems must be a contiguous [nseq, T, 10] tensor")
    if elems.device.type != "cuda":
        raise KfScanError("kfscan runs on the GPU only; elems is on %s" % elems.device)
    prec = {torch.float64: 0, torch.float32: 1}.get(elems.dtype)
    if prec is None:
        raise ValueError("elems must be float64 or float32")
    nseq, T, _ = elems.shape
    lib = load_library()
    n = ctypes.c_size_t(0)
    _check(lib.kf_selftest_scan_workspace(prec, group, items, T, nseq, ctypes.byref(n)),
           "kf_selftest_scan_workspace")
    ws = torch.empty(max(n.value, 256), dtype=torch.uint8, device=elems.device)
    out = torch.empty((nseq, T, 6), dtype=elems.dtype, device=elems.device)
    stream = torch.cuda.current_stream(elems.device).cuda_stream
    _check(lib.kf_selftest_scan(prec, group, int(bool(reverse)), items, T, nseq,
                                elems.data_ptr(), out.data_ptr(), ws.data_ptr(), ws.numel(),
                                stream), "kf_selftest_scan")
    if CHECK:
        flag = ctypes.c_uint32(0)
        rc = lib.kf_workspace_status(ws.data_ptr(), ws.numel(), ctypes.byref(flag), stream)
        _check(rc, "kf_workspace_status")
        if flag.value & KF_WS_TIMEOUT:
            raise KfScanError("kf_selftest_scan: a look-back wait timed out")
    return out


def supported(nx: int, ny: int, precision: str = "f32") -> bool:
    return bool(load_library().kf_supported(nx, ny, PRECISIONS[precision]))


def model_to_device(model, precision="f32", device="cuda"):
    """Copy numpy/torch model arrays to contiguous device tensors of the
    precision's storage dtype.  Returns a tuple (F, Q, H, R, m0, P0)."""
    dt = dtype_for(precision)
    return tuple(torch.as_tensor(a).to(device=device, dtype=dt).contiguous()
                 for a in _model_tensors(model))
