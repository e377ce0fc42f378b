"""CPU FP64 oracle for the parallel-in-time Kalman filter and smoothers.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library and never imports it.

The arithmetic lives in ``kf_oracle.c`` (plain C, FP64, sequential), compiled
with gcc into ``liboracle.so`` beside this file.  This module only marshals
numpy arrays.  Paper references (Sarkka & Garcia-Fernandez, arXiv 2511.10363):

* ``kf_filter``          -- Kalman filter, Sec. III-A (eqs. KF_mean_pred..KF_cov_upd)
* ``rts``                -- RTS smoother, Sec. III-B (forward-backward smoother)
* ``backward_info``      -- backward information filter, Sec. III-B
                            (eqs. tf_vector_pred..tf_matrix_upd)
* ``tf_combine``         -- two-filter combination (eqs. mean_tf_combination,
                            cov_tf_combination)
* ``filter_elements`` / ``filter_combine``  -- eqs. pkf_init1..3 and Lemma 1
* ``smooth_elements`` / ``smooth_combine``  -- eqs. prts_init1..2 and Lemma 2
* ``pkf`` / ``prts`` / ``ptfs``  -- Algorithms 5, 6 and 7 of Sec. IV with a
  caller-chosen scan from ``oracle.scans`` (sequential by default).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import scans

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kf_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
_lock = threading.Lock()

_dp = ctypes.POINTER(ctypes.c_double)


def build(force: bool = False) -> str:
    """Compile kf_oracle.c with gcc into liboracle.so (always when ``force``)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB_PATH)
            L, I, P = ctypes.c_long, ctypes.c_int, _dp
            lib.kfo_filter.argtypes = [I, I, L, P, L, P, L, P, L, P, L, P, I, P, I,
                                       P, P, P, P, P, P, P]
            lib.kfo_rts.argtypes = [I, L, P, L, P, P, P, P, P, P]
            lib.kfo_backward_info.argtypes = [I, I, L, P, L, P, L, P, L, P, L, P, I, P, I,
                                              P, P, P]
            lib.kfo_tf_combine.argtypes = [I, L, P, P, P, P, P, P]
            lib.kfo_filter_elements.argtypes = [I, I, L, P, L, P, L, P, L, P, L, P, I, P, I,
                                                P, P, P, P, P, P, P, P]
            lib.kfo_filter_combine.argtypes = [I, P, P, P]
            lib.kfo_smooth_elements.argtypes = [I, L, P, L, P, L, P, I, P, P, P, P, P]
            lib.kfo_smooth_combine.argtypes = [I, P, P, P]
            for f in (lib.kfo_filter, lib.kfo_rts, lib.kfo_backward_info, lib.kfo_tf_combine,
                      lib.kfo_filter_elements, lib.kfo_filter_combine,
                      lib.kfo_smooth_elements, lib.kfo_smooth_combine):
                f.restype = ctypes.c_int
            _lib = lib
    return _lib


class use_library:
    """Context manager that points the wrappers at another build of kf_oracle.c
    (the mutation tests plant mistakes in copies of the source)."""

    def __init__(self, path):
        self.path = path

    def __enter__(self):
        global _lib
        _load()
        self._saved = _lib
        lib = ctypes.CDLL(self.path)
        for name in ("kfo_filter", "kfo_rts", "kfo_backward_info", "kfo_tf_combine",
                     "kfo_filter_elements", "kfo_filter_combine", "kfo_smooth_elements",
                     "kfo_smooth_combine"):
            fn = getattr(lib, name)
            fn.argtypes = getattr(self._saved, name).argtypes
            fn.restype = ctypes.c_int
        _lib = lib
        return lib

    def __exit__(self, *exc):
        global _lib
        _lib = self._saved
        return False


def source_path() -> str:
    return _SRC


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _check(rc, what):
    if rc == 1:
        raise ValueError("oracle %s: bad arguments" % what)
    if rc == 2:
        raise np.linalg.LinAlgError("oracle %s: factorisation failed" % what)


class _Model:
    """Model arrays, shared (2-D) or per step (3-D with a leading T axis)."""

    def __init__(self, F, Q, H, R, T, u=None, d=None):
        self.F, self.Q, self.H, self.R = _f64(F), _f64(Q), _f64(H), _f64(R)
        self.nx = self.F.shape[-1]
        self.ny = self.H.shape[-2]
        n, m = self.nx, self.ny
        self.sF = self._stride(self.F, (n, n), T, "F")
        self.sQ = self._stride(self.Q, (n, n), T, "Q")
        self.sH = self._stride(self.H, (m, n), T, "H")
        self.sR = self._stride(self.R, (m, m), T, "R")
        self.u = None if u is None else _f64(u)
        self.d = None if d is None else _f64(d)
        self.u_step = int(self.u is not None and self.u.ndim == 2)
        self.d_step = int(self.d is not None and self.d.ndim == 2)
        if self.u is not None and self.u.shape[-1] != n:
            raise ValueError("u has the wrong width")
        if self.d is not None and self.d.shape[-1] != m:
            raise ValueError("d has the wrong width")
        if self.u_step and self.u.shape[0] < T:
            raise ValueError("per-step u needs T rows")
        if self.d_step and self.d.shape[0] < T:
            raise ValueError("per-step d needs T rows")

    @staticmethod
    def _stride(a, shape, T, name):
        if a.shape == shape:
            return 0
        if a.ndim == 3 and a.shape[1:] == shape and a.shape[0] >= T:
            return shape[0] * shape[1]
        raise ValueError("%s has shape %s, expected %s or (T,)+%s" % (name, a.shape, shape, shape))

    def args(self):
        return (_ptr(self.F), self.sF, _ptr(self.Q), self.sQ, _ptr(self.H), self.sH,
                _ptr(self.R), self.sR, _ptr(self.u), self.u_step, _ptr(self.d), self.d_step)


def kf_filter(F, Q, H, R, m0, P0, y, u=None, d=None):
    """Sequential Kalman filter (Sec. III-A).

    Returns ``(m_f, P_f, m_p, P_p)``: filtered x_{k|k}, P_{k|k} and predicted
    x_{k|k-1}, P_{k|k-1} for k = 1..T at rows 0..T-1.
    """
    lib = _load()
    y = _f64(y)
    T = y.shape[0]
    M = _Model(F, Q, H, R, T, u, d)
    n = M.nx
    m_f = np.empty((T, n)); P_f = np.empty((T, n, n))
    m_p = np.empty((T, n)); P_p = np.empty((T, n, n))
    rc = lib.kfo_filter(n, M.ny, T, *M.args(), _ptr(_f64(m0)), _ptr(_f64(P0)), _ptr(y),
                        _ptr(m_f), _ptr(P_f), _ptr(m_p), _ptr(P_p))
    _check(rc, "kf_filter")
    return m_f, P_f, m_p, P_p


def rts(F, m_f, P_f, m_p, P_p):
    """RTS backward pass (Sec. III-B) from the filter's filtered/predicted moments."""
    lib = _load()
    m_f, P_f, m_p, P_p = _f64(m_f), _f64(P_f), _f64(m_p), _f64(P_p)
    T, n = m_f.shape
    F = _f64(F)
    sF = 0 if F.ndim == 2 else n * n
    m_s = np.empty((T, n)); P_s = np.empty((T, n, n))
    rc = lib.kfo_rts(n, T, _ptr(F), sF, _ptr(m_f), _ptr(P_f), _ptr(m_p), _ptr(P_p),
                     _ptr(m_s), _ptr(P_s))
    _check(rc, "rts")
    return m_s, P_s


def smooth_rts(F, Q, H, R, m0, P0, y, u=None, d=None):
    """Filter + RTS smoother.  Returns ``(m_f, P_f, m_s, P_s)``."""
    m_f, P_f, m_p, P_p = kf_filter(F, Q, H, R, m0, P0, y, u, d)
    m_s, P_s = rts(F, m_f, P_f, m_p, P_p)
    return m_f, P_f, m_s, P_s


def backward_info(F, Q, H, R, y, u=None, d=None):
    """Backward information filter (Sec. III-B, two-filter smoother).

    Returns ``(eta, J)`` with eta_{k|k+1:T}, J_{k|k+1:T} at row k-1 (zero at k = T).
    """
    lib = _load()
    y = _f64(y)
    T = y.shape[0]
    M = _Model(F, Q, H, R, T, u, d)
    n = M.nx
    eta = np.empty((T, n)); J = np.empty((T, n, n))
    rc = lib.kfo_backward_info(n, M.ny, T, *M.args(), _ptr(y), _ptr(eta), _ptr(J))
    _check(rc, "backward_info")
    return eta, J


def tf_combine(m_f, P_f, eta, J):
    """Two-filter combination (eqs. mean_tf_combination, cov_tf_combination)."""
    lib = _load()
    m_f, P_f, eta, J = _f64(m_f), _f64(P_f), _f64(eta), _f64(J)
    T, n = m_f.shape
    m_s = np.empty((T, n)); P_s = np.empty((T, n, n))
    rc = lib.kfo_tf_combine(n, T, _ptr(m_f), _ptr(P_f), _ptr(eta), _ptr(J), _ptr(m_s), _ptr(P_s))
    _check(rc, "tf_combine")
    return m_s, P_s


def smooth_twofilter(F, Q, H, R, m0, P0, y, u=None, d=None):
    """Sequential two-filter smoother.  Returns ``(m_f, P_f, m_s, P_s)``."""
    m_f, P_f, _, _ = kf_filter(F, Q, H, R, m0, P0, y, u, d)
    eta, J = backward_info(F, Q, H, R, y, u, d)
    m_s, P_s = tf_combine(m_f, P_f, eta, J)
    return m_f, P_f, m_s, P_s


# ---------------------------------------------------------------------------
# Parallel-form building blocks (Sec. IV)
# ---------------------------------------------------------------------------

def filter_elements(F, Q, H, R, m0, P0, y, u=None, d=None):
    """Filtering elements (eqs. pkf_init1..pkf_init3) as a list of tuples
    ``(A, b, C, eta, J)`` for k = 1..T."""
    lib = _load()
    y = _f64(y)
    T = y.shape[0]
    M = _Model(F, Q, H, R, T, u, d)
    n = M.nx
    A = np.empty((T, n, n)); b = np.empty((T, n)); C = np.empty((T, n, n))
    eta = np.empty((T, n)); J = np.empty((T, n, n))
    rc = lib.kfo_filter_elements(n, M.ny, T, *M.args(), _ptr(_f64(m0)), _ptr(_f64(P0)), _ptr(y),
                                 _ptr(A), _ptr(b), _ptr(C), _ptr(eta), _ptr(J))
    _check(rc, "filter_elements")
    return [(A[k], b[k], C[k], eta[k], J[k]) for k in range(T)]


def _pack(parts):
    return np.concatenate([_f64(p).ravel() for p in parts])


def filter_combine(ei, ej):
    """Filtering operator of Lemma 1 on tuples ``(A, b, C, eta, J)``."""
    lib = _load()
    n = np.asarray(ei[1]).shape[0]
    a, b = _pack(ei), _pack(ej)
    out = np.empty(3 * n * n + 2 * n)
    _check(lib.kfo_filter_combine(n, _ptr(a), _ptr(b), _ptr(out)), "filter_combine")
    nn = n * n
    return (out[:nn].reshape(n, n), out[nn:nn + n].copy(), out[nn + n:2 * nn + n].reshape(n, n),
            out[2 * nn + n:2 * nn + 2 * n].copy(), out[2 * nn + 2 * n:].reshape(n, n))


def filter_identity(n):
    """Two-sided identity (I, 0, 0, 0, 0) of the filtering operator (reading C3)."""
    z = np.zeros((n, n))
    return (np.eye(n), np.zeros(n), z.copy(), np.zeros(n), z.copy())


def smooth_elements(F, Q, m_f, P_f, u=None):
    """Smoothing elements (eqs. prts_init1, prts_init2): list of ``(E, g, L)``."""
    lib = _load()
    m_f, P_f = _f64(m_f), _f64(P_f)
    T, n = m_f.shape
    F, Q = _f64(F), _f64(Q)
    sF = 0 if F.ndim == 2 else n * n
    sQ = 0 if Q.ndim == 2 else n * n
    uu = None if u is None else _f64(u)
    u_step = int(uu is not None and uu.ndim == 2)
    E = np.empty((T, n, n)); g = np.empty((T, n)); L = np.empty((T, n, n))
    rc = lib.kfo_smooth_elements(n, T, _ptr(F), sF, _ptr(Q), sQ, _ptr(uu), u_step,
                                 _ptr(m_f), _ptr(P_f), _ptr(E), _ptr(g), _ptr(L))
    _check(rc, "smooth_elements")
    return [(E[k], g[k], L[k]) for k in range(T)]


def smooth_combine(ei, ej):
    """Smoothing operator of Lemma 2 on tuples ``(E, g, L)``."""
    lib = _load()
    n = np.asarray(ei[1]).shape[0]
    a, b = _pack(ei), _pack(ej)
    out = np.empty(2 * n * n + n)
    _check(lib.kfo_smooth_combine(n, _ptr(a), _ptr(b), _ptr(out)), "smooth_combine")
    nn = n * n
    return (out[:nn].reshape(n, n), out[nn:nn + n].copy(), out[nn + n:].reshape(n, n))


def smooth_identity(n):
    """Two-sided identity (I, 0, 0) of the smoothing operator."""
    return (np.eye(n), np.zeros(n), np.zeros((n, n)))


def pkf(F, Q, H, R, m0, P0, y, u=None, d=None, scan=None):
    """Algorithm 5 (parallel Kalman filter) with a sequential stand-in for the scan.

    ``scan(elements, op, identity)`` defaults to ``scans.sequential``.
    Returns ``(m_f, P_f)``.
    """
    scan = scan or scans.sequential
    elems = filter_elements(F, Q, H, R, m0, P0, y, u, d)
    n = elems[0][1].shape[0]
    s = scan(elems, filter_combine, filter_identity(n))
    return np.stack([e[1] for e in s]), np.stack([e[2] for e in s])


def prts(F, Q, H, R, m0, P0, y, u=None, d=None, scan=None):
    """Algorithm 6 (parallel RTS smoother, filter pass included).

    The reverse scan is ``scans.reverse(scan)``.  Returns ``(m_f, P_f, m_s, P_s)``.
    """
    scan = scan or scans.sequential
    m_f, P_f = pkf(F, Q, H, R, m0, P0, y, u, d, scan)
    elems = smooth_elements(F, Q, m_f, P_f, u)
    n = m_f.shape[1]
    s = scans.reverse(scan)(elems, smooth_combine, smooth_identity(n))
    return m_f, P_f, np.stack([e[1] for e in s]), np.stack([e[2] for e in s])


def ptfs(F, Q, H, R, m0, P0, y, u=None, d=None, scan=None, right_neutral=None):
    """Algorithm 7 (parallel two-filter smoother, filter pass included).

    The reverse scan runs over ``(a_2, ..., a_T, e)``; ``right_neutral`` is the
    appended e (default: the two-sided identity; the paper's all-zero element
    gives the same eta/J because e is only ever a right operand).
    Returns ``(m_f, P_f, m_s, P_s)``.
    """
    scan = scan or scans.sequential
    elems = filter_elements(F, Q, H, R, m0, P0, y, u, d)
    n = elems[0][1].shape[0]
    ident = filter_identity(n)
    fwd = scan(elems, filter_combine, ident)
    e = ident if right_neutral is None else right_neutral
    bwd = scans.reverse(scan)(elems[1:] + [e], filter_combine, ident)
    m_f = np.stack([s[1] for s in fwd]); P_f = np.stack([s[2] for s in fwd])
    eta = np.stack([s[3] for s in bwd]); J = np.stack([s[4] for s in bwd])
    m_s, P_s = tf_combine(m_f, P_f, eta, J)
    return m_f, P_f, m_s, P_s
