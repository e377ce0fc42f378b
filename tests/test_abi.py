"""C-ABI checks that need no GPU: the library loads, exports every function
that include/kfscan.h declares, and its host-side argument checks and
workspace sizing behave as documented (nothing is launched)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "kfscan.h")
LIB = os.path.join(ROOT, "paper_2511_10363_amd", "libkfscan.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kf_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def kfscan():
    if not os.path.exists(LIB):
        pytest.fail("libkfscan.so is not built (run __graft_entry__.build())")
    from paper_2511_10363_amd import kfscan as k
    k.load_library()
    return k


def test_header_declares_the_three_entry_points():
    names = _declared()
    for n in ("kf_filter", "kf_smooth_rts", "kf_smooth_twofilter", "kf_workspace_size"):
        assert n in names


def test_every_declared_symbol_is_exported(kfscan):
    lib = ctypes.CDLL(LIB)
    for name in _declared():
        assert hasattr(lib, name), name
    assert set(kfscan.EXPORTS) <= set(_declared())


def test_abi_version_and_status_strings(kfscan):
    lib = kfscan.load_library()
    assert lib.kf_abi_version() == 1
    for code in range(5):
        assert kfscan.status_string(code)


def _problem(kfscan, nx=4, ny=2, prec=1, T=1 << 20, nseq=1, scan=0):
    p = kfscan.KfProblem()
    p.nx, p.ny, p.precision, p.scan, p.T, p.nseq = nx, ny, prec, scan, T, nseq
    return p


def test_workspace_size_and_validation(kfscan):
    lib = kfscan.load_library()
    n = ctypes.c_size_t(0)
    p = _problem(kfscan)
    assert lib.kf_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    assert n.value > 0 and n.value % 256 == 0
    n64 = ctypes.c_size_t(0)
    assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, prec=0)), ctypes.byref(n64)) == 0
    assert n64.value > n.value
    assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, nx=5)), ctypes.byref(n)) == 2
    assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, T=0)), ctypes.byref(n)) == 1
    assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, prec=7)), ctypes.byref(n)) == 1
    assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, nseq=0)), ctypes.byref(n)) == 1
    assert lib.kf_workspace_size(None, ctypes.byref(n)) == 1


def test_entry_points_reject_before_launch(kfscan):
    """Null pointers and missing workspaces are refused on the host."""
    lib = kfscan.load_library()
    p = _problem(kfscan, T=100)
    for name in ("kf_filter", "kf_smooth_rts", "kf_smooth_twofilter"):
        assert getattr(lib, name)(ctypes.byref(p), None, 0, None) == 1
    # all pointers set to a fake aligned address, but no workspace: workspace error
    for f in ("F", "Q", "H", "R", "m0", "P0", "y", "m_filt", "P_filt", "m_smooth", "P_smooth"):
        setattr(p, f, 4096)
    assert lib.kf_filter(ctypes.byref(p), None, 0, None) == 3
    assert lib.kf_filter(ctypes.byref(p), 4096 + 16, 1 << 30, None) == 3  # misaligned


def test_supported_shapes(kfscan):
    assert kfscan.supported(4, 2, "f32") and kfscan.supported(4, 2, "f64")
    assert not kfscan.supported(5, 2, "f32")
