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
    assert lib.kf_abi_version() == 5
    for code in range(6):
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


def _batch(kfscan, nx=4, ny=2, prec=1, nseq=100, nmodels=1, total=300000, scan=0):
    b = kfscan.KfBatch()
    b.nx, b.ny, b.precision, b.scan = nx, ny, prec, scan
    b.nseq, b.nmodels, b.total_steps = nseq, nmodels, total
    return b


def test_batch_workspace_size_and_validation(kfscan):
    """Ragged batches: host-side checks of kf_batch_workspace_size."""
    lib = kfscan.load_library()
    n = ctypes.c_size_t(0)
    size = lambda b: lib.kf_batch_workspace_size(ctypes.byref(b), ctypes.byref(n))  # noqa: E731
    assert size(_batch(kfscan)) == 0 and n.value > 0 and n.value % 256 == 0
    shared = n.value
    assert size(_batch(kfscan, nmodels=100)) == 0 and n.value > shared   # a model per sequence
    assert size(_batch(kfscan, nmodels=7)) == 1          # neither shared nor one per sequence
    assert size(_batch(kfscan, nseq=0)) == 1
    assert size(_batch(kfscan, nseq=(1 << 22) + 1)) == 1
    assert size(_batch(kfscan, total=0)) == 1
    assert size(_batch(kfscan, nx=5)) == 2
    assert size(_batch(kfscan, scan=2)) == 2            # tree scans are not offered for batches
    assert size(_batch(kfscan, prec=9)) == 1
    assert lib.kf_batch_workspace_size(None, ctypes.byref(n)) == 1


def test_batch_entry_points_reject_before_launch(kfscan):
    lib = kfscan.load_library()
    b = _batch(kfscan)
    for name in ("kf_filter_batch", "kf_smooth_rts_batch", "kf_smooth_twofilter_batch"):
        assert getattr(lib, name)(ctypes.byref(b), None, 0, None) == 1   # null pointers
    for f in ("F", "Q", "H", "R", "m0", "P0", "y", "m_filt", "P_filt", "m_smooth", "P_smooth"):
        setattr(b, f, 4096)
    assert lib.kf_filter_batch(ctypes.byref(b), None, 0, None) == 1      # T, offset still null
    b.T, b.offset = 4096, 8192
    assert lib.kf_filter_batch(ctypes.byref(b), None, 0, None) == 3      # no workspace
    status = ctypes.c_uint32(0)
    assert lib.kf_workspace_status(None, 0, ctypes.byref(status), None) == 3


def test_tv_workspace_size_and_validation(kfscan):
    lib = kfscan.load_library()
    n = ctypes.c_size_t(0)

    def tvp(**kw):
        p = kfscan.KfTvProblem()
        p.nx, p.ny, p.precision, p.scan = kw.get("nx", 4), 2, kw.get("prec", 1), kw.get("scan", 0)
        p.T, p.nseq = kw.get("T", 1 << 16), kw.get("nseq", 1)
        return p
    size = lambda p: lib.kf_tv_workspace_size(ctypes.byref(p), ctypes.byref(n))  # noqa: E731
    assert size(tvp()) == 0 and n.value > 0
    assert size(tvp(T=0)) == 1
    assert size(tvp(nx=5)) == 2
    assert size(tvp(scan=3)) == 0          # tree scans serve time-varying models too
    assert size(tvp(scan=3, nseq=70000)) == 2
    assert size(tvp(scan=6, T=(1 << 36) + 1)) == 2
    p = tvp(T=100)
    for name in ("kf_filter_tv", "kf_smooth_rts_tv", "kf_smooth_twofilter_tv"):
        assert getattr(lib, name)(ctypes.byref(p), None, 0, None) == 1   # null pointers


def test_sequential_workspace_is_one_line_of_control_words(kfscan):
    """KF_SCAN_SEQUENTIAL needs only the error words, for every entry kind,
    whatever the length; scan values past it are refused."""
    lib = kfscan.load_library()
    n = ctypes.c_size_t(0)
    seq = kfscan.SCANS["sequential"]
    assert seq == 5
    for T, nseq in ((1, 1), (1 << 30, 1), (1000, 1 << 20)):
        assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, T=T, nseq=nseq, scan=seq)),
                                     ctypes.byref(n)) == 0
        assert n.value == 256
    assert lib.kf_batch_workspace_size(ctypes.byref(_batch(kfscan, scan=seq, nmodels=100)),
                                       ctypes.byref(n)) == 0
    assert n.value == 256
    p = kfscan.KfTvProblem()
    p.nx, p.ny, p.precision, p.scan, p.T, p.nseq = 4, 2, 1, seq, 1 << 20, 1
    assert lib.kf_tv_workspace_size(ctypes.byref(p), ctypes.byref(n)) == 0
    assert n.value == 256
    assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, scan=9)), ctypes.byref(n)) == 1


def test_tree_scan_workspace_sizes(kfscan):
    """Element arrays in the workspace: Blelloch and Ladner-Fischer one padded
    array, Hillis-Steele two of T positions, Sengupta two padded ones."""
    lib = kfscan.load_library()
    n = ctypes.c_size_t(0)

    def size(scan, T):
        assert lib.kf_workspace_size(ctypes.byref(_problem(kfscan, T=T, scan=kfscan.SCANS[scan])),
                                     ctypes.byref(n)) == 0
        return n.value
    T = 100000
    base = size("lookback_generic", T)
    one = (3 * 16 + 2 * 4) * 4                             # FP32 filtering element, nx = 4
    assert size("ladner_fischer", T) - base >= one * (1 << 17)
    assert size("blelloch", T) == size("ladner_fischer", T)
    assert size("sengupta_a", T) - base >= 2 * one * (1 << 17)
    assert size("sengupta_b", T) == size("sengupta_a", T)
    assert size("hillis_steele", T) - base >= 2 * one * T


def _oracle_counts(name, T, N=None):
    """Operator applications of the oracle's scan over T elements (a cheap
    associative operator; only the count matters here)."""
    from oracle import scans
    cnt = [0]

    def op(x, y):
        cnt[0] += 1
        return x + y
    if name == "sengupta":
        scans.sengupta(list(range(T)), op, 0, N=N)
    else:
        scans.ALL[name](list(range(T)), op, 0)
    return cnt[0]


@pytest.mark.parametrize("T", [1, 2, 3, 8, 100, 1024, 5000, 1 << 15, 100000])
def test_scan_counts_match_the_oracle_algorithms(kfscan, T):
    """kf_scan_counts, read off the launch plan, equals the number of operator
    applications of the oracle's Algorithms 1-4 on the same length (both
    Blelloch versions finish only the T real positions in their last pass)."""
    assert kfscan.scan_counts("hillis_steele", T)[0] == _oracle_counts("hillis_steele", T)
    assert kfscan.scan_counts("ladner_fischer", T)[0] == _oracle_counts("ladner_fischer", T)
    assert kfscan.scan_counts("sengupta_a", T)[0] == _oracle_counts("sengupta", T, 1)
    assert kfscan.scan_counts("sengupta_b", T)[0] == _oracle_counts("sengupta", T, 16384)
    assert kfscan.scan_counts("blelloch", T)[0] == _oracle_counts("blelloch", T)


@pytest.mark.parametrize("T", [2, 16, 1024, 1 << 20])
def test_scan_steps_and_work(kfscan, T):
    """Span and work of Sec. II for T a power of two: Hillis-Steele log2 T
    steps and T log2 T - T + 1 applications; Blelloch 2 log2 T + 1 steps
    (with the final pass) and 3T - 2; in-place Ladner-Fischer two steps fewer,
    2 log2 T - 1, and 2T - 2 - log2 T, which Sengupta A matches."""
    lg = T.bit_length() - 1
    assert kfscan.scan_counts("hillis_steele", T) == (T * lg - T + 1, lg)
    assert kfscan.scan_counts("blelloch", T) == (3 * T - 2, 2 * lg + 1)
    assert kfscan.scan_counts("ladner_fischer", T) == (2 * T - 2 - lg, 2 * lg - 1)
    assert kfscan.scan_counts("sengupta_a", T) == (2 * T - 2 - lg, 2 * lg - 1)
    N = min(T, 16384)
    dstar = (T // N).bit_length() - 1
    want = 2 * (T - N) - dstar + N * (N.bit_length() - 1) - N + 1
    assert kfscan.scan_counts("sengupta_b", T)[0] == want


def test_scan_counts_refuse_other_scans(kfscan):
    lib = kfscan.load_library()
    c, n = ctypes.c_int64(0), ctypes.c_int64(0)
    for scan in ("auto", "lookback", "lookback_generic", "sequential"):
        assert lib.kf_scan_counts(kfscan.SCANS[scan], 1000, ctypes.byref(c), ctypes.byref(n)) == 2
    assert lib.kf_scan_counts(kfscan.SCANS["blelloch"], 0, ctypes.byref(c), ctypes.byref(n)) == 1
    assert lib.kf_scan_counts(9, 10, ctypes.byref(c), ctypes.byref(n)) == 1
