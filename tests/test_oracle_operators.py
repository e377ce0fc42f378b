"""Pins of the oracle's parallel-form pieces (Sec. IV): elements, operators and
Algorithms 5-7, against the sequential recursions (themselves pinned by brute
force in test_oracle_pins) and against the algebra the paper states:
associativity (Lemmas 1/2), the identity element (reading C3), the split
identity s_T = s_{k-1} (x) sbar_k (Sec. II-B), and the irrelevance of eta_1, J_1
(reading C4)."""
import numpy as np
import pytest

import oracle
from oracle import scans
import kf_workloads as W
from tests.test_oracle_pins import _rand_model, _close


def _random_filter_element(rng, n):
    """A valid filtering element: an aggregate of a few random model steps."""
    F, Q, H, R, m0, P0, u, d = _rand_model(rng, n, max(1, n // 2), tv=True, T=4, inputs=True)
    y = rng.standard_normal((4, H.shape[1]))
    el = oracle.filter_elements(F, Q, H, R, m0, P0, y, u, d)[1:]
    acc = el[0]
    for e in el[1:]:
        acc = oracle.filter_combine(acc, e)
    return acc


@pytest.mark.parametrize("n", [1, 2, 4])
def test_filter_operator_associative_and_identity(n):
    rng = np.random.default_rng(40 + n)
    a, b, c = (_random_filter_element(rng, n) for _ in range(3))
    left = oracle.filter_combine(oracle.filter_combine(a, b), c)
    right = oracle.filter_combine(a, oracle.filter_combine(b, c))
    for x, y in zip(left, right):
        _close(x, y, 1e-11)
    e = oracle.filter_identity(n)
    for x, y in zip(oracle.filter_combine(e, a), a):
        _close(x, y, 1e-14)
    for x, y in zip(oracle.filter_combine(a, e), a):
        _close(x, y, 1e-14)


@pytest.mark.parametrize("n", [2, 3, 4, 6])
def test_filter_operator_associative_on_wild_elements(n):
    """Random full-rank PSD C, J force pivoting in the (I + C_i J_j) solves."""
    from tests.test_oracle_mutants import wild_filter_element
    rng = np.random.default_rng(60 + n)
    for _ in range(5):
        a, b, c = (wild_filter_element(rng, n) for _ in range(3))
        left = oracle.filter_combine(oracle.filter_combine(a, b), c)
        right = oracle.filter_combine(a, oracle.filter_combine(b, c))
        for x, y in zip(left, right):
            _close(x, y, 1e-10)


def test_all_zero_element_is_only_a_right_neutral_for_eta_J():
    """Reading C3: the paper's e = (0,0,0,0,0) leaves eta, J unchanged as a right
    operand, but it is not a left identity."""
    rng = np.random.default_rng(5)
    a = _random_filter_element(rng, 3)
    z = tuple(np.zeros_like(np.asarray(p)) for p in a)
    r = oracle.filter_combine(a, z)
    _close(r[3], a[3], 1e-14); _close(r[4], a[4], 1e-14)
    l = oracle.filter_combine(z, a)
    assert np.max(np.abs(l[4])) == 0.0 and np.max(np.abs(a[4])) > 0.0


def test_smooth_operator_associative_and_identity():
    rng = np.random.default_rng(9)
    mdl, y = W.tracking(40, seed=3)
    m_f, P_f, _, _ = oracle.kf_filter(*mdl.arrays(), y)
    el = oracle.smooth_elements(mdl.F, mdl.Q, m_f, P_f)
    a, b, c = el[3], el[17], el[39]
    left = oracle.smooth_combine(oracle.smooth_combine(a, b), c)
    right = oracle.smooth_combine(a, oracle.smooth_combine(b, c))
    for x, y2 in zip(left, right):
        _close(x, y2, 1e-13)
    e = oracle.smooth_identity(4)
    for x, y2 in zip(oracle.smooth_combine(e, a), a):
        _close(x, y2, 1e-15)
    del rng


@pytest.mark.parametrize("tv,inputs", [(False, False), (True, True)])
def test_fold_equals_sequential(tv, inputs):
    """Algorithms 5-7 with a sequential scan reproduce the sequential filter,
    RTS and two-filter smoothers."""
    rng = np.random.default_rng(50)
    T = 60
    F, Q, H, R, m0, P0, u, d = _rand_model(rng, 4, 2, tv=tv, T=T, inputs=inputs)
    y = rng.standard_normal((T, 2))
    ref = oracle.smooth_rts(F, Q, H, R, m0, P0, y, u, d)
    m_f, P_f = oracle.pkf(F, Q, H, R, m0, P0, y, u, d)
    _close(m_f, ref[0], 1e-10); _close(P_f, ref[1], 1e-10)
    p = oracle.prts(F, Q, H, R, m0, P0, y, u, d)
    _close(p[2], ref[2], 1e-9); _close(p[3], ref[3], 1e-9)
    t = oracle.ptfs(F, Q, H, R, m0, P0, y, u, d)
    _close(t[2], ref[2], 1e-9); _close(t[3], ref[3], 1e-9)
    z = tuple(np.zeros_like(np.asarray(x)) for x in oracle.filter_identity(4))
    t0 = oracle.ptfs(F, Q, H, R, m0, P0, y, u, d, right_neutral=z)
    _close(t0[2], ref[2], 1e-9)


@pytest.mark.parametrize("name", ["hillis_steele", "blelloch", "ladner_fischer", "sengupta_a",
                                  "sengupta_b4"])
def test_paper_scans_on_kalman_elements(name):
    """Each scan of Sec. II gives the same filter/smoother as the fold (T not a power of 2)."""
    mdl, y = W.tracking(37, seed=8)
    scan = scans.ALL[name]
    ref = oracle.smooth_rts(*mdl.arrays(), y)
    r = oracle.prts(*mdl.arrays(), y, scan=scan)
    for a, b in zip(r, ref):
        _close(a, b, 1e-9)
    t = oracle.ptfs(*mdl.arrays(), y, scan=scan)
    _close(t[2], ref[2], 1e-9); _close(t[3], ref[3], 1e-9)


def test_split_identity_forward_backward():
    """s_T = s_{k-1} (x) sbar_k for every k (Sec. II-B) on filtering elements."""
    mdl, y = W.tracking(30, seed=4)
    el = oracle.filter_elements(*mdl.arrays(), y)
    ident = oracle.filter_identity(4)
    fwd = scans.sequential(el, oracle.filter_combine, ident)
    bwd = scans.reverse(scans.sequential)(el, oracle.filter_combine, ident)
    for k in range(1, 30):
        s = oracle.filter_combine(fwd[k - 1], bwd[k])
        _close(s[1], fwd[-1][1], 1e-9)
        _close(s[2], fwd[-1][2], 1e-9)


def test_eta1_J1_do_not_matter():
    """Reading C4: A_1 = 0, so randomising eta_1 and J_1 changes no filter output."""
    mdl, y = W.tracking(25, seed=6)
    el = oracle.filter_elements(*mdl.arrays(), y)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((4, 4))
    el2 = [(el[0][0], el[0][1], el[0][2], rng.standard_normal(4), X @ X.T)] + el[1:]
    ident = oracle.filter_identity(4)
    a = scans.sequential(el, oracle.filter_combine, ident)
    b = scans.sequential(el2, oracle.filter_combine, ident)
    for s1, s2 in zip(a, b):
        assert np.array_equal(s1[1], s2[1]) and np.array_equal(s1[2], s2[2])


@pytest.mark.parametrize("n", [2, 4])
def test_zero_decay_element_is_an_anchor(n):
    """Lemmas 1 and 2: an element whose decay matrix (A, resp. E) is exactly
    zero fixes the anchored part of every product it takes part in -- (b, C) of
    p (x) x and (eta, J) of x (x) q for filtering elements, (g, L) of x (x) q for
    smoothing elements -- whatever the other operand.  The first filtering
    element (A_1 = 0, eq. pkf_init2) and the last smoothing element (E_T = 0,
    eq. prts_init2) are such anchors; the GPU look-back also stops at any
    aggregate whose decay matrix has underflowed to zero."""
    rng = np.random.default_rng(70 + n)
    for _ in range(4):
        p, q, x = (_random_filter_element(rng, n) for _ in range(3))
        x = (np.zeros((n, n)),) + tuple(x[1:])
        r = oracle.filter_combine(p, x)
        assert np.array_equal(r[1], x[1]) and np.array_equal(r[2], x[2])
        r = oracle.filter_combine(x, q)
        assert np.array_equal(r[3], x[3]) and np.array_equal(r[4], x[4])
        # the product keeps a zero decay matrix (it stays an anchor)
        assert np.array_equal(oracle.filter_combine(p, x)[0], np.zeros((n, n)))
    F, Q, H, R, m0, P0, u, d = _rand_model(rng, n, 1, tv=False, T=6, inputs=False)
    y = rng.standard_normal((6, 1))
    m_f, P_f, _, _ = oracle.kf_filter(F, Q, H, R, m0, P0, y)
    el = oracle.smooth_elements(F, Q, m_f, P_f)
    for k in range(5):
        xs = (np.zeros((n, n)),) + tuple(el[k][1:])
        r = oracle.smooth_combine(xs, el[k + 1])
        assert np.array_equal(r[1], xs[1]) and np.array_equal(r[2], xs[2])
