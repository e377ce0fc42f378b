"""Scan algorithms of Sec. II (oracle.scans) with an exact non-commutative operator.

Elements are 2x2 integer matrices modulo 2^31-1 under matrix product: associative,
not commutative, exact.  Every algorithm must reproduce the sequential
definition bit for bit, forward and reversed, for any T (padding with the
identity when T is not a power of two), and must use the number of operator
applications its work complexity predicts (Sec. II-C..F, derived counts:
Hillis-Steele T log2 T - T + 1, Blelloch 3T - 2 including the identity
applications, in-place Ladner-Fischer and Sengupta with N = 1 2T - 2 - log2 T).
"""
import math

import numpy as np
import pytest

from oracle import scans

MOD = 2 ** 31 - 1
IDENT = ((1, 0), (0, 1))


def mat_op(x, y):
    return (((x[0][0] * y[0][0] + x[0][1] * y[1][0]) % MOD, (x[0][0] * y[0][1] + x[0][1] * y[1][1]) % MOD),
            ((x[1][0] * y[0][0] + x[1][1] * y[1][0]) % MOD, (x[1][0] * y[0][1] + x[1][1] * y[1][1]) % MOD))


def _elems(T, seed):
    rng = np.random.default_rng(seed)
    v = rng.integers(0, 1000, size=(T, 2, 2))
    return [tuple(tuple(int(c) for c in row) for row in m) for m in v]


def _counting(op):
    cnt = [0]

    def f(x, y):
        cnt[0] += 1
        return op(x, y)
    return f, cnt


ALGS = ["hillis_steele", "blelloch", "ladner_fischer", "sengupta_a", "sengupta_b4"]


@pytest.mark.parametrize("name", ALGS)
@pytest.mark.parametrize("T", [1, 2, 3, 5, 8, 13, 16, 31, 64, 100])
def test_scan_exact(name, T):
    a = _elems(T, T)
    ref = scans.sequential(a, mat_op)
    assert scans.ALL[name](a, mat_op, IDENT) == ref
    rref = [None] * T
    acc = None
    for k in range(T - 1, -1, -1):
        acc = a[k] if acc is None else mat_op(a[k], acc)
        rref[k] = acc
    assert scans.reverse(scans.ALL[name])(a, mat_op, IDENT) == rref


@pytest.mark.parametrize("T", [8, 16, 1024])
def test_combine_counts(T):
    lg = int(math.log2(T))
    expect = {
        "hillis_steele": T * lg - T + 1,
        "blelloch": 3 * T - 2,
        "ladner_fischer": 2 * T - 2 - lg,
        "sengupta_a": 2 * T - 2 - lg,
    }
    a = _elems(T, 1)
    for name, want in expect.items():
        op, cnt = _counting(mat_op)
        scans.ALL[name](a, op, IDENT)
        assert cnt[0] == want, (name, cnt[0], want)


def test_sengupta_general_threshold_count():
    """Sengupta with threshold N: 2(T-N) - log2(T/N) reduce/down-sweep combines
    plus N log2 N - N + 1 for Hillis-Steele on the top level."""
    T, N = 256, 16
    a = _elems(T, 2)
    op, cnt = _counting(mat_op)
    out = scans.sengupta(a, op, IDENT, N=N)
    assert out == scans.sequential(a, mat_op)
    assert cnt[0] == 2 * (T - N) - int(math.log2(T // N)) + N * int(math.log2(N)) - N + 1
