"""Exact host scans of the affine maps of kf_selftest_scan (test helper).

An element is (A, b, C) with A, C in Z_p^{2x2}, b in Z_p^2, stored as the 10
numbers A00 A01 A10 A11 b0 b1 C00 C01 C10 C11.  "i then j" composes to
(A_j A_i, A_j b_i + b_j, A_j C_i + C_j).  The forward result at row k is
a_0 then ... then a_k, the reverse one a_{T-1} then ... then a_k; each row
keeps (b, C), 6 numbers.  Arithmetic is in Python / int64 integers, exact.
"""
from __future__ import annotations

import numpy as np


def _split(e):
    A = e[..., 0:4].reshape(e.shape[:-1] + (2, 2))
    b = e[..., 4:6]
    C = e[..., 6:10].reshape(e.shape[:-1] + (2, 2))
    return A, b, C


def sequential(elems: np.ndarray, p: int, reverse: bool = False) -> np.ndarray:
    """Plain loop over the rows of one sequence [T, 10] (pure Python integers)."""
    T = elems.shape[0]
    rows = [[int(v) for v in r] for r in elems]
    out = np.zeros((T, 6), dtype=np.int64)
    v = [0, 0]
    M = [[0, 0], [0, 0]]
    order = range(T - 1, -1, -1) if reverse else range(T)
    for k in order:
        r = rows[k]
        A = [[r[0], r[1]], [r[2], r[3]]]
        v = [(A[0][0] * v[0] + A[0][1] * v[1] + r[4]) % p,
             (A[1][0] * v[0] + A[1][1] * v[1] + r[5]) % p]
        C = [[r[6], r[7]], [r[8], r[9]]]
        M = [[(A[i][0] * M[0][j] + A[i][1] * M[1][j] + C[i][j]) % p for j in range(2)]
             for i in range(2)]
        out[k] = [v[0], v[1], M[0][0], M[0][1], M[1][0], M[1][1]]
    return out


def doubling(elems: np.ndarray, p: int, reverse: bool = False) -> np.ndarray:
    """The same result by recursive doubling over [nseq, T, 10] in int64 (every
    intermediate is below 2 p^2 + p < 2^63 for p < 2^30)."""
    e = np.asarray(elems, dtype=np.int64)
    if reverse:
        e = e[:, ::-1]
    A, b, C = (x.copy() for x in _split(e))
    T = e.shape[1]
    s = 1
    while s < T:
        # row k := row k-s then row k (for k >= s)
        Ai, bi, Ci = A[:, :-s], b[:, :-s], C[:, :-s]
        Aj, bj, Cj = A[:, s:], b[:, s:], C[:, s:]
        nA = np.einsum("nkij,nkjl->nkil", Aj, Ai) % p
        nb = (np.einsum("nkij,nkj->nki", Aj, bi) + bj) % p
        nC = (np.einsum("nkij,nkjl->nkil", Aj, Ci) + Cj) % p
        A[:, s:], b[:, s:], C[:, s:] = nA, nb, nC
        s *= 2
    out = np.concatenate([b, C.reshape(C.shape[:-2] + (4,))], axis=-1)
    return out[:, ::-1] if reverse else out


def random_elements(rng, nseq: int, T: int, p: int, anchor_rate: float = 0.0,
                    reverse: bool = False) -> np.ndarray:
    """Uniform elements below p; the first (forward) or last (reverse) of each
    sequence, and a fraction anchor_rate of the others, get A = 0."""
    e = rng.integers(0, p, size=(nseq, T, 10), dtype=np.int64)
    if anchor_rate > 0:
        mask = rng.random((nseq, T)) < anchor_rate
        e[mask, 0:4] = 0
    e[:, T - 1 if reverse else 0, 0:4] = 0
    return e
