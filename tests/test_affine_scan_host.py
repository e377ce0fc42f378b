"""The exact host scans used as expected values by the scan-skeleton GPU test
agree with each other (plain loop against recursive doubling) and with
hand-computed compositions."""
import numpy as np

from tests import affine_scan as S


def test_two_elements_by_hand():
    p = 101
    # a0 = (A=0, b=(3,4), C=[[1,2],[3,4]]), a1 = (A=[[2,0],[1,1]], b=(5,6), C=I)
    e = np.array([[[0, 0, 0, 0, 3, 4, 1, 2, 3, 4],
                   [2, 0, 1, 1, 5, 6, 1, 0, 0, 1]]], dtype=np.int64)
    fwd = S.sequential(e[0], p)
    assert fwd[0].tolist() == [3, 4, 1, 2, 3, 4]
    # a0 then a1: b = A1 (3,4) + (5,6) = (11, 13); C = A1 [[1,2],[3,4]] + I = [[3,4],[4,7]]
    assert fwd[1].tolist() == [11, 13, 3, 4, 4, 7]
    e[0, 0, 0:4] = [1, 1, 0, 1]
    e[0, 1, 0:4] = 0
    rev = S.sequential(e[0], p, reverse=True)
    assert rev[1].tolist() == [5, 6, 1, 0, 0, 1]
    # a1 then a0: b = A0 (5,6) + (3,4) = (14, 10); C = A0 I + C0 = [[2,3],[3,5]]
    assert rev[0].tolist() == [14, 10, 2, 3, 3, 5]


def test_operator_is_not_commutative():
    p = 33554393
    rng = np.random.default_rng(3)
    e = S.random_elements(rng, 1, 2, p)
    e[0, 0, 0:4] = rng.integers(1, p, 4)
    ab = S.sequential(e[0], p)[1]
    ba = S.sequential(e[0, ::-1].copy(), p)[1]
    assert not np.array_equal(ab, ba)


def test_doubling_matches_loop():
    rng = np.random.default_rng(7)
    for p in (2039, 33554393):
        for rev in (False, True):
            for rate in (0.0, 0.05):
                e = S.random_elements(rng, 3, 777, p, anchor_rate=rate, reverse=rev)
                want = np.stack([S.sequential(e[i], p, reverse=rev) for i in range(3)])
                got = S.doubling(e, p, reverse=rev)
                assert np.array_equal(got, want)


def test_anchor_cuts_the_prefix():
    p = 2039
    rng = np.random.default_rng(11)
    e = S.random_elements(rng, 1, 50, p)
    e[0, 20, 0:4] = 0
    full = S.sequential(e[0], p)
    tail = S.sequential(e[0, 20:].copy(), p)
    assert np.array_equal(full[20:], tail)
