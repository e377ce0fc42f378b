"""All-prefix-sum (scan) algorithms of Sec. II, written plainly over Python lists.

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Every function takes ``(a, op, identity)`` -- a list of elements a_1..a_T, an
associative (not necessarily commutative) operator ``op(x, y) = x (x) y`` and
its two-sided identity -- and returns a new list with the inclusive prefix sums
s_k = a_1 (x) ... (x) a_k (Sec. II-B).  ``identity`` pads a series whose length is
not a power of two, which the paper's algorithms assume (Sec. II opening).

* ``sequential``      -- the definition: one left-to-right loop.
* ``hillis_steele``   -- Algorithm 1.  Reading C13: the level loop runs for
                         d = 0..log2(T)-1 (the last iteration of the printed
                         range does nothing).
* ``blelloch``        -- Algorithm 2 (up-sweep, zero the root, down-sweep,
                         final pass with the saved input).
* ``ladner_fischer``  -- Algorithm 3 (in place, inclusive).
* ``sengupta``        -- Algorithm 4 with threshold ``N`` (N = 1 is "Sengupta A").
* ``reverse(scan)``   -- the reversed all-prefix-sums s_k = a_k (x) ... (x) a_T of
                         Sec. II-B, by reversing the series and swapping the
                         operands of the operator (reading C5), so the left
                         operand always stays the earlier one in time.
"""
from __future__ import annotations


def _pow2_at_least(T: int) -> int:
    p = 1
    while p < T:
        p *= 2
    return p


def _log2(p: int) -> int:
    return p.bit_length() - 1


def sequential(a, op, identity=None):
    out = []
    acc = None
    for x in a:
        acc = x if acc is None else op(acc, x)
        out.append(acc)
    return out


def hillis_steele(a, op, identity=None):
    """Algorithm 1.  Works for any T (no padding needed)."""
    T = len(a)
    cur = list(a)
    step = 1
    while step < T:
        prev = list(cur)                    # b <- copy(a)
        for i in range(0, T - step):        # 0-based: i = 1..T-2^d in the paper
            j = i + step
            cur[j] = op(prev[i], prev[j])
        step *= 2
    return cur


def blelloch(a, op, identity):
    """Algorithm 2 on the series padded with ``identity`` to a power of two."""
    T = len(a)
    if T == 0:
        return []
    P = _pow2_at_least(T)
    x = [None] + list(a) + [identity] * (P - T)      # 1-based storage x[1..P]
    saved = list(x)                                   # b <- copy(a)
    D = _log2(P)
    for d in range(D):                                # up-sweep
        for i in range(0, P, 2 ** (d + 1)):
            j, k = i + 2 ** d, i + 2 ** (d + 1)
            x[k] = op(x[j], x[k])
    x[P] = identity                                   # a_T <- neutral element
    for d in range(D - 1, -1, -1):                    # down-sweep
        for i in range(0, P, 2 ** (d + 1)):
            j, k = i + 2 ** d, i + 2 ** (d + 1)
            t = x[j]
            x[j] = x[k]
            x[k] = op(x[k], t)
    for i in range(1, P + 1):                         # final pass: exclusive -> inclusive
        x[i] = op(x[i], saved[i])
    return x[1:T + 1]


def ladner_fischer(a, op, identity):
    """Algorithm 3 (in-place Ladner-Fischer) on the padded series."""
    T = len(a)
    if T == 0:
        return []
    P = _pow2_at_least(T)
    x = [None] + list(a) + [identity] * (P - T)
    D = _log2(P)
    for d in range(D):                                # up-sweep
        for i in range(0, P, 2 ** (d + 1)):
            j, k = i + 2 ** d, i + 2 ** (d + 1)
            x[k] = op(x[j], x[k])
    for d in range(D - 1, -1, -1):                    # down-sweep
        for i in range(2 ** (d + 1), P, 2 ** (d + 1)):
            j = i + 2 ** d
            x[j] = op(x[i], x[j])
    return x[1:T + 1]


def sengupta(a, op, identity, N=1):
    """Algorithm 4: reduce levels up to a series of length N, Hillis-Steele on
    that level, then the down-sweep.  ``N`` is rounded to a power of two in
    [1, padded T]."""
    T = len(a)
    if T == 0:
        return []
    P = _pow2_at_least(T)
    N = min(_pow2_at_least(max(1, int(N))), P)
    dstar = _log2(P // N)
    levels = [[None] + list(a) + [identity] * (P - T)]   # a^(0), 1-based
    for d in range(1, dstar + 1):                        # reduce passes
        prev = levels[d - 1]
        cur = [None] * (P // 2 ** d + 1)
        for i in range(1, P // 2 ** d + 1):
            cur[i] = op(prev[2 * i - 1], prev[2 * i])
        levels.append(cur)
    top = levels[dstar]
    levels[dstar] = [None] + hillis_steele(top[1:], op)  # scan of the top level
    for d in range(dstar - 1, -1, -1):                   # down-sweep
        cur, up = levels[d], levels[d + 1]
        for i in range(1, P // 2 ** d + 1):
            if i > 1:
                if i % 2 == 1:
                    cur[i] = op(up[(i - 1) // 2], cur[i])
                else:
                    cur[i] = up[i // 2]
    return levels[0][1:T + 1]


def reverse(scan):
    """Turn a forward scan into the reversed all-prefix-sums of Sec. II-B."""
    def rscan(a, op, identity=None):
        swapped = lambda x, y: op(y, x)                  # noqa: E731
        return list(reversed(scan(list(reversed(a)), swapped, identity)))
    rscan.__name__ = "reverse_" + getattr(scan, "__name__", "scan")
    return rscan


ALL = {
    "sequential": sequential,
    "hillis_steele": hillis_steele,
    "blelloch": blelloch,
    "ladner_fischer": ladner_fischer,
    "sengupta_a": lambda a, op, identity: sengupta(a, op, identity, N=1),
    "sengupta_b4": lambda a, op, identity: sengupta(a, op, identity, N=4),
}
