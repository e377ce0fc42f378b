"""All-prefix-sum (scan) algorithms of Sec. II, written plainly over Python lists.

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Every function takes ``(a, op, identity)`` -- a list of elements a_1..a_T, an
associative (not necessarily commutative) operator ``op(x, y) = x (x) y`` and
its two-sided identity -- and returns a new list with the inclusive prefix sums
s_k = a_1 (x) ... (x) a_k (Sec. II-B).  ``identity`` pads a series whose length is
not a power of two, which the paper's algorithms assume (Sec. II opening).

* ``sequential``      -- the definition: one left-to-right loop.
* ``hillis_steele``   -- Algorithm 1.  Reading C13: log2(T) rounds, distances
                         1, 2, .., 2^(log2(T)-1) (a round at distance T would do
                         nothing).
* ``blelloch``        -- Algorithm 2 (pairwise reduction, the exclusive prefix
                         pushed down the tree from the identity at the root, a
                         last inclusive pass).
* ``ladner_fischer``  -- Algorithm 3 (in place, inclusive: pairwise reduction,
                         then each block total completed with the prefix that
                         ends where the block begins).
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


def sequential(a, op, identity=None):
    out = []
    acc = None
    for x in a:
        acc = x if acc is None else op(acc, x)
        out.append(acc)
    return out


def hillis_steele(a, op, identity=None):
    """Algorithm 1: log2(T) rounds; in the round with distance s every
    position j >= s combines the value s places before it with its own, both
    taken from the previous round.  Works for any T (no padding needed)."""
    cur = list(a)
    s = 1
    while s < len(cur):
        cur = cur[:s] + [op(cur[j - s], cur[j]) for j in range(s, len(cur))]
        s *= 2
    return cur


def _padded(a, identity):
    return list(a) + [identity] * (_pow2_at_least(len(a)) - len(a))


def _block_totals(x, op):
    """Totals of the dyadic blocks of the power-of-two series x, found by
    pairwise reduction (the up-sweep shared by Algorithms 2 and 3): a dict
    {(lo, hi): x[lo] (x) ... (x) x[hi-1]} over the nodes of the balanced binary
    tree on [0, len(x)).  One operator application per inner node."""
    tot = {}

    def node(lo, hi):
        if hi - lo == 1:
            v = x[lo]
        else:
            mid = (lo + hi) // 2
            v = op(node(lo, mid), node(mid, hi))
        tot[(lo, hi)] = v
        return v

    node(0, len(x))
    return tot


def blelloch(a, op, identity):
    """Algorithm 2 on the series padded with ``identity`` to a power of two.

    After the pairwise reduction, the exclusive prefix is pushed down the
    tree: a node that receives the prefix c of everything before it hands c to
    its left child and c (x) (left child's total) to its right child, starting
    from the identity at the root.  A last pass turns the exclusive prefix of
    each position into the inclusive one."""
    T = len(a)
    if T == 0:
        return []
    x = _padded(a, identity)
    tot = _block_totals(x, op)
    excl = [None] * len(x)

    def push(lo, hi, c):
        if hi - lo == 1:
            excl[lo] = c
            return
        mid = (lo + hi) // 2
        push(lo, mid, c)
        push(mid, hi, op(c, tot[(lo, mid)]))

    push(0, len(x), identity)
    return [op(excl[i], x[i]) for i in range(T)]


def ladner_fischer(a, op, identity):
    """Algorithm 3 (in-place Ladner-Fischer) on the padded series.

    After the pairwise reduction, position k (1-based) holds the total of the
    dyadic block that ends at k and has the length of k's lowest set bit.
    That is already the inclusive prefix when the block starts at 1 (k a power
    of two); every other position needs the inclusive prefix that ends where
    its block begins, combined on the left, and that position is finished
    earlier because it lies at a smaller index."""
    T = len(a)
    if T == 0:
        return []
    x = _padded(a, identity)
    tot = _block_totals(x, op)
    out = [None] * (len(x) + 1)          # out[k]: inclusive prefix ending at k (1-based)
    for k in range(1, len(x) + 1):
        width = k & -k
        own = tot[(k - width, k)]
        out[k] = own if k == width else op(out[k - width], own)
    return out[1:T + 1]


def sengupta(a, op, identity, N=1):
    """Algorithm 4: pairwise reduction until at most N elements remain, the
    Hillis-Steele scan on those, then expansion level by level.  ``N`` is
    rounded to a power of two in [1, padded T].

    Expansion of one level: with S the inclusive scan of the pairs
    (x_0 (x) x_1, x_2 (x) x_3, ...), the prefix at the second element of pair i
    is S_i, and at the first element it is S_{i-1} (x) x_{2i} (x_0 alone for
    i = 0)."""
    T = len(a)
    if T == 0:
        return []
    x = _padded(a, identity)
    N = min(_pow2_at_least(max(1, int(N))), len(x))

    def scan_level(v):
        if len(v) <= N:
            return hillis_steele(v, op)
        S = scan_level([op(v[2 * i], v[2 * i + 1]) for i in range(len(v) // 2)])
        out = []
        for i, s in enumerate(S):
            out.append(v[0] if i == 0 else op(S[i - 1], v[2 * i]))
            out.append(s)
        return out

    return scan_level(x)[:T]


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
