"""One cumulant element at a time, straight from a window (oracle helper,
test infrastructure only).

``cumulant_at(W, idx)`` follows Alg. 4 for a single multi-index: the raw
moment of Eq. (mom) minus, over every partition of the positions into two or
more parts, the product of the lower-order cumulants at the sub-multi-indices
(computed the same way, memoised by their sorted index).  Moments are means
of row products over the window ``W`` in FP64 (numpy's pairwise summation).
Used to check full-size runs on sampled outputs.
"""
from __future__ import annotations

import numpy as np


def partitions(items):
    """Set partitions of a list: insert the first item into each part of every
    partition of the rest, or give it a part of its own."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in partitions(rest):
        yield [[first]] + p
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]


def moment_at(W: np.ndarray, idx) -> float:
    prod = np.ones(W.shape[0])
    for i in idx:
        prod = prod * W[:, i]
    return float(np.mean(prod))


def cumulant_at(W: np.ndarray, idx, cache=None) -> float:
    if cache is None:
        cache = {}
    key = tuple(sorted(int(i) for i in idx))
    if key in cache:
        return cache[key]
    m = moment_at(W, key)
    A = 0.0
    for pi in partitions(list(range(len(key)))):
        if len(pi) < 2:
            continue
        prod = 1.0
        for part in pi:
            prod *= cumulant_at(W, [key[q] for q in part], cache)
        A += prod
    cache[key] = m - A
    return cache[key]


def sample_elements(n: int, b: int, k: int, count: int, rng) -> tuple:
    """(pyramid offsets, global multi-indices) of `count` random stored
    order-k elements whose indices are all < n (no padding)."""
    from . import tuples

    tl = tuples(n, b, k)
    offs, idxs = [], []
    while len(offs) < count:
        r = int(rng.integers(len(tl)))
        a = [int(v) for v in rng.integers(0, b, size=k)]
        idx = [int(j) * b + am for j, am in zip(tl[r], a)]
        if max(idx) >= n:
            continue
        e = 0
        for am in a:
            e = e * b + am
        offs.append(r * b ** k + e)
        idxs.append(idx)
    return np.array(offs), idxs


def indices_of(n: int, b: int, k: int, offs) -> list:
    """Global multi-index of each stored order-k element at the pyramid
    offsets `offs` (block r = off // b^k in lexicographic order, within-block
    digits a_1..a_k, a_1 slowest), or None where an index is padding (>= n)."""
    from . import tuples

    tl = tuples(n, b, k)
    out = []
    for off in offs:
        r, e = divmod(int(off), b ** k)
        a = []
        for _ in range(k):
            e, am = divmod(e, b)
            a.append(am)
        a.reverse()
        idx = [int(j) * b + am for j, am in zip(tl[r], a)]
        out.append(idx if max(idx) < n else None)
    return out
