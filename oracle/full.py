"""Full n^k tensors for tiny n (oracle helpers, test infrastructure only).

``unpack`` turns a pyramid (Sec. 2.3 block layout, columns zero-padded to
ceil(n/b)*b) into the full super-symmetric n^k tensor by sorting every
multi-index and reading its stored element; ``pack`` goes the other way.
"""
from __future__ import annotations

import itertools

import numpy as np

from . import tuples


def _block_rank(n: int, b: int, k: int):
    return {tuple(int(v) for v in t): r for r, t in enumerate(tuples(n, b, k))}


def unpack(P, n: int, b: int, k: int) -> np.ndarray:
    """Pyramid -> full tensor of shape (n,)*k, element i read at sort(i)."""
    P = np.asarray(P, dtype=np.float64)
    rank = _block_rank(n, b, k)
    T = np.zeros((n,) * k)
    for i in itertools.product(range(n), repeat=k):
        s = sorted(i)
        blk = rank[tuple(v // b for v in s)]
        off = 0
        for v in s:
            off = off * b + v % b
        T[i] = P[blk * b ** k + off]
    return T


def pack(T, n: int, b: int, k: int) -> np.ndarray:
    """Full tensor -> pyramid; padded entries are zero."""
    T = np.asarray(T, dtype=np.float64)
    tl = tuples(n, b, k)
    P = np.zeros(len(tl) * b ** k)
    for r, j in enumerate(tl):
        for e, a in enumerate(itertools.product(range(b), repeat=k)):
            i = tuple(int(jm) * b + am for jm, am in zip(j, a))
            if all(v < n for v in i):
                P[r * b ** k + e] = T[i]
    return P
