"""The high-order precision sweep's closed form, at its full shape (n=48,
b=4, t=50000, p=2000): rows X = S W with S i.i.d. standardized Exp(1)
sources and W orthogonal, so the cumulant tensors transform as
C_k(x)_{i1..ik} = sum_a C_k(s)_{a1..ak} W_{a1 i1} ... W_{ak ik} and, mapped back
with W, the source-space tensors are diagonal with the Exp(1) cumulants
(k-1)! up to sampling error.  After two slides the GPU's order-3 tensor,
mapped back, is compared element by element with the third central moments
of the source window computed directly by numpy (an independent route: no
oracle, no pyramid); the order-4 tensor is checked against the closed form
(diagonal near 3! = 6, off-diagonal entries near 0, bounds set from the
sampling spread of these sources)."""
import itertools

import numpy as np
import pytest

import oracle
import streams
from tests.gpu_helpers import TOL, to_device

pytestmark = pytest.mark.gpu


def _full(P, n, b, k):
    """Pyramid (library layout: sorted block tuples, b^k elements each) ->
    full (n,)*k tensor, vectorised over the sorted multi-indices."""
    tl = oracle.tuples(n, b, k)
    nbar = -(-n // b)
    rank = np.full((nbar,) * k, -1, np.int64)
    rank[tuple(np.asarray(tl).T)] = np.arange(len(tl))
    idx = np.array(list(itertools.combinations_with_replacement(range(n), k)))
    blk = rank[tuple((idx // b).T)]
    off = np.zeros(len(idx), np.int64)
    for q in range(k):
        off = off * b + idx[:, q] % b
    vals = np.asarray(P, dtype=np.float64)[blk * b ** k + off]
    T = np.zeros((n,) * k)
    for perm in itertools.permutations(range(k)):
        T[tuple(idx[:, list(perm)].T)] = vals
    return T


def _to_sources(T, W):
    k = T.ndim
    for _ in range(k):  # contract the leading mode with W, move the result to the end
        T = np.tensordot(T, W, axes=([0], [1]))
    return T


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_mixed_exp_source_space_closed_form(prec):
    import paper_1701_06446_amd as cum

    s = streams.mixed_exp_stream(steps=2)
    n, b, t, p = s.n, s.b, s.t, s.p
    rows = np.ascontiguousarray(s.rows.astype(np.float64 if prec == "fp64" else np.float32))
    dev = to_device(rows)
    ctx = cum.cum_init(n, 4, b, dev[:t], prec=prec)
    for w in (1, 2):
        cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
    C3 = _to_sources(_full(cum.cum_get(ctx, 3), n, b, 3), s.mixing)
    C4 = _to_sources(_full(cum.cum_get(ctx, 4), n, b, 4), s.mixing)
    cum.cum_free(ctx)

    # the source window, straight from the rows the GPU read
    S = rows[2 * p:2 * p + t].astype(np.float64) @ s.mixing.T
    Sc = S - S.mean(0)
    ref3 = np.einsum("la,lb,lc->abc", Sc, Sc, Sc, optimize=True) / t
    err3 = np.linalg.norm(C3 - ref3) / np.linalg.norm(ref3)
    print("prec=%s order-3 source-space rel err %.3e" % (prec, err3))
    assert err3 <= TOL[prec]

    d3, d4 = np.einsum("aaa->a", C3), np.einsum("aaaa->a", C4)
    off3 = C3 - np.einsum("a,ab,ac->abc", d3, np.eye(n), np.eye(n))
    off4 = C4.copy()
    off4[np.arange(n), np.arange(n), np.arange(n), np.arange(n)] = 0.0
    print("diag C3 %.3f..%.3f  |off| %.3f   diag C4 %.3f..%.3f  |off| %.3f" %
          (d3.min(), d3.max(), np.abs(off3).max(), d4.min(), d4.max(), np.abs(off4).max()))
    assert np.all(np.abs(d3 - 2.0) <= 0.4) and np.abs(off3).max() <= 0.15
    assert np.all(np.abs(d4 - 6.0) <= 3.0) and np.abs(off4).max() <= 0.8
