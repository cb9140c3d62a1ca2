"""Pipelined sliding updates (CUM_PIPELINE=1) — the update launch stores
the increment, and its fold into the running sums, the combine and the
norms run on a side stream beside the next update — against the same
updates run one after another on the context's stream (the default,
CUM_PIPELINE=0): bitwise equal running
sums, cumulants and norms, with reads between the steps and without, for
every precision; plus host-memory inputs, a recalculation in the middle and
the norms read on the device."""
import os

import numpy as np
import pytest
import torch

import streams

pytestmark = pytest.mark.gpu


def _pair(n, d, b, window, prec):
    import paper_1701_06446_amd as cum

    old = os.environ.get("CUM_PIPELINE")
    try:
        os.environ["CUM_PIPELINE"] = "1"
        piped = cum.cum_init(n, d, b, window, prec=prec)
        os.environ["CUM_PIPELINE"] = "0"
        plain = cum.cum_init(n, d, b, window, prec=prec)
    finally:
        if old is None:
            os.environ.pop("CUM_PIPELINE", None)
        else:
            os.environ["CUM_PIPELINE"] = old
    return piped, plain


def _same(cum, a, b, d):
    for k in range(1, d + 1):
        assert np.array_equal(cum.cum_get_moments(a, k), cum.cum_get_moments(b, k)), k
        assert np.array_equal(cum.cum_get(a, k), cum.cum_get(b, k)), k
    fa, na = cum.cum_norms(a)
    fb, nb = cum.cum_norms(b)
    assert np.array_equal(fa, fb, equal_nan=True) and np.array_equal(na, nb, equal_nan=True)


@pytest.mark.parametrize("prec,n,b", [("fp64", 24, 4), ("fp32", 24, 4), ("bf16x3", 24, 4), ("fp32", 20, 3)])
def test_pipelined_updates_bitwise_equal_to_serial(prec, n, b):
    """(n = 20, b = 3: padded columns, whose elements the update never writes.)"""
    import paper_1701_06446_amd as cum

    s = streams.regime_change_stream(n=n, d=4, b=b, t=2000, p=200, steps=9, switch=4)
    dt = np.float64 if prec == "fp64" else np.float32
    rows = np.ascontiguousarray(s.rows.astype(dt))
    dev = torch.from_numpy(rows).cuda()
    t, p = s.t, s.p
    piped, plain = _pair(s.n, s.d, s.b, dev[:t], prec)
    for w in range(1, 10):
        X_new, X_old = dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p]
        if w == 5:  # host inputs: staged, then the same pipelined update
            X_new, X_old = rows[t + (w - 1) * p:t + w * p], rows[(w - 1) * p:w * p]
        cum.cum_update(piped, X_new, X_old)
        cum.cum_update(plain, X_new, X_old)
        if w in (2, 6):
            _same(cum, piped, plain, s.d)
        if w == 7:  # a recalculation of the current window on both
            win = dev[w * p:w * p + t]
            cum.cum_recompute(piped, win)
            cum.cum_recompute(plain, win)
    # the norms read on the device after the last step
    ptr = cum.cum_norms_device(piped)
    assert ptr != 0
    cum.cum_sync(piped)
    _same(cum, piped, plain, s.d)
    cum.cum_free(piped)
    cum.cum_free(plain)
