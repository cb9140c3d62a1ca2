"""cum_recompute: the from-scratch recalculation of the current window on an
existing context (what Eq. (upcmplx) compares the update with).  After 30
updates, recomputing the window gives bit for bit what a fresh context
initialised on that window gives (same contraction, same order), matches the
oracle, and a FIFO context keeps sliding correctly afterwards."""
import numpy as np
import pytest

import oracle
import streams
from tests.gpu_helpers import TOL, as_input, rel_err, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["sliding", "fifo"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_recompute_equals_fresh_init(mode, prec):
    import paper_1701_06446_amd as cum

    s = streams.regime_change_stream(t=2000, p=100, steps=40, switch=10)
    n, d, b, t, p = s.n, s.d, s.b, s.t, s.p
    rows = as_input(s.rows, prec)
    dev = to_device(rows)

    def make(X):
        return cum.cum_init_fifo(n, d, b, X, p, prec=prec) if mode == "fifo" else cum.cum_init(n, d, b, X, prec=prec)

    ctx = make(dev[:t])
    for w in range(1, 31):
        cum.cum_update(ctx, dev[t + (w - 1) * p: t + w * p], None if mode == "fifo" else dev[(w - 1) * p: w * p])
    win = dev[30 * p: 30 * p + t]
    cum.cum_recompute(ctx, win)
    fresh = make(win)
    for k in range(1, d + 1):
        assert np.array_equal(cum.cum_get(ctx, k), cum.cum_get(fresh, k)), k
    Co = oracle.SlidingOracle(rows[30 * p: 30 * p + t].astype(np.float64), n, d, b).cumulants()
    for k in range(2, d + 1):
        assert rel_err(cum.cum_get(ctx, k), Co[k - 1], n, b, k) <= TOL[prec]
    # both keep sliding the same way
    for w in range(31, 41):
        for c in (ctx, fresh):
            cum.cum_update(c, dev[t + (w - 1) * p: t + w * p], None if mode == "fifo" else dev[(w - 1) * p: w * p])
    for k in range(1, d + 1):
        assert np.array_equal(cum.cum_get(ctx, k), cum.cum_get(fresh, k)), k
    Co = oracle.SlidingOracle(rows[40 * p: 40 * p + t].astype(np.float64), n, d, b).cumulants()
    for k in range(2, d + 1):
        assert rel_err(cum.cum_get(ctx, k), Co[k - 1], n, b, k) <= TOL[prec]
    cum.cum_free(ctx)
    cum.cum_free(fresh)


def test_recompute_from_host_rows():
    import paper_1701_06446_amd as cum

    s = streams.gaussian_stream(steps=5)
    rows = as_input(s.rows, "fp32")
    ctx = cum.cum_init(s.n, s.d, s.b, rows[:s.t])
    cum.cum_recompute(ctx, rows[3 * s.p: 3 * s.p + s.t])
    fresh = cum.cum_init(s.n, s.d, s.b, rows[3 * s.p: 3 * s.p + s.t])
    for k in range(1, s.d + 1):
        assert np.array_equal(cum.cum_get(ctx, k), cum.cum_get(fresh, k))
    with pytest.raises(ValueError):
        cum.cum_recompute(ctx, rows[: s.t - 1])
    cum.cum_free(ctx)
    cum.cum_free(fresh)
