"""cum_update_noalloc (host inputs staged through the library's fixed device
array, no allocation) against cum_update (host inputs staged through a
buffer the context allocates): the same window, the same rows, two calls in
a row, the second with fewer rows; the results must agree bit for bit (the
same kernels consume the same values)."""
import numpy as np
import pytest

from tests.gpu_helpers import as_input, to_device

pytestmark = pytest.mark.gpu


def _rows(seed, m, n):
    return np.random.default_rng(seed).standard_normal((m, n)) + 0.2


def _state(cum, ctx, d):
    return [cum.cum_get(ctx, k) for k in range(1, d + 1)] + list(cum.cum_norms(ctx))


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_matches_update_sliding(prec):
    import paper_1701_06446_amd as cum

    n, d, b, t = 60, 4, 4, 4000
    rows = as_input(_rows(21, t + 1300, n), prec)
    dev = to_device(rows)
    ref = cum.cum_init(n, d, b, dev[:t], prec=prec)
    new = cum.cum_init(n, d, b, dev[:t], prec=prec)
    lo = 0
    for p in (1000, 300):  # the second call stages fewer rows
        xn, xo = rows[t + lo:t + lo + p], rows[lo:lo + p]  # host memory
        cum.cum_update(ref, xn, xo)
        cum.cum_update_noalloc(new, xn, xo)
        lo += p
        for a, c in zip(_state(cum, ref, d), _state(cum, new, d)):
            assert np.array_equal(a, c, equal_nan=True)
    cum.cum_free(ref)
    cum.cum_free(new)


def test_noalloc_matches_update_fifo():
    import paper_1701_06446_amd as cum

    n, d, b, t, p = 24, 4, 4, 1200, 200
    rows = as_input(_rows(22, t + 2 * p, n), "fp32")
    dev = to_device(rows)
    ref = cum.cum_init_fifo(n, d, b, dev[:t], p, prec="fp32")
    new = cum.cum_init_fifo(n, d, b, dev[:t], p, prec="fp32")
    for w in range(2):
        xn = rows[t + w * p:t + (w + 1) * p]
        cum.cum_update(ref, xn)
        cum.cum_update_noalloc(new, xn)
        for a, c in zip(_state(cum, ref, d), _state(cum, new, d)):
            assert np.array_equal(a, c, equal_nan=True)
    cum.cum_free(ref)
    cum.cum_free(new)


def test_noalloc_rejects_rows_beyond_the_array():
    """2 * p * n * 8 bytes beyond 16 MiB is refused before any work, and
    the context stays usable."""
    import paper_1701_06446_amd as cum

    n, d, b, t, p = 255, 2, 8, 5000, 4200
    rows = as_input(_rows(23, t + p, n), "fp64")
    dev = to_device(rows)
    ctx = cum.cum_init(n, d, b, dev[:t], prec="fp64")
    before = _state(cum, ctx, d)
    with pytest.raises(cum.CumError) as e:
        cum.cum_update_noalloc(ctx, rows[t:t + p], rows[:p])
    assert e.value.status == cum.CUM_ESIZE
    for a, c in zip(before, _state(cum, ctx, d)):
        assert np.array_equal(a, c, equal_nan=True)
    cum.cum_update_noalloc(ctx, rows[t:t + 1000], rows[:1000])  # within the limit
    cum.cum_free(ctx)
