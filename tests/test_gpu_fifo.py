"""FIFO mode (the batch-moment queue of Sec. 2.4, after Alg. 2): the window's moments are
the same numbers as in sliding mode, so the checks are the oracle on the
current window, past the point where the queue has wrapped around (every
stored increment replaced at least once); bit-exact sums on integer-valued
data (nothing drifts when the leaving batch's increment is folded out);
batched members against single contexts (to the contraction's rounding); and
the error paths."""
import numpy as np
import pytest

import oracle
import streams
from tests.gpu_helpers import TOL, as_input, assert_same_to_rounding, rel_err, to_device

pytestmark = pytest.mark.gpu


def _fifo_case(stream, prec, steps, check_at):
    import paper_1701_06446_amd as cum

    n, d, b, t, p = stream.n, stream.d, stream.b, stream.t, stream.p
    rows = as_input(stream.rows[: t + steps * p], prec)
    dev = to_device(rows)
    ctx = cum.cum_init_fifo(n, d, b, dev[:t], p, prec=prec)
    worst = np.zeros(d + 1)
    for w in range(1, steps + 1):
        cum.cum_update(ctx, dev[t + (w - 1) * p: t + w * p])
        if w not in check_at:
            continue
        Co = oracle.SlidingOracle(rows[w * p: w * p + t], n, d, b).cumulants()
        for k in range(1, d + 1):
            worst[k] = max(worst[k], rel_err(cum.cum_get(ctx, k), Co[k - 1], n, b, k))
        fro_g, _ = cum.cum_norms(ctx)
        fro_o, _ = oracle.norms(Co, n, b)
        np.testing.assert_allclose(fro_g[1:], fro_o[1:], rtol=max(TOL[prec], 1e-12))
    cum.cum_free(ctx)
    print("fifo prec=%s worst rel err per order: %s" % (prec, worst[1:]))
    assert np.all(worst[2:] <= TOL[prec]), worst


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_fifo_gaussian_n20_d4_b2(prec):
    """n=20, d=4, b=2, t=2000, p=100: 20 slots, 45 steps (two wrap-arounds)."""
    s = streams.gaussian_stream(steps=45)
    _fifo_case(s, prec, steps=45, check_at={1, 19, 20, 21, 40, 45})


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fifo_regime_change_n60_d4_b4(prec):
    """n=60, d=4, b=4, t=2000, p=100 with the regime change at step 10."""
    s = streams.regime_change_stream(t=2000, p=100, steps=25, switch=10)
    _fifo_case(s, prec, steps=25, check_at={5, 20, 25})


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fifo_integer_data_is_exact(prec):
    """Integer rows in [-3, 3] (n=12, d=4, b=4, t=400, p=50, 8 slots): every
    product and partial sum is an exact integer in FP32, so after 30 updates
    t * M_k must be the window's integer sums exactly, and equal in FIFO and
    sliding mode."""
    import paper_1701_06446_amd as cum

    n, d, b, t, p, steps = 12, 4, 4, 400, 50, 30
    rng = np.random.default_rng(1701)
    rows = as_input(rng.integers(-3, 4, size=(t + steps * p, n)).astype(np.float64), prec)
    dev = to_device(rows)
    fifo = cum.cum_init_fifo(n, d, b, dev[:t], p, prec=prec)
    slide = cum.cum_init(n, d, b, dev[:t], prec=prec)
    for w in range(1, steps + 1):
        cum.cum_update(fifo, dev[t + (w - 1) * p: t + w * p])
        cum.cum_update(slide, dev[t + (w - 1) * p: t + w * p], dev[(w - 1) * p: w * p])
    Mo = oracle.moments_of(rows[steps * p: steps * p + t].astype(np.float64), n, d, b)
    for k in range(1, d + 1):
        exact = np.rint(np.asarray(Mo[k - 1]) * t)
        for ctx in (fifo, slide):
            mt = cum.cum_get_moments(ctx, k) * t
            assert np.max(np.abs(mt - np.rint(mt))) < 1e-6
            assert np.array_equal(np.rint(mt), exact), k
    cum.cum_free(fifo)
    cum.cum_free(slide)


def test_fifo_batched_members_match_single_contexts():
    """Two FIFO and two sliding members in one batch equal their own single
    contexts to rounding after 25 steps (the FIFO slots wrap at 20)."""
    import paper_1701_06446_amd as cum

    steps = 25
    ss = streams.batched_streams(m=4, steps=steps, workload_id=13, n_max=24)
    dev = [to_device(as_input(s.rows, "fp32")) for s in ss]

    def make(i, s, d):
        if i % 2 == 0:
            return cum.cum_init_fifo(s.n, s.d, s.b, d[:s.t], s.p, prec="fp32")
        return cum.cum_init(s.n, s.d, s.b, d[:s.t], prec="fp32")

    members = [make(i, s, d) for i, (s, d) in enumerate(zip(ss, dev))]
    single = [make(i, s, d) for i, (s, d) in enumerate(zip(ss, dev))]
    bt = cum.cum_batch_create(members)
    for w in range(1, steps + 1):
        xn = [d[s.t + (w - 1) * s.p:s.t + w * s.p] for s, d in zip(ss, dev)]
        xo = [None if i % 2 == 0 else d[(w - 1) * s.p:w * s.p] for i, (s, d) in enumerate(zip(ss, dev))]
        cum.cum_batch_update(bt, xn, xo)
        for c, a, o in zip(single, xn, xo):
            cum.cum_update(c, a, o)
    cum.cum_batch_sync(bt)
    for i, s in enumerate(ss):
        for k in range(1, s.d + 1):
            assert_same_to_rounding(cum.cum_get(members[i], k), cum.cum_get(single[i], k), "fp32", (i, k),
                                    s.n, s.b, k)
        window = as_input(s.rows, "fp32")[steps * s.p: steps * s.p + s.t].astype(np.float64)
        Co = oracle.SlidingOracle(window, s.n, s.d, s.b).cumulants()
        for k in range(2, s.d + 1):
            assert rel_err(cum.cum_get(members[i], k), Co[k - 1], s.n, s.b, k) <= TOL["fp32"]
    cum.cum_batch_free(bt)
    for c in members + single:
        cum.cum_free(c)


def test_fifo_argument_errors():
    import paper_1701_06446_amd as cum

    rows = to_device(as_input(np.random.default_rng(3).standard_normal((600, 8)), "fp32"))
    with pytest.raises(cum.CumError) as e:
        cum.cum_init_fifo(8, 3, 2, rows[:500], 300)          # t % p != 0
    assert e.value.status == cum.CUM_EINVAL
    with pytest.raises(cum.CumError) as e:
        cum.cum_init_fifo(8, 3, 2, rows[:500], 0)            # p < 1
    assert e.value.status == cum.CUM_EINVAL
    big = to_device(as_input(np.random.default_rng(4).standard_normal((4096, 8)), "fp32"))
    with pytest.raises(cum.CumError) as e:
        cum.cum_init_fifo(8, 3, 2, big, 4096)                # p > 2048
    assert e.value.status == cum.CUM_ESIZE
    ctx = cum.cum_init_fifo(8, 3, 2, rows[:500], 100)
    with pytest.raises(cum.CumError) as e:
        cum.cum_update(ctx, rows[500:550])                   # p differs from the batch size
    assert e.value.status == cum.CUM_EINVAL
    cum.cum_update(ctx, rows[500:600], rows[:100])           # X_old is accepted and not read
    plain = cum.cum_init(8, 3, 2, rows[:500])
    with pytest.raises(cum.CumError) as e:
        cum.cum_update(plain, rows[500:600])                 # sliding mode needs X_old
    assert e.value.status == cum.CUM_EINVAL
    cum.cum_free(ctx)
    cum.cum_free(plain)
