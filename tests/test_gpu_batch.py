"""Batched streams: 64 uneven streams updated by one captured graph.  Every
member must equal its own single-context run to the contraction's rounding
(single contexts may take the four-tiles-per-workgroup update kernel, which
sums rows in another order) and match the oracle: the full pyramid for small
streams, sampled elements (per-element oracle on the final window) for the
others."""
import numpy as np
import pytest

import oracle
import streams
from oracle.element import cumulant_at, sample_elements
from tests.gpu_helpers import TOL, as_input, assert_same_to_rounding, rel_err, to_device

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_64_streams(prec):
    import paper_1701_06446_amd as cum

    steps = 3
    ss = streams.batched_streams(m=64, steps=steps)
    rows = [as_input(s.rows, prec) for s in ss]
    dev = [to_device(r) for r in rows]
    batched = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec=prec) for s, d in zip(ss, dev)]
    single = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec=prec) for s, d in zip(ss, dev)]
    bt = cum.cum_batch_create(batched)
    for w in range(1, steps + 1):
        xn = [d[s.t + (w - 1) * s.p:s.t + w * s.p] for s, d in zip(ss, dev)]
        xo = [d[(w - 1) * s.p:w * s.p] for s, d in zip(ss, dev)]
        cum.cum_batch_update(bt, xn, xo)
        for c, a, b in zip(single, xn, xo):
            cum.cum_update(c, a, b)
    cum.cum_batch_sync(bt)
    rng = np.random.default_rng(11)
    worst = 0.0
    for i, s in enumerate(ss):
        for k in range(1, s.d + 1):
            assert_same_to_rounding(cum.cum_get(batched[i], k), cum.cum_get(single[i], k), prec, (i, k),
                                    s.n, s.b, k)
        fb, nb = cum.cum_norms(batched[i])
        fs, ns = cum.cum_norms(single[i])
        assert_same_to_rounding(fb[1:], fs[1:], prec, (i, "norms"))
        window = rows[i][steps * s.p:steps * s.p + s.t].astype(np.float64)
        if s.n <= 12:
            orc = oracle.SlidingOracle(window, s.n, s.d, s.b)
            Co = orc.cumulants()
            for k in range(2, s.d + 1):
                worst = max(worst, rel_err(cum.cum_get(batched[i], k), Co[k - 1], s.n, s.b, k))
        elif i % 4 == 0:
            cache = {}
            for k in range(2, s.d + 1):
                offs, idxs = sample_elements(s.n, s.b, k, 8, rng)
                ref = np.array([cumulant_at(window, idx, cache) for idx in idxs])
                g = cum.cum_get(batched[i], k)[offs]
                worst = max(worst, float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
    cum.cum_batch_free(bt)
    for c in batched + single:
        cum.cum_free(c)
    print("prec=%s worst per-stream rel err %.3e" % (prec, worst))
    assert worst <= TOL[prec]


def test_batch_and_direct_updates_interleave():
    """A member updated directly between batch steps stays in stream order."""
    import paper_1701_06446_amd as cum

    ss = streams.batched_streams(m=3, steps=4, workload_id=9, n_max=24)
    dev = [to_device(as_input(s.rows, "fp32")) for s in ss]
    ctxs = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec="fp32") for s, d in zip(ss, dev)]
    ref = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec="fp32") for s, d in zip(ss, dev)]
    bt = cum.cum_batch_create(ctxs)
    for w in range(1, 5):
        xn = [d[s.t + (w - 1) * s.p:s.t + w * s.p] for s, d in zip(ss, dev)]
        xo = [d[(w - 1) * s.p:w * s.p] for s, d in zip(ss, dev)]
        if w % 2:
            cum.cum_batch_update(bt, xn, xo)
        else:
            for c, a, b in zip(ctxs, xn, xo):
                cum.cum_update(c, a, b)
        for c, a, b in zip(ref, xn, xo):
            cum.cum_update(c, a, b)
    for c, r, s in zip(ctxs, ref, ss):
        for k in range(1, s.d + 1):
            assert_same_to_rounding(cum.cum_get(c, k), cum.cum_get(r, k), "fp32", k, s.n, s.b, k)
    cum.cum_batch_free(bt)


def test_batch_rejects_host_pointers():
    import paper_1701_06446_amd as cum

    ss = streams.batched_streams(m=2, steps=1, workload_id=10, n_max=16)
    hosts = [as_input(s.rows, "fp32") for s in ss]
    ctxs = [cum.cum_init(s.n, s.d, s.b, h[:s.t], prec="fp32") for s, h in zip(ss, hosts)]
    bt = cum.cum_batch_create(ctxs)
    with pytest.raises(cum.CumError) as e:
        cum.cum_batch_update(bt, [h[s.t:s.t + s.p] for s, h in zip(ss, hosts)],
                             [h[:s.p] for s, h in zip(ss, hosts)])
    assert e.value.status == cum.CUM_EINVAL
    cum.cum_batch_free(bt)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_with_an_idle_member(prec):
    """A member handed 0 rows in a batch step keeps its state (its tiles run
    with no chunks); the others slide as usual."""
    import paper_1701_06446_amd as cum

    ss = streams.batched_streams(m=3, steps=3, workload_id=12, n_max=32)
    dev = [to_device(as_input(s.rows, prec)) for s in ss]
    ctxs = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec=prec) for s, d in zip(ss, dev)]
    ref = [cum.cum_init(s.n, s.d, s.b, d[:s.t], prec=prec) for s, d in zip(ss, dev)]
    bt = cum.cum_batch_create(ctxs)
    done = [0, 0, 0]
    for w in range(1, 4):
        xn, xo = [], []
        for i, (s, d) in enumerate(zip(ss, dev)):
            if w == 2 and i == 1:
                xn.append(d[:0])
                xo.append(d[:0])
                continue
            done[i] += 1
            c = done[i]
            xn.append(d[s.t + (c - 1) * s.p:s.t + c * s.p])
            xo.append(d[(c - 1) * s.p:c * s.p])
        cum.cum_batch_update(bt, xn, xo)
        for r, a, b in zip(ref, xn, xo):
            if a.shape[0]:
                cum.cum_update(r, a, b)
    cum.cum_batch_sync(bt)
    for c, r, s in zip(ctxs, ref, ss):
        for k in range(1, s.d + 1):
            assert_same_to_rounding(cum.cum_get(c, k), cum.cum_get(r, k), prec, k, s.n, s.b, k)
        fc, _ = cum.cum_norms(c)
        fr, _ = cum.cum_norms(r)
        assert_same_to_rounding(fc[1:], fr[1:], prec, "norms")
    cum.cum_batch_free(bt)
    for c in ctxs + ref:
        cum.cum_free(c)
