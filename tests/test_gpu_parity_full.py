"""GPU parity at the benchmark's full sizes: every stored element of the
n = 60, d = 4 stream against the pyramid oracle; at d = 6 (too large for the
pyramid oracle) sampled outputs the oracle computes one element at a time
(Alg. 4 on moments taken straight from the current window); and a
full-pyramid d = 6 case at a size the oracle finishes in seconds."""
import numpy as np
import pytest

import oracle
import streams
from oracle.element import cumulant_at, sample_elements
from tests.gpu_helpers import TOL, as_input, assert_mean_match, assert_norms_match, rel_err, to_device

pytestmark = pytest.mark.gpu


# The oracle's trajectory over the benchmark stream, one per input dtype
# (the fp32 and split-bf16 paths read the same FP32-rounded rows).
_FULL_STEPS, _FULL_SWITCH = 5, 2
_full_cache = {}


def _full_oracle(dtype):
    key = np.dtype(dtype).name
    if key not in _full_cache:
        s = streams.regime_change_stream(steps=_FULL_STEPS, switch=_FULL_SWITCH)
        rows = np.ascontiguousarray(s.rows.astype(dtype))
        t, p = s.t, s.p
        orc = oracle.SlidingOracle(rows[:t], s.n, s.d, s.b)
        traj = []
        for w in range(1, _FULL_STEPS + 1):
            orc.update(rows[t + (w - 1) * p:t + w * p], rows[(w - 1) * p:w * p])
            Co = orc.cumulants()
            traj.append((Co, oracle.norms(Co, s.n, s.b)))
        _full_cache[key] = (s, rows, traj)
    return _full_cache[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_regime_change_full_size_full_pyramid(prec):
    """n=60, d=4, b=4, t=20000, p=1000 (the benchmark's workload and launch
    configuration), 5 steps with the regime change after step 2: every
    stored element of C_1..C_4, the norms and nu_3, nu_4 against the FP64
    oracle after every step (eight 256-row chunks of added and of dropped
    rows per update, so the minus phase spans several chunks)."""
    import paper_1701_06446_amd as cum

    s, rows, traj = _full_oracle(np.float64 if prec == "fp64" else np.float32)
    dev = to_device(rows)
    t, p = s.t, s.p
    ctx = cum.cum_init(s.n, s.d, s.b, dev[:t], prec=prec)
    worst = np.zeros(s.d + 1)
    for w in range(1, _FULL_STEPS + 1):
        cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
        Co, (fro_o, nu_o) = traj[w - 1]
        Cg = [cum.cum_get(ctx, k) for k in range(1, s.d + 1)]
        for k in range(1, s.d + 1):
            worst[k] = max(worst[k], rel_err(Cg[k - 1], Co[k - 1], s.n, s.b, k))
        assert_mean_match(Cg[0], Co[0], Co[1], s.n, s.b, prec)
        fro_g, nu_g = cum.cum_norms(ctx)
        assert_norms_match(fro_g, nu_g, fro_o, nu_o, prec)
    cum.cum_free(ctx)
    print("prec=%s worst rel err per order over %d steps: %s" % (prec, _FULL_STEPS, worst[1:]))
    assert np.all(worst[2:] <= TOL[prec]), worst


# Sampled oracle values of the d = 6 sweep, per input dtype and step (the
# fp32 and split-bf16 paths read the same rows and are checked on the same
# elements).
_D6_STEPS, _D6_SAMPLES = 3, 100
_d6_cache = {}


def _d6_reference(dtype):
    key = np.dtype(dtype).name
    if key not in _d6_cache:
        s = streams.mixed_exp_stream(steps=_D6_STEPS)
        rows = np.ascontiguousarray(s.rows.astype(dtype))
        rng = np.random.default_rng(4)
        refs = []
        for w in range(1, _D6_STEPS + 1):
            window = rows[w * s.p:w * s.p + s.t].astype(np.float64)
            cache = {}
            per_k = {}
            for k in range(2, s.d + 1):
                offs, idxs = sample_elements(s.n, s.b, k, _D6_SAMPLES, rng)
                per_k[k] = (offs, np.array([cumulant_at(window, idx, cache) for idx in idxs]))
            refs.append(per_k)
        _d6_cache[key] = (s, rows, refs)
    return _d6_cache[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_mixed_exp_d6_full_size_sampled(prec):
    """n=48, d=6, b=4, t=50000, p=2000 (the high-order precision sweep), three
    updates; after each, 100 sampled elements per order 2..6 (eight 256-row
    chunks of each sign per update)."""
    import paper_1701_06446_amd as cum

    s, rows, refs = _d6_reference(np.float64 if prec == "fp64" else np.float32)
    dev = to_device(rows)
    t, p = s.t, s.p
    ctx = cum.cum_init(s.n, s.d, s.b, dev[:t], prec=prec)
    worst = np.zeros(s.d + 1)
    for w in range(1, _D6_STEPS + 1):
        cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
        for k in range(2, s.d + 1):
            offs, ref = refs[w - 1][k]
            g = cum.cum_get(ctx, k)[offs]
            worst[k] = max(worst[k], float(np.linalg.norm(g - ref) / np.linalg.norm(ref)))
    cum.cum_free(ctx)
    print("prec=%s sampled rel err per order 2..6: %s" % (prec, worst[2:]))
    assert np.all(worst[2:] <= TOL[prec]), worst


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_d6_full_pyramid_ragged(prec):
    """n=13 (b=4 does not divide n: one padded column block), d=6, t=600,
    p=150, 3 steps: every stored element against the pyramid oracle."""
    import paper_1701_06446_amd as cum

    s = streams.mixed_exp_stream(n=13, d=6, b=4, t=600, p=150, steps=3)
    rows = as_input(s.rows, prec)
    dev = to_device(rows)
    t, p = s.t, s.p
    ctx = cum.cum_init(s.n, s.d, s.b, dev[:t], prec=prec)
    orc = oracle.SlidingOracle(rows[:t], s.n, s.d, s.b)
    for w in range(1, 4):
        cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
        orc.update(rows[t + (w - 1) * p:t + w * p], rows[(w - 1) * p:w * p])
    Co = orc.cumulants()
    errs = [rel_err(cum.cum_get(ctx, k), Co[k - 1], s.n, s.b, k) for k in range(1, s.d + 1)]
    fro, _ = cum.cum_norms(ctx)
    fo, _ = oracle.norms(Co, s.n, s.b)
    cum.cum_free(ctx)
    print("prec=%s rel err per order: %s" % (prec, np.array(errs)))
    assert max(errs[1:]) <= TOL[prec]
    np.testing.assert_allclose(fro[1:], fo[1:], rtol=max(TOL[prec], 1e-12))
