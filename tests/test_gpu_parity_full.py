"""GPU parity at the benchmark's full sizes, on sampled outputs the oracle
computes one element at a time (Alg. 4 on moments taken straight from the
current window), and a full-pyramid d = 6 case at a size the oracle finishes
in seconds."""
import numpy as np
import pytest

import oracle
import streams
from oracle.element import cumulant_at, sample_elements
from tests.gpu_helpers import TOL, as_input, rel_err, to_device

pytestmark = pytest.mark.gpu


def _sampled_rel_err(C_gpu, window, n, b, k, count, rng, cache):
    offs, idxs = sample_elements(n, b, k, count, rng)
    ref = np.array([cumulant_at(window, idx, cache) for idx in idxs])
    return float(np.linalg.norm(C_gpu[offs] - ref) / np.linalg.norm(ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_regime_change_full_size_sampled(prec):
    """n=60, d=4, b=4, t=20000, p=1000 (the benchmark's workload), 4 steps
    across the regime change; 60 sampled elements per order."""
    import paper_1701_06446_amd as cum

    s = streams.regime_change_stream(steps=4, switch=2)
    rows = as_input(s.rows, prec)
    dev = to_device(rows)
    t, p = s.t, s.p
    ctx = cum.cum_init(s.n, s.d, s.b, dev[:t], prec=prec)
    for w in range(1, 5):
        cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
    window = rows[4 * p:4 * p + t].astype(np.float64)
    rng = np.random.default_rng(3)
    cache = {}
    worst = 0.0
    for k in range(2, s.d + 1):
        worst = max(worst, _sampled_rel_err(cum.cum_get(ctx, k), window, s.n, s.b, k, 60, rng, cache))
    # the device norms agree with Alg. 5 applied to the returned pyramids
    fro, nu = cum.cum_norms(ctx)
    for k in range(1, s.d + 1):
        assert abs(fro[k] - oracle.block_norm(cum.cum_get(ctx, k), s.n, s.b, k)) <= 1e-12 * fro[k]
    cum.cum_free(ctx)
    print("prec=%s sampled rel err %.3e" % (prec, worst))
    assert worst <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_mixed_exp_d6_full_size_sampled(prec):
    """n=48, d=6, b=4, t=50000, p=2000 (the high-order precision sweep), one
    update; 12 sampled elements per order 2..6."""
    import paper_1701_06446_amd as cum

    s = streams.mixed_exp_stream(steps=1)
    rows = as_input(s.rows, prec)
    dev = to_device(rows)
    t, p = s.t, s.p
    ctx = cum.cum_init(s.n, s.d, s.b, dev[:t], prec=prec)
    cum.cum_update(ctx, dev[t:t + p], dev[:p])
    window = rows[p:p + t].astype(np.float64)
    rng = np.random.default_rng(4)
    cache = {}
    errs = []
    for k in range(2, s.d + 1):
        errs.append(_sampled_rel_err(cum.cum_get(ctx, k), window, s.n, s.b, k, 12, rng, cache))
    cum.cum_free(ctx)
    print("prec=%s sampled rel err per order 2..6: %s" % (prec, np.array(errs)))
    assert max(errs) <= TOL[prec]


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
