"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs."""
import numpy as np
import pytest

import oracle
import streams
from tests.gpu_helpers import TOL, as_input, assert_mean_match, assert_norms_match, rel_err, to_device

pytestmark = pytest.mark.gpu


def _run_case(stream, prec, steps, device_inputs=True, check_every=1):
    import paper_1701_06446_amd as cum

    n, d, b, t, p = stream.n, stream.d, stream.b, stream.t, stream.p
    rows = as_input(stream.rows[: t + steps * p], prec)
    dev = to_device(rows) if device_inputs else None
    src = dev if device_inputs else rows
    ctx = cum.cum_init(n, d, b, src[:t], prec=prec)
    orc = oracle.SlidingOracle(rows[:t], n, d, b)
    worst = np.zeros(d + 1)
    for w in range(0, steps + 1):
        if w > 0:
            lo, hi = (w - 1) * p, w * p
            cum.cum_update(ctx, src[t + lo: t + hi], src[lo:hi])
            orc.update(rows[t + lo: t + hi], rows[lo:hi])
        if w % check_every and w != steps:
            continue
        Co = orc.cumulants()
        Cg = [cum.cum_get(ctx, k) for k in range(1, d + 1)]
        for k in range(1, d + 1):
            worst[k] = max(worst[k], rel_err(Cg[k - 1], Co[k - 1], n, b, k))
        assert_mean_match(Cg[0], Co[0], Co[1], n, b, prec)
        fro_g, nu_g = cum.cum_norms(ctx)
        fro_o, nu_o = oracle.norms(Co, n, b)
        assert_norms_match(fro_g, nu_g, fro_o, nu_o, prec)
    cum.cum_free(ctx)
    print("prec=%s worst rel err per order: %s" % (prec, worst[1:]))
    assert np.all(worst[2:] <= TOL[prec]), worst
    return worst


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_gaussian_n20_d4_b2(prec):
    """n=20, d=4, b=2, t=2000, p=100, 20 steps, every step checked."""
    s = streams.gaussian_stream()
    _run_case(s, prec, steps=20)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_regime_change_n60_d4_b4_small_window(prec):
    """n=60, d=4, b=4 at a window the oracle finishes in seconds (t=2000,
    p=100), 6 steps with the regime change inside: several tiles per pivot and
    ragged pivot GEMM edges."""
    s = streams.regime_change_stream(t=2000, p=100, steps=6, switch=3)
    _run_case(s, prec, steps=6)
