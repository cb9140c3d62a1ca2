"""The combine (every order in one launch over each order-d block's
sub-block lattice, or order by order) and its two formulas: Alg. 4's partition sum and the
recursion c_I = m_I - sum_{B holding I's first position} c_B m_{I\\B}.  Both
against the FP64 oracle (which follows Alg. 4 on the plain definition) on
shapes that use the lattice (d = 2..6 with small b, b not a power of two,
b not dividing n, b = 8), on shapes combined order by order, and against
each other."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import TOL, as_input, rel_err, to_device

pytestmark = pytest.mark.gpu

SHAPES = [  # n, d, b, t, p
    (20, 4, 2, 1500, 100),
    (20, 4, 3, 1500, 100),
    (60, 4, 4, 1500, 100),
    (17, 3, 8, 1500, 100),
    (16, 4, 8, 800, 100),
    (12, 5, 2, 800, 100),
    (8, 6, 2, 600, 100),
    (9, 2, 4, 600, 100),
]


def _rows(n, t, p, steps, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    x = rng.standard_normal((t + steps * p, n)) @ A.T + 0.3
    return x + 0.5 * (rng.exponential(size=x.shape) - 1.0)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "n%d_d%d_b%d" % s[:3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_partitions_and_recursion_vs_oracle(shape, prec):
    import paper_1701_06446_amd as cum

    n, d, b, t, p = shape
    steps = 2
    rows = as_input(_rows(n, t, p, steps, 31 + n + d + b), prec)
    dev = to_device(rows)
    part = cum.cum_init(n, d, b, dev[:t], prec=prec)
    rec = cum.cum_init(n, d, b, dev[:t], prec=prec)
    cum.cum_set_combine(rec, "recursion")
    for w in range(1, steps + 1):
        for c in (part, rec):
            cum.cum_update(c, dev[t + (w - 1) * p: t + w * p], dev[(w - 1) * p: w * p])
    Co = oracle.SlidingOracle(rows[steps * p: steps * p + t].astype(np.float64), n, d, b).cumulants()
    for k in range(1, d + 1):
        gp, gr = cum.cum_get(part, k), cum.cum_get(rec, k)
        ep, er = rel_err(gp, Co[k - 1], n, b, k), rel_err(gr, Co[k - 1], n, b, k)
        assert ep <= TOL[prec] and er <= TOL[prec], (k, ep, er)
        if prec == "fp64":
            assert rel_err(gr, gp, n, b, k) <= 1e-12, k
    fp, _ = cum.cum_norms(part)
    fr, _ = cum.cum_norms(rec)
    fo, _ = oracle.norms(Co, n, b)
    np.testing.assert_allclose(fp[1:], fo[1:], rtol=max(TOL[prec], 1e-12))
    np.testing.assert_allclose(fr[1:], fo[1:], rtol=max(TOL[prec], 1e-12))
    cum.cum_free(part)
    cum.cum_free(rec)


PER_ORDER = [  # n, d, b, t, p: lattices beyond the 64 KB of LDS, combined order by order
    (24, 6, 4, 600, 100),
    (16, 5, 8, 600, 100),
]


@pytest.mark.parametrize("shape", PER_ORDER, ids=lambda s: "n%d_d%d_b%d" % s[:3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_per_order_partitions_and_recursion_vs_oracle(shape, prec):
    """d = 6 with b = 4 and d = 5 with b = 8: the lattice does not fit, so
    each order is combined on its own (lower-order sub-blocks staged where
    they fit in LDS, gathered otherwise); the recursion takes the moments
    of the sub-blocks without the first position from the running sums."""
    test_partitions_and_recursion_vs_oracle(shape, prec)
