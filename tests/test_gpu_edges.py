"""GPU edge cases: empty and ragged inputs, p = 1, p = t and p beyond one
contraction chunk, host inputs, rows whose length is not a multiple of 16
bytes, b = 1 and b = n, d = 1 and 2, constant windows, the column maximum,
determinism, and exact slide-vs-recompute agreement on integer data."""
import numpy as np
import pytest

import oracle
from tests.gpu_helpers import TOL, as_input, assert_mean_match, assert_norms_match, rel_err, to_device

pytestmark = pytest.mark.gpu


def _rows(seed, m, n, scale=1.0, shift=0.3):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, n)) * scale + shift


def _check_against_oracle(n, d, b, t, p, steps, prec, seed=0, device=True, data=None):
    import paper_1701_06446_amd as cum

    raw = data if data is not None else _rows(seed, t + steps * p, n)
    rows = as_input(raw, prec)
    src = to_device(rows) if device else rows
    ctx = cum.cum_init(n, d, b, src[:t], prec=prec)
    orc = oracle.SlidingOracle(rows[:t], n, d, b)
    for w in range(1, steps + 1):
        cum.cum_update(ctx, src[t + (w - 1) * p:t + w * p], src[(w - 1) * p:w * p])
        orc.update(rows[t + (w - 1) * p:t + w * p], rows[(w - 1) * p:w * p])
    Co = orc.cumulants()
    Cg = [cum.cum_get(ctx, k) for k in range(1, d + 1)]
    errs = [rel_err(Cg[k - 1], Co[k - 1], n, b, k) for k in range(1, d + 1)]
    fro, nu = cum.cum_norms(ctx)
    cum.cum_free(ctx)
    gate = errs[1:] if d > 1 else errs
    assert max(gate) <= TOL[prec], (n, d, b, t, p, prec, errs)
    if d > 1:
        assert_mean_match(Cg[0], Co[0], Co[1], n, b, prec)
    fo, no = oracle.norms(Co, n, b)
    assert_norms_match(fro, nu, fo, no, prec)
    return errs, fro, nu


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("p", [1, 7, 300])
def test_batch_sizes(prec, p):
    """p = 1 (single row), a ragged p, and p = t (the whole window replaced)."""
    t = 300
    _check_against_oracle(n=11, d=4, b=3, t=t, p=p, steps=2, prec=prec, seed=p)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batch_beyond_one_chunk(prec):
    """p = 2500 > 2048: the update is contracted and folded in two chunks."""
    _check_against_oracle(n=9, d=3, b=4, t=5000, p=2500, steps=2, prec=prec, seed=5)


def test_zero_rows_is_noop():
    import paper_1701_06446_amd as cum

    rows = as_input(_rows(1, 200, 8), "fp32")
    dev = to_device(rows)
    ctx = cum.cum_init(8, 3, 2, dev, prec="fp32")
    before = [cum.cum_get(ctx, k) for k in (1, 2, 3)]
    cum.cum_update(ctx, dev[:0], dev[:0])
    after = [cum.cum_get(ctx, k) for k in (1, 2, 3)]
    for a, c in zip(before, after):
        assert np.array_equal(a, c)
    cum.cum_free(ctx)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_host_inputs(prec):
    """Inputs in host memory are staged by the library."""
    _check_against_oracle(n=12, d=4, b=4, t=400, p=50, steps=3, prec=prec, seed=2, device=False)


@pytest.mark.parametrize("prec,n", [("fp32", 13), ("fp64", 7), ("bf16x3", 13)])
def test_rows_not_multiple_of_16_bytes(prec, n):
    """Row lengths of 52 (fp32) and 56 (fp64) bytes take the scalar chunk loader."""
    _check_against_oracle(n=n, d=4, b=2, t=256, p=40, steps=2, prec=prec, seed=n)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("b", [1, 10])
def test_block_size_one_and_n(prec, b):
    _check_against_oracle(n=10, d=4, b=b, t=300, p=30, steps=2, prec=prec, seed=b)


@pytest.mark.parametrize("d", [1, 2])
def test_low_orders_nu_is_nan(d):
    errs, fro, nu = _check_against_oracle(n=16, d=d, b=4, t=300, p=30, steps=2, prec="fp64", seed=d)
    assert np.all(np.isnan(nu))


def test_constant_window_nu_nan():
    """A constant window has C_k = 0 for k >= 2: norms 0 and nu undefined."""
    import paper_1701_06446_amd as cum

    rows = np.full((200, 6), 1.5)
    dev = to_device(rows)
    ctx = cum.cum_init(6, 4, 2, dev[:100], prec="fp64")
    cum.cum_update(ctx, dev[100:150], dev[:50])
    fro, nu = cum.cum_norms(ctx)
    cum.cum_free(ctx)
    assert np.allclose(fro[2:], 0.0, atol=1e-12)
    assert abs(fro[1] - 1.5 * np.sqrt(6)) < 1e-12
    assert np.all(np.isnan(nu[3:]))


def test_max_columns_sampled():
    """n = 255 (the column limit), d = 3, b = 8: sampled elements."""
    import paper_1701_06446_amd as cum
    from oracle.element import cumulant_at, sample_elements

    n, d, b, t, p = 255, 3, 8, 512, 64
    rows = as_input(_rows(9, t + p, n), "fp32")
    dev = to_device(rows)
    ctx = cum.cum_init(n, d, b, dev[:t], prec="fp32")
    cum.cum_update(ctx, dev[t:t + p], dev[:p])
    window = rows[p:p + t].astype(np.float64)
    rng = np.random.default_rng(1)
    cache = {}
    for k in (2, 3):
        offs, idxs = sample_elements(n, b, k, 40, rng)
        ref = np.array([cumulant_at(window, idx, cache) for idx in idxs])
        g = cum.cum_get(ctx, k)[offs]
        assert np.linalg.norm(g - ref) <= TOL["fp32"] * np.linalg.norm(ref)
    cum.cum_free(ctx)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_bitwise_determinism(prec):
    """No floating-point atomics: two identical runs give identical bits."""
    import paper_1701_06446_amd as cum

    rows = as_input(_rows(4, 3000, 20), prec)
    dev = to_device(rows)
    outs = []
    for _ in range(2):
        ctx = cum.cum_init(20, 4, 4, dev[:2000], prec=prec)
        for w in range(1, 6):
            cum.cum_update(ctx, dev[2000 + (w - 1) * 200:2000 + w * 200], dev[(w - 1) * 200:w * 200])
        outs.append([cum.cum_get(ctx, k) for k in range(1, 5)] + list(cum.cum_norms(ctx)))
        cum.cum_free(ctx)
    for a, c in zip(*outs):
        assert np.array_equal(a, c, equal_nan=True)


def test_integer_data_slide_equals_recompute_fp64():
    """On small-integer data every sum is exact in FP64, so the slid state
    equals the state of a context initialised on the current window, bit for
    bit (Eq. (momupdate) holds exactly)."""
    import paper_1701_06446_amd as cum

    rng = np.random.default_rng(6)
    n, d, b, t, p = 14, 4, 4, 1000, 100
    rows = rng.integers(-4, 5, size=(t + 6 * p, n)).astype(np.float64)
    dev = to_device(rows)
    slid = cum.cum_init(n, d, b, dev[:t], prec="fp64")
    for w in range(1, 7):
        cum.cum_update(slid, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
    fresh = cum.cum_init(n, d, b, dev[6 * p:6 * p + t], prec="fp64")
    for k in range(1, d + 1):
        assert np.array_equal(cum.cum_get_moments(slid, k), cum.cum_get_moments(fresh, k))
    cum.cum_free(slid)
    cum.cum_free(fresh)


def test_memory_cap_gives_enomem(monkeypatch):
    import paper_1701_06446_amd as cum

    monkeypatch.setenv("CUM_DEVICE_MEM_CAP", "1024")
    rows = as_input(_rows(1, 100, 8), "fp32")
    with pytest.raises(cum.CumError) as e:
        cum.cum_init(8, 3, 2, rows, prec="fp32")
    assert e.value.status == cum.CUM_ENOMEM


def test_profile_sampling_counts():
    """cum_profile_sample: only the last of every `every` launches of a class
    is bracketed; every < 1 is rejected; cum_profile_enable resets it."""
    import paper_1701_06446_amd as cum

    rows = as_input(_rows(3, 400 + 9 * 20, 12), "fp32")
    dev = to_device(rows)
    ctx = cum.cum_init(12, 3, 2, dev[:400], prec="fp32")
    cum.cum_profile_enable(ctx, ["update", "combine"], every=3)
    for w in range(1, 8):
        cum.cum_update(ctx, dev[400 + (w - 1) * 20:400 + w * 20], dev[(w - 1) * 20:w * 20])
    prof = cum.cum_profile_read(ctx)
    # 7 launches per class, every 3: the 3rd and the 6th are bracketed
    assert prof["update"][0] == 2 and prof["combine"][0] == 2 and prof["norms"][0] == 0
    assert all(v[1] > 0 for k, v in prof.items() if k != "norms")
    assert cum._lib.cum_profile_sample(ctx.handle, 0) == cum.CUM_EINVAL
    cum.cum_profile_enable(ctx, ["update"])
    cum.cum_update(ctx, dev[540:560], dev[140:160])
    cum.cum_update(ctx, dev[560:580], dev[160:180])
    assert cum.cum_profile_read(ctx)["update"][0] == 2
    cum.cum_free(ctx)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("pipelined", [False, True], ids=["serial", "pipelined"])
def test_norms_carried_by_next_update(prec, pipelined):
    """Serial updates (CUM_PIPELINE=0): a step's norms are finished by the
    next update launch (one extra workgroup) or on demand, so after two
    updates the device buffer holds the first update's norms as that launch
    formed them, and cum_norms then forms and returns the second's.
    Pipelined updates form every step's norms on the side stream right
    after its combine: once the device is idle the buffer holds the second
    update's.  Both against the oracle."""
    import ctypes
    import os

    import torch

    import paper_1701_06446_amd as cum

    n, d, b, t, p = 24, 4, 4, 600, 50
    rows = as_input(_rows(11, t + 2 * p, n), prec)
    dev = to_device(rows)
    old = os.environ.get("CUM_PIPELINE")
    os.environ["CUM_PIPELINE"] = "1" if pipelined else "0"
    try:
        ctx = cum.cum_init(n, d, b, dev[:t], prec=prec)
    finally:
        if old is None:
            os.environ.pop("CUM_PIPELINE", None)
        else:
            os.environ["CUM_PIPELINE"] = old
    ptr = cum.cum_norms_device(ctx)  # the buffer's address does not change
    orc = oracle.SlidingOracle(rows[:t], n, d, b)
    cum.cum_update(ctx, dev[t:t + p], dev[:p])
    orc.update(rows[t:t + p], rows[:p])
    fo1, _ = oracle.norms(orc.cumulants(), n, b)
    cum.cum_update(ctx, dev[t + p:t + 2 * p], dev[p:2 * p])
    orc.update(rows[t + p:t + 2 * p], rows[p:2 * p])
    fo2, _ = oracle.norms(orc.cumulants(), n, b)
    torch.cuda.synchronize()
    host = np.zeros(2 * (d + 1), np.float64)
    hip = ctypes.CDLL("libamdhip64.so")
    assert hip.hipMemcpy(ctypes.c_void_p(host.ctypes.data), ctypes.c_void_p(ptr),
                         ctypes.c_size_t(host.nbytes), 2) == 0  # device to host
    tol = max(TOL[prec], 1e-12)
    np.testing.assert_allclose(host[1:d + 1], (fo2 if pipelined else fo1)[1:], rtol=tol)
    fro, nu = cum.cum_norms(ctx)
    np.testing.assert_allclose(fro[1:], fo2[1:], rtol=tol)
    cum.cum_free(ctx)


def test_inputs_switching_between_allocations():
    """The library remembers the device allocation the last rows came from
    and skips the pointer query for rows inside it: rows from that tensor,
    then host rows, rows from a second device tensor, rows whose X_old lies
    in another allocation than X_new, and the first tensor again, every step
    against the oracle."""
    import paper_1701_06446_amd as cum

    n, d, b, t, p = 12, 4, 4, 300, 40
    rows = as_input(_rows(11, t + 6 * p, n), "fp64")
    a = to_device(rows)
    bdev = to_device(rows.copy())
    ctx = cum.cum_init(n, d, b, a[:t], prec="fp64")
    orc = oracle.SlidingOracle(rows[:t], n, d, b)
    sources = [(a, a), (rows, rows), (bdev, bdev), (a, bdev), (bdev, a), (a, a)]
    for w, (sn, so) in enumerate(sources, start=1):
        new, old = slice(t + (w - 1) * p, t + w * p), slice((w - 1) * p, w * p)
        cum.cum_update(ctx, sn[new], so[old])
        orc.update(rows[new], rows[old])
        Co = orc.cumulants()
        errs = [rel_err(cum.cum_get(ctx, k), Co[k - 1], n, b, k) for k in range(2, d + 1)]
        assert max(errs) <= TOL["fp64"], (w, errs)
    cum.cum_free(ctx)
