"""Host-side checks of the C-ABI (no GPU): every symbol include/cum.h declares
is exported, the host-only planning calls are right, and argument validation
rejects bad calls before touching the device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    with open(os.path.join(ROOT, "include", "cum.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cum_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    import paper_1701_06446_amd as cum

    lib = ctypes.CDLL(cum.LIB_PATH)
    names = declared_symbols()
    assert "cum_init" in names and "cum_update" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) <= set(cum.EXPORTS)


@pytest.mark.parametrize("n,b,k", [(20, 2, 4), (60, 4, 4), (48, 4, 6), (7, 3, 5), (5, 5, 3), (13, 4, 2), (9, 1, 3)])
def test_num_blocks_closed_form(n, b, k):
    import paper_1701_06446_amd as cum

    nbar = -(-n // b)
    assert cum.cum_num_blocks(n, b, k) == math.comb(nbar + k - 1, k)
    assert cum.cum_num_elems(n, b, k) == math.comb(nbar + k - 1, k) * b ** k


@pytest.mark.parametrize("n,b,k", [(20, 2, 4), (60, 4, 4), (7, 3, 3), (5, 2, 5), (9, 2, 6), (6, 1, 4), (13, 4, 3),
                                   (11, 4, 1), (11, 4, 2), (3, 3, 6)])
def test_pivot_decomposition_covers_each_element_once(n, b, k):
    """Every stored order-k element is produced by exactly one (pivot, row,
    column) product of the update, with matching global indices."""
    import paper_1701_06446_amd as cum

    bad, hits = cum.cum_plan_coverage(n, b, k)
    assert bad == 0
    assert hits.min() == 1 and hits.max() == 1


def test_plan_items_counts_tiles():
    import paper_1701_06446_amd as cum

    # n=60, b=4: every pivot GEMM tiled by 32x32 outputs
    nbar = 15
    total = 0
    for k in range(1, 5):
        h = (k + 1) // 2
        m = k - h
        for v in range(nbar):
            rows = math.comb(v + h - 1, h - 1) * 4 ** h
            cols = (math.comb(nbar - v + m - 1, m) if m else 1) * 4 ** m
            total += -(-rows // 32) * -(-cols // 32)
    assert cum.cum_plan_items(60, 4, 4) == total


def test_validation_without_device():
    import paper_1701_06446_amd as cum

    X = np.zeros((10, 5), np.float32)
    for kwargs in ({"n": 5, "d": 7, "b": 1}, {"n": 5, "d": 0, "b": 1}, {"n": 5, "d": 3, "b": 0},
                   {"n": 5, "d": 3, "b": 6}, {"n": 256, "d": 2, "b": 1}):
        Xk = np.zeros((10, kwargs["n"]), np.float32)
        with pytest.raises(cum.CumError) as e:
            cum.cum_init(kwargs["n"], kwargs["d"], kwargs["b"], Xk)
        assert e.value.status == cum.CUM_EINVAL
    with pytest.raises(cum.CumError) as e:
        cum.cum_init(5, 3, 1, X, prec=7)
    assert e.value.status == cum.CUM_EINVAL
    lib = cum._lib
    assert lib.cum_update(None, None, None, 1) == cum.CUM_EINVAL
    assert lib.cum_get(None, 1, None, 0) == cum.CUM_EINVAL
    assert lib.cum_free(None) == cum.CUM_OK
    assert lib.cum_num_blocks(0, 1, 1) == -1
    assert lib.cum_strerror(cum.CUM_ESIZE).decode().startswith("size")


def test_dtype_mismatch_is_rejected_by_binding():
    import paper_1701_06446_amd as cum

    with pytest.raises(ValueError):
        cum.cum_init(5, 3, 1, np.zeros((10, 5), np.float64), prec="fp32")
    with pytest.raises(ValueError):
        cum.cum_init(5, 3, 1, np.zeros((10, 4), np.float32), prec="fp32")


def _pivot_dims(n, d, b):
    nbar = -(-n // b)
    for k in range(1, d + 1):
        h = (k + 1) // 2
        m = k - h
        for v in range(nbar):
            rows = math.comb(v + h - 1, h - 1) * b ** h
            cols = (math.comb(nbar - v + m - 1, m) if m else 1) * b ** m
            yield rows, cols


@pytest.mark.parametrize("n,d,b", [(60, 4, 4), (32, 4, 4), (48, 6, 4), (20, 4, 2), (13, 3, 3)])
def test_four_tile_packing(n, d, b):
    """Every 32x32 tile lands in exactly one four-tile workgroup, each
    multiplies exactly its 16x16 fragments inside the pivot GEMM, and the
    dearest workgroup stays within one tile (4 fragments) of the average."""
    import paper_1701_06446_amd as cum

    frags, tiles = cum.cum_plan_groups(n, d, b)
    items = cum.cum_plan_items(n, d, b)
    want = sum(-(-r // 16) * -(-c // 16) for r, c in _pivot_dims(n, d, b))
    assert len(frags) == -(-items // 4)
    assert tiles.sum() == items and tiles.max() <= 4
    assert frags.sum() == want
    assert frags.max() <= -(-want // len(frags)) + 3
