"""Choice of the block size b per stream shape.

The block size trades redundant work in diagonal blocks and ragged update
tiles (larger b) against per-block combine work (smaller b), and the best
value depends on the order (the paper's block-size sweep, Sec. 3.2).

``choose_b`` is deterministic: it minimises a cost model of one sliding
update of the stream as a member of a batched step, computed on the host from
the library's own launch plan,

    cost(b) = 2p * F(b) * PER_FRAG_ROW[prec] + N_d(b) * PER_BLOCK[d][b],

F(b) the 16x16 output fragments of the update launch (``cum_plan_groups``)
and N_d(b) the order-d blocks (the fused combine runs one wave per block).
The constants were measured once on MI355X: update and combine kernel times
of single contexts over n = 16..96, d = 3, 4, b = 2, 4, 8 and p = 100, 1000
(the marginal time per fragment-row of the largest updates and per block of
the largest combines).  In a batch the members' launches are packed
together, so the marginal costs, not single-launch latencies, decide.

``choose_b_measured`` keeps the measure-and-cache variant: it times a few
updates of every candidate with the library's event profiler (its choice can
flip between runs where two candidates are close).  Throughput figures for
autotuned streams should be counted against the b-independent element count
sum_k C(n+k-1, k), so that a larger b (more redundant products) cannot
inflate them.
"""
from __future__ import annotations

import json
import os
from math import comb

import numpy as np

CANDIDATES = (2, 4, 8)


def cache_path() -> str:
    return os.environ.get("CUM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "cumstream_autotune.json"))


def _arch() -> str:
    import torch

    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name)


def _key(arch, n, d, t, p, prec) -> str:
    return "%s|n=%d|d=%d|t=%d|p=%d|%s" % (arch, n, d, t, p, prec)


def load_cache(path=None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path=None):
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def distinct_elements(n: int, d: int) -> int:
    """b-independent size of orders 1..d: sum_k C(n+k-1, k)."""
    return sum(comb(n + k - 1, k) for k in range(1, d + 1))


def candidates(n: int, prec: str):
    return [b for b in CANDIDATES if b <= n] or [1]


def time_update(n, d, b, t, p, prec, reps=12, seed=0) -> float:
    """Mean update time (ms) of one context of this shape on the device."""
    import torch

    import paper_1701_06446_amd as cum

    dt = np.float64 if prec == "fp64" else np.float32
    rows = np.random.default_rng(seed).standard_normal((t + (reps + 1) * p, n)).astype(dt)
    dev = torch.from_numpy(rows).to("cuda")
    ctx = cum.cum_init(n, d, b, dev[:t], prec=prec)
    cum.cum_update(ctx, dev[t:t + p], dev[:p])  # warm-up
    cum.cum_profile_enable(ctx, True)
    for w in range(2, reps + 2):
        cum.cum_update(ctx, dev[t + (w - 1) * p:t + w * p], dev[(w - 1) * p:w * p])
    prof = cum.cum_profile_read(ctx)
    cum.cum_free(ctx)
    return sum(ms for _, ms in prof.values()) / reps


# marginal seconds per (16x16 fragment x signed row) of the update launch
PER_FRAG_ROW = {"fp32": 6.9e-12, "bf16x3": 6.6e-12, "fp64": 12.9e-12}
# marginal seconds per order-d block of the combine (d <= 4: the fused lattice
# combine, one wave per block; b = 8 at d = 4 stages 52 KB per block and runs
# few waves per CU; d >= 5: the per-order combines)
PER_BLOCK = {
    1: {1: 0.1e-9, 2: 0.1e-9, 4: 0.1e-9, 8: 0.1e-9},
    2: {1: 0.2e-9, 2: 0.2e-9, 4: 0.3e-9, 8: 0.5e-9},
    3: {1: 0.3e-9, 2: 0.3e-9, 4: 0.5e-9, 8: 2.0e-9},
    4: {1: 0.6e-9, 2: 0.64e-9, 4: 1.03e-9, 8: 33e-9},
    5: {1: 2e-9, 2: 2e-9, 4: 5e-9, 8: 300e-9},
    6: {1: 5e-9, 2: 5e-9, 4: 50e-9, 8: 1e-6},
}


def model_cost(n, d, b, p, prec="fp32") -> float:
    """Modelled seconds of one sliding update of p rows (both the new and the
    leaving rows contracted) plus its combine, as a batch member."""
    import paper_1701_06446_amd as cum

    frags, _ = cum.cum_plan_groups(n, d, b)
    return 2 * p * int(frags.sum()) * PER_FRAG_ROW[prec] + cum.cum_num_blocks(n, b, d) * PER_BLOCK[d][b]


PREFERRED = 4     # the default block size, kept unless another is clearly cheaper
MARGIN = 0.10     # "clearly": by more than this fraction of the modelled cost


def choose_b(n, d, t, p, prec="fp32") -> int:
    """The candidate with the least modelled cost (ties: the smaller b), or
    PREFERRED when it is within MARGIN of that; deterministic, no device
    work.  t does not enter: the update and the combine do not depend on the
    window length."""
    costs = {b: model_cost(n, d, b, p, prec) for b in candidates(n, prec)}
    best = min(sorted(costs), key=lambda b: costs[b])
    if PREFERRED in costs and costs[PREFERRED] <= (1 + MARGIN) * costs[best]:
        return PREFERRED
    return best


def choose_b_measured(n, d, t, p, prec="fp32", cache=None, timer=time_update, arch=None) -> int:
    """The fastest candidate block size for this shape by measurement (cached)."""
    own = cache is None
    cache = load_cache() if own else cache
    arch = arch or _arch()
    key = _key(arch, n, d, t, p, prec)
    if key in cache:
        return int(cache[key]["b"])
    times = {b: timer(n, d, b, t, p, prec) for b in candidates(n, prec)}
    best = min(times, key=times.get)
    cache[key] = {"b": best, "ms": {str(k): v for k, v in times.items()}}
    if own:
        save_cache(cache)
    return best
