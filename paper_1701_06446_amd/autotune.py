"""Measure-and-cache choice of the block size b per stream shape.

The block size trades redundant work in diagonal blocks (larger b) against
per-block overhead (smaller b), and the best value falls as the order grows
(the paper's block-size sweep, Sec. 3.2).  ``choose_b`` times a few updates of
every candidate on the device with the library's own event profiler and keeps
the fastest; results are cached in a JSON file keyed by GPU architecture and
(n, d, t, p, precision).  Throughput figures for autotuned streams should be
counted against the b-independent element count sum_k C(n+k-1, k), so that a
larger b (more redundant products) cannot inflate them.
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


def choose_b(n, d, t, p, prec="fp32", cache=None, timer=time_update, arch=None) -> int:
    """The fastest candidate block size for this shape (cached)."""
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
