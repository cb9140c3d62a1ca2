"""Autotuner logic (no GPU): candidate sets, choice of the fastest, caching."""
from math import comb


def test_candidates_and_distinct_elements():
    from paper_1701_06446_amd import autotune

    assert autotune.candidates(96, "fp32") == [2, 4, 8]
    assert autotune.candidates(6, "fp32") == [2, 4]
    assert autotune.candidates(1, "fp32") == [1]
    assert autotune.distinct_elements(60, 4) == sum(comb(60 + k - 1, k) for k in range(1, 5))


def test_choose_b_picks_fastest_and_caches(tmp_path):
    from paper_1701_06446_amd import autotune

    calls = []

    def fake_timer(n, d, b, t, p, prec):
        calls.append(b)
        return {2: 3.0, 4: 1.5, 8: 2.0}[b]

    cache = {}
    assert autotune.choose_b(40, 4, 2000, 100, "fp32", cache=cache, timer=fake_timer, arch="gfx950") == 4
    assert sorted(calls) == [2, 4, 8]
    assert autotune.choose_b(40, 4, 2000, 100, "fp32", cache=cache, timer=fake_timer, arch="gfx950") == 4
    assert len(calls) == 3  # second call served from the cache
    path = tmp_path / "tune.json"
    autotune.save_cache(cache, str(path))
    assert autotune.load_cache(str(path)) == cache
