"""Autotuner logic (no GPU): candidate sets, the deterministic cost-model
choice, and the measured variant's choice of the fastest and its cache."""
from math import comb


def test_candidates_and_distinct_elements():
    from paper_1701_06446_amd import autotune

    assert autotune.candidates(96, "fp32") == [2, 4, 8]
    assert autotune.candidates(6, "fp32") == [2, 4]
    assert autotune.candidates(1, "fp32") == [1]
    assert autotune.distinct_elements(60, 4) == sum(comb(60 + k - 1, k) for k in range(1, 5))


def test_measured_choice_picks_fastest_and_caches(tmp_path):
    from paper_1701_06446_amd import autotune

    calls = []

    def fake_timer(n, d, b, t, p, prec):
        calls.append(b)
        return {2: 3.0, 4: 1.5, 8: 2.0}[b]

    cache = {}
    assert autotune.choose_b_measured(40, 4, 2000, 100, "fp32", cache=cache, timer=fake_timer, arch="gfx950") == 4
    assert sorted(calls) == [2, 4, 8]
    assert autotune.choose_b_measured(40, 4, 2000, 100, "fp32", cache=cache, timer=fake_timer, arch="gfx950") == 4
    assert len(calls) == 3  # second call served from the cache
    path = tmp_path / "tune.json"
    autotune.save_cache(cache, str(path))
    assert autotune.load_cache(str(path)) == cache


def test_model_choice_is_deterministic_and_the_argmin():
    """choose_b is the argmin of model_cost over the candidates, or the
    preferred b = 4 within the margin (the launch plan is host-only), the
    same on every call; at d = 4 and large n the
    many 16-element blocks of b = 2 and the 52 KB lattice of b = 8 lose to
    b = 4."""
    from paper_1701_06446_amd import autotune

    for n, d, p in [(96, 4, 730), (80, 4, 68), (48, 3, 400), (16, 3, 100), (64, 4, 1000)]:
        costs = {b: autotune.model_cost(n, d, b, p) for b in autotune.candidates(n, "fp32")}
        best = autotune.choose_b(n, d, 20 * p, p)
        assert costs[best] == min(costs.values()) or (
            best == autotune.PREFERRED and costs[best] <= (1 + autotune.MARGIN) * min(costs.values()))
        assert all(autotune.choose_b(n, d, 20 * p, p) == best for _ in range(3))
    assert autotune.choose_b(96, 4, 14600, 730) == 4
    assert autotune.choose_b(80, 4, 1360, 68) == 4
