"""Pins of the FP64 oracle against things other than itself: brute force on
tiny inputs, textbook closed forms, the paper's worked d=3 example and counting
formulas, scipy's univariate statistics, exact invariants and the Exp(1)
closed form.  No GPU."""
import itertools
import math
import os

import numpy as np
import pytest
from scipy import stats

import oracle
from oracle.full import pack, unpack
from tests.noise_floor import gaussian_noise_floor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def int_rows(rng, t, n, lo=-3, hi=4):
    return rng.integers(lo, hi, size=(t, n)).astype(np.float64)


# ---------------------------------------------------------------------------
# block structure and partitions


@pytest.mark.parametrize("n,b,k", [(5, 2, 3), (6, 1, 4), (7, 3, 2), (20, 2, 4), (60, 4, 4), (48, 4, 6)])
def test_block_counts_and_order(n, b, k):
    nbar = -(-n // b)
    assert oracle.nblocks(n, b, k) == math.comb(nbar + k - 1, k)
    if math.comb(nbar + k - 1, k) < 5000:
        want = list(itertools.combinations_with_replacement(range(nbar), k))
        got = [tuple(r) for r in oracle.tuples(n, b, k)]
        assert got == want


def stirling2(s, k):
    # S(s,k) = k S(s-1,k) + S(s-1,k-1)
    S = [[0] * (s + 1) for _ in range(s + 1)]
    S[0][0] = 1
    for i in range(1, s + 1):
        for j in range(1, i + 1):
            S[i][j] = j * S[i - 1][j] + S[i - 1][j - 1]
    return S[s][k]


@pytest.mark.parametrize("s", [1, 2, 3, 4, 5, 6])
def test_partition_counts(s):
    """Partitions into sigma parts are the Stirling numbers S(s, sigma); their
    sum is the Bell number (Eq. (n1) and the text after it)."""
    bell = [1, 1, 2, 5, 15, 52, 203][s]
    tot = 0
    for sigma in range(1, s + 1):
        c = oracle.count_partitions(s, sigma)
        assert c == stirling2(s, sigma)
        tot += c
    assert tot == bell


def test_multiplication_count_eq_n1():
    """Eq. (n1): sum_sigma S(d, sigma)(sigma - 1) < (d - 1) B(d); 22 for d = 4,
    471 for d = 6 (counted from the oracle's partition lists)."""
    for d, want in ((4, 22), (6, 471)):
        cnt = sum(oracle.count_partitions(d, s) * (s - 1) for s in range(2, d + 1))
        assert cnt == want
        assert cnt < (d - 1) * [1, 1, 2, 5, 15, 52, 203][d]


# ---------------------------------------------------------------------------
# moments


def brute_moment(X, k):
    """m_i = (1/t) sum_l prod_m x[l, i_m] for every i in n^k (Eq. (mom))."""
    t, n = X.shape
    M = np.zeros((n,) * k)
    for i in itertools.product(range(n), repeat=k):
        p = np.ones(t)
        for m in i:
            p = p * X[:, m]
        M[i] = p.sum() / t
    return M


@pytest.mark.parametrize("n,d,b", [(4, 4, 1), (5, 3, 2), (5, 4, 2), (6, 3, 3), (4, 2, 3), (3, 5, 2)])
def test_moments_brute_force_integer_exact(n, d, b):
    rng = np.random.default_rng(1 + n * 10 + d + 100 * b)
    X = int_rows(rng, 40, n)
    Ms = oracle.moments_of(X, n, d, b)
    for k in range(1, d + 1):
        # integer data: sums are exact, so the division by t is the only rounding
        assert np.array_equal(unpack(Ms[k - 1], n, b, k), brute_moment(X, k))


def test_padding_entries_exactly_zero():
    n, b, d = 5, 2, 3
    rng = np.random.default_rng(3)
    X = rng.standard_normal((50, n))
    o = oracle.SlidingOracle(X, n, d, b)
    for k, C in enumerate(o.cumulants(), start=1):
        tl = oracle.tuples(n, b, k)
        for r, j in enumerate(tl):
            for e, a in enumerate(itertools.product(range(b), repeat=k)):
                if any(jm * b + am >= n for jm, am in zip(j, a)):
                    assert C[r * b ** k + e] == 0.0


def test_sliding_equals_recompute_bitwise_integer():
    """Eq. (momupdate) is an identity: on integer data (all sums exact) the
    slid sums equal the recomputed window's sums bit for bit."""
    n, d, b, t, p = 6, 4, 2, 60, 7
    rng = np.random.default_rng(11)
    rows = int_rows(rng, t + 9 * p, n)
    o = oracle.SlidingOracle(rows[:t], n, d, b)
    for w in range(1, 10):
        o.update(rows[t + (w - 1) * p: t + w * p], rows[(w - 1) * p: w * p])
        ref = oracle.SlidingOracle(rows[w * p: w * p + t], n, d, b)
        for a, c in zip(o.sums(), ref.sums()):
            assert np.array_equal(a, c)


def test_sliding_matches_recompute_real_data():
    n, d, b, t, p = 7, 4, 3, 500, 50
    rng = np.random.default_rng(12)
    rows = rng.standard_normal((t + 12 * p, n)) * 3 + 1
    o = oracle.SlidingOracle(rows[:t], n, d, b)
    for w in range(1, 13):
        o.update(rows[t + (w - 1) * p: t + w * p], rows[(w - 1) * p: w * p])
    ref = oracle.SlidingOracle(rows[12 * p: 12 * p + t], n, d, b)
    for k, (a, c) in enumerate(zip(o.cumulants(), ref.cumulants()), start=1):
        assert oracle.block_norm(a - c, n, b, k) <= 1e-13 * oracle.block_norm(c, n, b, k)


# ---------------------------------------------------------------------------
# combine (Alg. 3/4)


def full_cumulants(X, n, d, b):
    o = oracle.SlidingOracle(X, n, d, b)
    return [unpack(C, n, b, k) for k, C in enumerate(o.cumulants(), start=1)]


def test_worked_example_d3():
    """The paper's worked third-order example (Sec. 2.6):
    c_{123} = m_{123} - c_{12} c_3 - c_{13} c_2 - c_{23} c_1 - c_1 c_2 c_3."""
    with open(os.path.join(GOLDEN, "worked_d3.txt")) as f:
        terms = [l.split() for l in f if l.strip() and not l.startswith("#")]
    n, b = 4, 1
    rng = np.random.default_rng(5)
    X = rng.standard_normal((300, n)) + 0.7
    o = oracle.SlidingOracle(X, n, 3, b)
    M3 = unpack(o.moments()[2], n, b, 3)
    C1, C2, C3 = [unpack(C, n, b, k) for k, C in enumerate(o.cumulants(), start=1)]
    for i in itertools.product(range(n), repeat=3):
        val = M3[i]
        for sign, *parts in terms:
            prod = 1.0
            for part in parts:
                idx = tuple(i[int(c) - 1] for c in part)
                prod *= {1: C1, 2: C2}[len(idx)][idx]
            val += float(sign) * prod
        assert abs(val - C3[i]) <= 1e-13 * (1 + abs(C3[i]))


@pytest.mark.parametrize("n,b", [(4, 1), (5, 2), (4, 3)])
def test_closed_forms_orders_2_3_4(n, b):
    """C2 = biased covariance, C3 = third central moment,
    C4 = mu4 - (mu2(x)mu2 + two transpositions)."""
    rng = np.random.default_rng(7 + n + b)
    X = rng.standard_normal((400, n)) @ rng.standard_normal((n, n)) + rng.standard_normal(n)
    C1, C2, C3, C4 = full_cumulants(X, n, 4, b)
    Y = X - X.mean(0)
    t = X.shape[0]
    assert np.allclose(C1, X.mean(0), rtol=0, atol=1e-13 * np.abs(X).max())
    assert np.allclose(C2, np.cov(X.T, bias=True), rtol=1e-12, atol=1e-12)
    mu3 = np.einsum("li,lj,lk->ijk", Y, Y, Y) / t
    assert np.allclose(C3, mu3, rtol=1e-10, atol=1e-11)
    mu2 = Y.T @ Y / t
    mu4 = np.einsum("li,lj,lk,lm->ijkm", Y, Y, Y, Y) / t
    c4 = mu4 - (np.einsum("ij,km->ijkm", mu2, mu2) + np.einsum("ik,jm->ijkm", mu2, mu2)
                + np.einsum("im,jk->ijkm", mu2, mu2))
    assert np.allclose(C4, c4, rtol=1e-9, atol=1e-9)


def set_partitions(elems):
    """All set partitions of a list, by inserting the first element into every
    part of every partition of the rest (a different construction from the
    oracle's restricted growth strings)."""
    if not elems:
        yield []
        return
    first, rest = elems[0], elems[1:]
    for part in set_partitions(rest):
        yield [[first]] + part
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]


@pytest.mark.parametrize("d,n,b", [(4, 3, 2), (5, 3, 1), (6, 2, 1)])
def test_moebius_formula(d, n, b):
    """Cumulants from raw moments by the Moebius inversion over the partition
    lattice, c = sum_pi (-1)^(|pi|-1) (|pi|-1)! prod_B m_B, agree with Alg. 4."""
    rng = np.random.default_rng(20 + d)
    X = rng.exponential(1.0, (200, n)) + 0.3 * rng.standard_normal((200, n))
    o = oracle.SlidingOracle(X, n, d, b)
    Ms = [unpack(M, n, b, k) for k, M in enumerate(o.moments(), start=1)]
    Cd = unpack(o.cumulants()[d - 1], n, b, d)
    parts = list(set_partitions(list(range(d))))
    assert len(parts) == [1, 1, 2, 5, 15, 52, 203][d]
    for i in itertools.product(range(n), repeat=d):
        c = 0.0
        for pi in parts:
            q = len(pi)
            prod = 1.0
            for B in pi:
                prod *= Ms[len(B) - 1][tuple(i[m] for m in B)]
            c += (-1) ** (q - 1) * math.factorial(q - 1) * prod
        assert abs(c - Cd[i]) <= 1e-11 * (1 + abs(Cd[i]))


def test_recursion_on_block_containing_first_index():
    """c = m - sum over blocks B containing the first index (B != all) of
    c_B * m_(complement): a third formula for the same cumulant."""
    d, n, b = 5, 3, 2
    rng = np.random.default_rng(33)
    X = rng.gamma(2.0, 1.0, (150, n))
    o = oracle.SlidingOracle(X, n, d, b)
    Ms = [unpack(M, n, b, k) for k, M in enumerate(o.moments(), start=1)]
    Cs = [unpack(C, n, b, k) for k, C in enumerate(o.cumulants(), start=1)]
    for i in itertools.product(range(n), repeat=d):
        acc = Ms[d - 1][i]
        for r in range(0, d - 1):
            for rest in itertools.combinations(range(1, d), r):
                B = (0,) + rest
                comp = [m for m in range(d) if m not in B]
                acc -= Cs[len(B) - 1][tuple(i[m] for m in B)] * Ms[len(comp) - 1][tuple(i[m] for m in comp)]
        assert abs(acc - Cs[d - 1][i]) <= 1e-11 * (1 + abs(acc))


def test_univariate_scipy_and_closed_forms():
    """n = 1: nu_3 = |skewness| and nu_4 = |excess kurtosis| (Sec. 4.1);
    kappa_5 = mu5 - 10 mu3 mu2 and kappa_6 = mu6 - 15 mu4 mu2 - 10 mu3^2 + 30 mu2^3."""
    rng = np.random.default_rng(9)
    x = rng.gamma(3.0, 1.0, 5000) - 1.0
    o = oracle.SlidingOracle(x[:, None], 1, 6, 1)
    C = [c[0] for c in o.cumulants()]
    fro, nu = o.norms()
    assert abs(nu[3] - abs(stats.skew(x, bias=True))) < 1e-12
    assert abs(nu[4] - abs(stats.kurtosis(x, fisher=True, bias=True))) < 1e-12
    y = x - x.mean()
    mu = [np.mean(y ** k) for k in range(7)]
    assert abs(C[4] - (mu[5] - 10 * mu[3] * mu[2])) < 1e-10 * abs(mu[5])
    k6 = mu[6] - 15 * mu[4] * mu[2] - 10 * mu[3] ** 2 + 30 * mu[2] ** 3
    assert abs(C[5] - k6) < 1e-10 * abs(mu[6])


def test_exp1_closed_form():
    """Exp(1) has kappa_k = (k - 1)!; the estimates lie within a few standard
    errors sqrt(m_2k / t) (Sec. 4.3) of it."""
    rng = np.random.default_rng(17)
    t = 400_000
    x = rng.exponential(1.0, t)
    C = [c[0] for c in oracle.SlidingOracle(x[:, None], 1, 4, 1).cumulants()]
    for k in (1, 2, 3, 4):
        se = math.sqrt(math.factorial(2 * k) / t)
        assert abs(C[k - 1] - math.factorial(k - 1)) < 6 * se, (k, C[k - 1])


def test_gaussian_higher_cumulants_vanish():
    """Gaussian windows: ||C_3||, ||C_4|| shrink like t^(-1/2) relative to the
    covariance scale, so nu_3, nu_4 are small (Sec. 4.1)."""
    rng = np.random.default_rng(19)
    n, t = 4, 200_000
    A = rng.standard_normal((n, n))
    X = rng.standard_normal((t, n)) @ A.T + 2.0
    fro, nu = oracle.SlidingOracle(X, n, 4, 2).norms()
    assert nu[3] < 0.05 and nu[4] < 0.05, nu


def test_gaussian_norms_match_the_noise_floor():
    """||C_3||^2 and ||C_4||^2 of Gaussian windows (Alg. 4 then Alg. 5 over
    the full tensor, Eq. (me)) average to the closed-form sampling noise of
    gaussian_noise_floor; nu_4 (Eq. (mef)) to sqrt of that over ||S||_F^2.
    A dropped or mis-signed pair term of Alg. 4 leaves a mean of the size of
    S x S in C_4 (far above the floor), and a wrong block multiplicity in
    Alg. 5 scales the norm by up to k!.  32 windows: the relative standard
    error of the mean ratio is about 2.5 % (k=3) and 1 % (k=4)."""
    import streams

    n, t, runs = 12, 20000, 32
    S = streams.covariance(streams.rng_for(11), n)
    E3, E4 = gaussian_noise_floor(S, t, 3), gaussian_noise_floor(S, t, 4)
    r3, r4, v4 = [], [], []
    for run in range(runs):
        X = streams.gaussian_rows(streams.rng_for(11, run + 1), t, S) + 0.7
        fro, nu = oracle.SlidingOracle(X, n, 4, 4).norms()
        r3.append(fro[3] ** 2 / E3)
        r4.append(fro[4] ** 2 / E4)
        v4.append(nu[4])
    assert abs(np.mean(r3) - 1) < 0.10, np.mean(r3)
    assert abs(np.mean(r4) - 1) < 0.04, np.mean(r4)
    assert abs(np.mean(v4) / (math.sqrt(E4) / np.sum(S * S)) - 1) < 0.04


# ---------------------------------------------------------------------------
# norms (Alg. 5) and invariants


@pytest.mark.parametrize("n,b,k", [(5, 1, 3), (5, 2, 3), (7, 3, 4), (4, 3, 2), (6, 2, 4), (3, 2, 5)])
def test_block_norm_equals_full_norm(n, b, k):
    rng = np.random.default_rng(n * 100 + b * 10 + k)
    X = rng.standard_normal((80, n)) + 0.5
    C = oracle.SlidingOracle(X, n, k, b).cumulants()[k - 1]
    assert abs(oracle.block_norm(C, n, b, k) - np.linalg.norm(unpack(C, n, b, k).ravel())) \
        <= 1e-13 * np.linalg.norm(unpack(C, n, b, k).ravel())


def test_pack_unpack_roundtrip_and_supersymmetry():
    """Moments of integer data are exact, so every stored moment equals the one
    at its sorted index bit for bit; cumulants of a diagonal block sum the same
    partition products in another order, so they agree to a few ulps."""
    n, b, k = 5, 2, 4
    rng = np.random.default_rng(2)
    X = int_rows(rng, 30, n)
    o = oracle.SlidingOracle(X, n, k, b)
    M = o.moments()[k - 1]
    C = o.cumulants()[k - 1]
    assert np.array_equal(pack(unpack(M, n, b, k), n, b, k), M)
    Cr = pack(unpack(C, n, b, k), n, b, k)
    assert np.max(np.abs(Cr - C)) <= 1e-14 * np.max(np.abs(C))
    Tm, Tc = unpack(M, n, b, k), unpack(C, n, b, k)
    tl = oracle.tuples(n, b, k)
    for r, j in enumerate(tl):
        for e, a in enumerate(itertools.product(range(b), repeat=k)):
            i = tuple(int(jm) * b + am for jm, am in zip(j, a))
            if all(v < n for v in i):
                assert M[r * b ** k + e] == Tm[tuple(sorted(i))]
                assert abs(C[r * b ** k + e] - Tc[tuple(sorted(i))]) <= 1e-14 * np.max(np.abs(C))


def test_scaling_bitwise():
    """C_k(2X) = 2^k C_k(X) exactly (powers of two scale without rounding)."""
    n, d, b = 5, 4, 2
    rng = np.random.default_rng(4)
    X = rng.standard_normal((64, n))
    a = oracle.SlidingOracle(X, n, d, b).cumulants()
    c = oracle.SlidingOracle(2 * X, n, d, b).cumulants()
    for k in range(1, d + 1):
        assert np.array_equal(c[k - 1], a[k - 1] * 2.0 ** k)


def test_padding_is_exact_b_not_dividing_n():
    n, d = 5, 4
    rng = np.random.default_rng(8)
    X = rng.standard_normal((90, n))
    for k, (c1, c2) in enumerate(zip(full_cumulants(X, n, d, 1), full_cumulants(X, n, d, 3)), start=1):
        assert np.allclose(c1, c2, rtol=1e-12, atol=1e-14)


def test_shift_orthogonal_and_permutation():
    n, d, b = 4, 4, 2
    rng = np.random.default_rng(10)
    X = rng.exponential(1.0, (300, n))
    base = oracle.SlidingOracle(X, n, d, b)
    fro0, _ = base.norms()
    shifted, _ = oracle.SlidingOracle(X + np.array([3.0, -1.0, 0.5, 2.0]), n, d, b).norms()
    assert np.allclose(shifted[2:], fro0[2:], rtol=1e-9)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    rot, _ = oracle.SlidingOracle(X @ Q, n, d, b).norms()
    assert np.allclose(rot[1:], fro0[1:], rtol=1e-11)
    perm = [2, 0, 3, 1]
    Cb = full_cumulants(X, n, d, b)
    Cp = full_cumulants(X[:, perm], n, d, b)
    for k in range(1, d + 1):
        assert np.allclose(Cp[k - 1], Cb[k - 1][np.ix_(*([perm] * k))], rtol=1e-12, atol=1e-14)


def test_element_oracle_matches_pyramid_oracle():
    """The per-element route (numpy, one multi-index at a time) and the C
    pyramid oracle agree; the C oracle is pinned above, this pins the sampler
    used for full-size checks."""
    from oracle.element import cumulant_at, sample_elements

    n, d, b = 7, 4, 3
    rng = np.random.default_rng(40)
    X = rng.exponential(1.0, (500, n)) - 0.5
    C = oracle.SlidingOracle(X, n, d, b).cumulants()
    cache = {}
    for k in range(1, d + 1):
        offs, idxs = sample_elements(n, b, k, 25, rng)
        for o, idx in zip(offs, idxs):
            assert abs(C[k - 1][o] - cumulant_at(X, idx, cache)) <= 1e-12 * (1 + abs(C[k - 1][o]))


def test_indices_of_inverts_sample_elements():
    """The offset -> multi-index map agrees with the sampler's own pairs, and
    padded elements map to None (n = 13, b = 4: columns 13..15 are padding)."""
    from oracle.element import indices_of, sample_elements

    rng = np.random.default_rng(0)
    for n, b, k in [(13, 4, 3), (9, 2, 4), (6, 3, 2)]:
        offs, idxs = sample_elements(n, b, k, 30, rng)
        assert indices_of(n, b, k, offs) == idxs
    import oracle

    # order 2, n = 13, b = 4: blocks (j1 <= j2) of 16 elements; the
    # elements with both indices < 13 are 13 * 13 minus the lower triangle
    # of the off-diagonal blocks: sum over j1 < j2 of rows(j1) * rows(j2)
    rows = [4, 4, 4, 1]
    want = sum(rows[j] * rows[j] for j in range(4)) + sum(rows[i] * rows[j] for i in range(4) for j in range(i + 1, 4))
    got = indices_of(13, 4, 2, range(oracle.pyramid_size(13, 4, 2)))
    assert sum(1 for g in got if g is not None) == want


def test_student_t_lower_tail_closed_form():
    """The stream study's even-nu Student-t CDF (closed form) against
    scipy's, in the range its samples fall in."""
    import torch
    from scipy import stats

    import streams

    t = torch.linspace(0.0, 10.0, 501, dtype=torch.float64)
    for nu in (2, 4, 10):
        got = streams._student_t_cdf_lower(t, nu).numpy()
        ref = stats.t.cdf(-t.numpy(), nu)
        assert np.max(np.abs(got - ref) / ref) < 1e-9, nu
