"""Seeded synthetic data streams (rows = samples, columns = marginals).

This module only draws random numbers: it holds none of the cumulant method's
arithmetic, and both the HIP path and the oracle read the arrays it returns.

Every generator is numpy ``Generator(PCG64)`` seeded with
``SeedSequence([170106446, workload_id, sub])``, draws in FP64 and returns a
row-major array; callers cast to the path's input type (FP32 paths round once,
the oracle widens the same rounded values back to FP64).

A stream of ``t + steps*p`` rows is laid out as: rows ``[0, t)`` form the first
window; step ``w`` (1-based) appends ``rows[t+(w-1)p : t+wp]`` and drops the
window's oldest rows ``rows[(w-1)p : wp]`` (the sliding window of Sec. 2.1).

The workloads mirror the paper's setting (Sec. 4.2): a Gaussian window whose
later updates come from a non-Gaussian copula with the same covariance.  The
paper's own t-copula covariance is not given, so the covariance here is
``A A^T/n + I`` with a seeded Gaussian A, and the copula is Gaussian with
Student-t(6) and Exp(1) marginals standardized to that covariance's variances.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SEED_ROOT = 170106446


def rng_for(workload_id: int, sub: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_ROOT, workload_id, sub])))


def covariance(rng: np.random.Generator, n: int) -> np.ndarray:
    A = rng.standard_normal((n, n))
    return A @ A.T / n + np.eye(n)


def gaussian_rows(rng, m: int, sigma: np.ndarray) -> np.ndarray:
    L = np.linalg.cholesky(sigma)
    z = rng.standard_normal((m, sigma.shape[0]))
    return z @ L.T


def copula_rows(rng, m: int, sigma: np.ndarray) -> np.ndarray:
    """Gaussian copula with correlation of ``sigma``; columns ``< n/2`` get a
    standardized Student-t(6) marginal, the rest a standardized Exp(1)
    marginal, each scaled to the column's variance ``sigma[j, j]``."""
    from scipy import special, stats

    n = sigma.shape[0]
    sd = np.sqrt(np.diag(sigma))
    z = gaussian_rows(rng, m, sigma) / sd
    x = np.empty_like(z)
    h = n // 2
    zt = z[:, :h]
    # t quantile of Phi(z), evaluated in the tail that keeps precision
    x[:, :h] = np.sign(zt) * stats.t.isf(special.ndtr(-np.abs(zt)), 6) / np.sqrt(1.5)
    # Exp(1) quantile of Phi(z) is -log(1 - Phi(z)) = -log(Phi(-z))
    x[:, h:] = -special.log_ndtr(-z[:, h:]) - 1.0
    return x * sd


def exp_sources(rng, m: int, n: int) -> np.ndarray:
    return rng.exponential(1.0, (m, n)) - 1.0


def haar_orthogonal(rng, n: int) -> np.ndarray:
    G = rng.standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    return Q * np.sign(np.diag(R))


@dataclass
class Stream:
    name: str
    n: int
    d: int
    b: int
    t: int
    p: int
    steps: int
    rows: np.ndarray  # (t + steps*p, n), FP64

    def window(self) -> np.ndarray:
        return self.rows[: self.t]

    def step(self, w: int):
        """(X_new, X_old) of step w = 1..steps."""
        t, p = self.t, self.p
        return self.rows[t + (w - 1) * p: t + w * p], self.rows[(w - 1) * p: w * p]

    def current_window(self, w: int) -> np.ndarray:
        """The window after step w (w = 0 is the first window)."""
        return self.rows[w * self.p: w * self.p + self.t]


def gaussian_stream(n=20, d=4, b=2, t=2000, p=100, steps=20, workload_id=1) -> Stream:
    """Plain Gaussian stream: rows i.i.d. N(0, A A^T/n + I)."""
    rng = rng_for(workload_id)
    sigma = covariance(rng, n)
    rows = gaussian_rows(rng, t + steps * p, sigma)
    return Stream("gaussian", n, d, b, t, p, steps, rows)


def regime_change_stream(n=60, d=4, b=4, t=20000, p=1000, steps=200, switch=None,
                         workload_id=2) -> Stream:
    """Gaussian window and updates up to step ``switch`` (default steps//2),
    copula updates afterwards (the regime change of Sec. 4.2)."""
    rng = rng_for(workload_id)
    sigma = covariance(rng, n)
    if switch is None:
        switch = steps // 2
    g = gaussian_rows(rng, t + switch * p, sigma)
    c = copula_rows(rng, (steps - switch) * p, sigma)
    return Stream("regime_change", n, d, b, t, p, steps, np.vstack([g, c]))


def mixed_exp_stream(n=48, d=6, b=4, t=50000, p=2000, steps=50, workload_id=3) -> Stream:
    """Rows S W with S i.i.d. standardized Exp(1) sources and W Haar-orthogonal."""
    rng = rng_for(workload_id)
    W = haar_orthogonal(rng, n)
    S = exp_sources(rng, t + steps * p, n)
    s = Stream("mixed_exp", n, d, b, t, p, steps, S @ W)
    s.mixing = W
    return s


def exp_copula_rows(rng, m: int, sigma: np.ndarray) -> np.ndarray:
    """Gaussian copula with correlation of ``sigma`` and standardized Exp(1)
    marginals scaled to the variances ``sigma[j, j]``."""
    from scipy import special

    sd = np.sqrt(np.diag(sigma))
    z = gaussian_rows(rng, m, sigma) / sd
    return (-special.log_ndtr(-z) - 1.0) * sd


def batched_streams(m=64, steps=40, b=4, workload_id=5, n_max=96):
    """Independent streams of uneven shape: n uniform in {8, 12, ..., n_max},
    d uniform in {3, 4}, t uniform in [1000, 20000] rounded to a multiple of
    20, p = t/20; rows N(0, Sigma_s) or a Gaussian copula with Exp(1)
    marginals (a coin flip per stream).  One child seed per stream."""
    root = np.random.SeedSequence([SEED_ROOT, workload_id, 0])
    out = []
    for i, child in enumerate(root.spawn(m)):
        rng = np.random.Generator(np.random.PCG64(child))
        n = int(rng.choice(np.arange(8, n_max + 1, 4)))
        d = int(rng.integers(3, 5))
        t = int(round(rng.uniform(1000, 20000) / 20.0)) * 20
        p = t // 20
        sigma = covariance(rng, n)
        gen = exp_copula_rows if rng.random() < 0.5 else gaussian_rows
        rows = gen(rng, t + steps * p, sigma)
        s = Stream("batched_%02d" % i, n, d, min(b, n), t, p, steps, rows)
        s.kind = gen.__name__
        out.append(s)
    return out


def adjoint_workload(t=10000, n=32, workload_id=4):
    """(X, W) for the ICA-style contrast: X = T A^T with T i.i.d. standardized
    Student-t(5) sources and A = G_A / sqrt(n); W = Q + 0.05 G_W / sqrt(n)
    with Q Haar-orthogonal (near-orthogonal unmixing)."""
    rng = rng_for(workload_id)
    T = rng.standard_t(5, size=(t, n)) / np.sqrt(5.0 / 3.0)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    Q = haar_orthogonal(rng, n)
    W = Q + 0.05 * rng.standard_normal((n, n)) / np.sqrt(n)
    return T @ A.T, W


def stream_by_name(name: str, **kw) -> Stream:
    return {"gaussian": gaussian_stream, "regime_change": regime_change_stream,
            "mixed_exp": mixed_exp_stream}[name](**kw)


def _student_t_cdf_lower(t_abs, nu: int):
    """P(T <= -|t|) for a Student-t with an even number nu of degrees of
    freedom, in closed form: 1/2 - |t| / (2 sqrt(nu + t^2)) *
    sum_{j < nu/2} (2j)! / (4^j j!^2) (nu / (nu + t^2))^j (torch, float64)."""
    import torch

    assert nu % 2 == 0 and nu > 0
    r = nu / (nu + t_abs * t_abs)
    term = torch.ones_like(t_abs)
    acc = torch.ones_like(t_abs)
    for j in range(1, nu // 2):
        term = term * r * (2 * j - 1) / (2 * j)
        acc = acc + term
    return 0.5 - 0.5 * t_abs / torch.sqrt(nu + t_abs * t_abs) * acc


def tcopula_study_rows(run: int, n=100, t=1_000_000, tup=25_000, windows=61, nu=10, device="cuda",
                       workload_id=6):
    """Rows of the paper-scale stream study on the GPU (torch, float32): the
    first window of t rows i.i.d. N(0, Sigma), then (windows - 1) batches of
    tup rows from a Student-t copula with nu degrees of freedom and the
    correlation of Sigma, whose marginals are the first window's Gaussian
    marginals N(0, Sigma_jj).  Sigma = A A^T / n + I with a seeded Gaussian A
    (one Sigma for every run); each run draws from its own seeded generator.
    t-copula rows: z ~ N(0, R), w ~ chi^2_nu (a sum of nu squared normals),
    u_j = F_nu(z_j / sqrt(w / nu)), x_j = sqrt(Sigma_jj) Phi^{-1}(u_j), with
    Phi^{-1}(F_nu(-|y|)) taken in the lower tail for precision."""
    import torch

    sigma = covariance(rng_for(workload_id), n)
    sd = np.sqrt(np.diag(sigma))
    L = torch.from_numpy(np.linalg.cholesky(sigma)).to(device)
    Lr = torch.from_numpy(np.linalg.cholesky(sigma / np.outer(sd, sd))).to(device)
    sdt = torch.from_numpy(sd).to(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(np.random.SeedSequence([SEED_ROOT, workload_id, 1, run]).generate_state(1)[0]))
    m = (windows - 1) * tup
    out = torch.empty((t + m, n), dtype=torch.float32, device=device)
    step = 250_000
    for lo in range(0, t, step):
        hi = min(t, lo + step)
        z = torch.randn((hi - lo, n), generator=g, device=device, dtype=torch.float64)
        out[lo:hi] = (z @ L.T).float()
    for lo in range(0, m, step):
        hi = min(m, lo + step)
        z = torch.randn((hi - lo, n), generator=g, device=device, dtype=torch.float64) @ Lr.T
        w = (torch.randn((hi - lo, nu), generator=g, device=device, dtype=torch.float64) ** 2).sum(dim=1)
        y = z / torch.sqrt(w / nu)[:, None]
        lower = _student_t_cdf_lower(y.abs(), nu)
        x = -torch.special.ndtri(lower) * torch.sign(y)
        out[t + lo:t + hi] = (x * sdt).float()
    return out, sigma
