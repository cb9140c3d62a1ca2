"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on
the same seeded inputs and compare per order."""
from __future__ import annotations

import numpy as np

import oracle

TOL = {"fp64": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


def as_input(rows: np.ndarray, prec: str) -> np.ndarray:
    """The exact values both sides consume: FP32 paths read FP32-rounded rows,
    and the oracle widens those same values back to FP64."""
    dt = np.float64 if prec == "fp64" else np.float32
    return np.ascontiguousarray(rows.astype(dt))


def rel_err(C_gpu, C_ref, n, b, k) -> float:
    """||C_gpu - C_ref||_F / ||C_ref||_F over the full n^k tensor (Alg. 5 weights)."""
    num = oracle.block_norm(np.asarray(C_gpu) - np.asarray(C_ref), n, b, k)
    den = oracle.block_norm(C_ref, n, b, k)
    return num / den if den > 0 else num


def to_device(a: np.ndarray):
    import torch

    return torch.from_numpy(a).to("cuda")


# Same window, different kernels (a batched member against its own single
# context): the contraction sums rows in another order.  Each side is within
# TOL of the exact cumulants (relative Frobenius over the full tensor), so
# they agree to 2 TOL in the same measure.


def assert_same_to_rounding(a, b, prec, what="", n=None, bb=None, k=None):
    a, b = np.asarray(a), np.asarray(b)
    if k is None:  # plain vectors (norms)
        err = float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
    else:
        err = rel_err(a, b, n, bb, k)
    assert err <= 2 * TOL[prec], (what, err)


def nu_rtol(prec: str, k: int) -> float:
    """Tolerance of nu_k = ||C_k|| / ||C_2||^(k/2) (Eq. (mef)).  Each norm is
    within the order's relative Frobenius error of the oracle's (reverse
    triangle inequality), so to first order nu_k moves by at most
    (1 + k/2) times the path's error bound."""
    return (1.0 + k / 2.0) * max(TOL[prec], 1e-12)


def assert_norms_match(fro_g, nu_g, fro_o, nu_o, prec: str):
    """Norms per order (k >= 1) and the estimator nu_k (k >= 3) against the
    oracle's; a NaN nu (||C_2|| = 0) must be NaN on both sides."""
    fro_g, nu_g, fro_o, nu_o = map(np.asarray, (fro_g, nu_g, fro_o, nu_o))
    np.testing.assert_allclose(fro_g[1:], fro_o[1:], rtol=max(TOL[prec], 1e-12))
    for k in range(3, len(fro_o)):
        if np.isnan(nu_o[k]):
            assert np.isnan(nu_g[k]), (k, nu_g[k])
        else:
            assert abs(nu_g[k] - nu_o[k]) <= nu_rtol(prec, k) * abs(nu_o[k]), (k, nu_g[k], nu_o[k])


def assert_mean_match(C1_g, C1_o, C2_o, n: int, b: int, prec: str):
    """C_1 (the window mean) has no natural relative scale (it may be near
    zero), so its error is gated absolutely against the rows' RMS size
    sqrt(sum_i E[x_i^2]) = sqrt(trace C_2 + ||C_1||^2), times the path's
    tolerance."""
    C1_g, C1_o, C2_o = map(np.asarray, (C1_g, C1_o, C2_o))
    npad = -(-n // b) * b
    diag = 0.0
    for i in range(n):  # element (i, i) of the order-2 pyramid
        j, a = divmod(i, b)
        blk = j * (2 * (npad // b) - j + 1) // 2  # rank of block (j, j)
        diag += C2_o[blk * b * b + a * b + a]
    scale = np.sqrt(max(diag, 0.0) + float(np.sum(C1_o ** 2)))
    err = float(np.linalg.norm(C1_g - C1_o))
    assert err <= max(TOL[prec], 1e-12) * scale, (err, scale)
