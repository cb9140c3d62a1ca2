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
