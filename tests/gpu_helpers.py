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
