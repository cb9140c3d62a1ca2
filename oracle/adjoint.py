"""Oracle for the loss L = sum_k w_k ||C_k(X W^T)||_F^2 and its gradients
(test infrastructure only).

Plain torch FP64 on the CPU with full n^k tensors: Y = X W^T; raw moments
M_k = (1/t) sum_l y_l^(x)k (Eq. (mom)), as products of row-wise Khatri-Rao
powers; cumulants by Alg. 3/4 on full tensors, C_s = M_s minus, over every
partition of the s positions into 2..s parts, the outer product of the
lower-order cumulants of the parts (one einsum per partition); the loss sums
squared Frobenius norms; torch autograd supplies dL/dX and dL/dW.
"""
from __future__ import annotations

import itertools
import string

import torch


def set_partitions(items):
    """All set partitions of a list (insert the first item into each part of
    every partition of the rest, or give it a part of its own)."""
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for p in set_partitions(rest):
        yield [[first]] + p
        for i in range(len(p)):
            yield p[:i] + [[first] + p[i]] + p[i + 1:]


def moments(Y: torch.Tensor, d: int):
    """M_1..M_d as full tensors (M_k has shape (n,)*k): the sum over rows of
    y^(x)k, written as P_h^T P_m / t with P_j the row-wise Khatri-Rao power
    y^(x)j of every row, h = ceil(k/2) and m = k - h (a matmul as the step)."""
    t, n = Y.shape
    P = [torch.ones(t, 1, dtype=Y.dtype)]
    for j in range(1, (d + 1) // 2 + 1):
        P.append((P[-1].unsqueeze(2) * Y.unsqueeze(1)).reshape(t, -1))
    out = []
    for k in range(1, d + 1):
        h = (k + 1) // 2
        out.append((P[h].T @ P[k - h] / t).reshape((n,) * k))
    return out


def cumulants(M):
    """Alg. 3/4 on full tensors, orders 1..d in increasing order."""
    d = len(M)
    C = []
    letters = string.ascii_letters
    for s in range(1, d + 1):
        idx = letters[:s]
        A = torch.zeros_like(M[s - 1])
        for pi in set_partitions(list(range(s))):
            if len(pi) < 2:
                continue
            spec = ",".join("".join(idx[q] for q in part) for part in pi) + "->" + idx
            A = A + torch.einsum(spec, *[C[len(part) - 1] for part in pi])
        C.append(M[s - 1] - A)
    return C


def loss(X: torch.Tensor, W: torch.Tensor, weights: dict, d: int = None) -> torch.Tensor:
    """sum_k weights[k] * ||C_k(X W^T)||_F^2."""
    d = d or max(weights)
    Y = X @ W.T
    C = cumulants(moments(Y, d))
    return sum(w * (C[k - 1] ** 2).sum() for k, w in weights.items())


def loss_and_grads(X, W, weights: dict, d: int = None):
    """(L, dL/dX, dL/dW) in FP64 via autograd."""
    X = torch.as_tensor(X, dtype=torch.float64).clone().requires_grad_(True)
    W = torch.as_tensor(W, dtype=torch.float64).clone().requires_grad_(True)
    L = loss(X, W, weights, d)
    gX, gW = torch.autograd.grad(L, (X, W))
    return float(L.detach()), gX.detach(), gW.detach()


def per_order_losses(X, W, d: int):
    X = torch.as_tensor(X, dtype=torch.float64)
    W = torch.as_tensor(W, dtype=torch.float64)
    C = cumulants(moments(X @ W.T, d))
    return [float((c ** 2).sum()) for c in C]
