"""Pins of the adjoint oracle (no GPU): central finite differences, the
homogeneity and bilinearity identities, shift invariance, and agreement of
its cumulant norms with the pyramid oracle."""
import numpy as np
import torch

import oracle
from oracle import adjoint


def _data(seed, t=400, n=6):
    rng = np.random.default_rng(seed)
    S = rng.standard_t(5, size=(t, n)) / np.sqrt(5 / 3)
    A = rng.standard_normal((n, n)) / np.sqrt(n)
    X = S @ A.T
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    W = Q + 0.05 * rng.standard_normal((n, n)) / np.sqrt(n)
    return torch.tensor(X), torch.tensor(W)


def test_norms_match_pyramid_oracle():
    X, W = _data(1)
    Y = (X @ W.T).numpy()
    fro, _ = oracle.SlidingOracle(Y, Y.shape[1], 4, 2).norms()
    L = adjoint.per_order_losses(X, W, 4)
    for k in range(1, 5):
        assert abs(L[k - 1] - fro[k] ** 2) <= 1e-12 * max(1.0, L[k - 1])


def test_central_differences():
    X, W = _data(2)
    w = {3: 1.0, 4: 1.0}
    L, gX, gW = adjoint.loss_and_grads(X, W, w)
    rng = np.random.default_rng(3)

    def cd(dX, dW, h):
        return float(adjoint.loss(X + h * dX, W + h * dW, w) - adjoint.loss(X - h * dX, W - h * dW, w)) / (2 * h)

    for _ in range(16):
        dX = torch.tensor(rng.standard_normal(X.shape))
        dW = torch.tensor(rng.standard_normal(W.shape))
        an = float((gX * dX).sum() + (gW * dW).sum())
        d1, d2 = cd(dX, dW, 1e-3), cd(dX, dW, 5e-4)
        # central differences at h = 1e-3 carry an O(h^2) truncation error;
        # Richardson extrapolation of two step sizes removes it
        assert abs(d1 - an) <= 1e-3 * abs(an)
        assert abs((4 * d2 - d1) / 3 - an) <= 1e-7 * abs(an)


def test_identities():
    X, W = _data(4)
    w = {3: 1.0, 4: 1.0}
    L, gX, gW = adjoint.loss_and_grads(X, W, w)
    L3, L4 = adjoint.per_order_losses(X, W, 4)[2:4]
    # degree-2k homogeneity of ||C_k||^2 in X
    assert abs(float((gX * X).sum()) - (6 * L3 + 8 * L4)) <= 1e-10 * (6 * L3 + 8 * L4)
    # Y = X W^T is bilinear
    assert abs(float((gW * W).sum()) - float((gX * X).sum())) <= 1e-10 * abs(float((gX * X).sum()))
    # cumulants of order >= 2 ignore a common shift of the rows
    assert float(gX.sum(0).abs().max()) <= 1e-10 * float(gX.abs().max())


def test_moments_match_the_plain_definition():
    """The adjoint oracle's moments (products of row-wise Khatri-Rao powers
    of orders ceil(k/2) and k - ceil(k/2)) against Eq. (mom) written out
    element by element: M_k[i_1..i_k] = (1/t) sum_l prod_q y[l, i_q], over
    every multi-index of a small window, orders 1..5."""
    import itertools

    import numpy as np
    import torch

    from oracle import adjoint

    rng = np.random.default_rng(7)
    t, n, d = 40, 3, 5
    Y = rng.standard_normal((t, n)) + 0.3
    M = adjoint.moments(torch.from_numpy(Y), d)
    for k in range(1, d + 1):
        want = np.zeros((n,) * k)
        for idx in itertools.product(range(n), repeat=k):
            want[idx] = np.mean(np.prod(Y[:, list(idx)], axis=1))
        assert np.allclose(M[k - 1].numpy(), want, rtol=1e-13, atol=1e-15), k
