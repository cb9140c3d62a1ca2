"""The HIP adjoint of L = ||C_3(XW^T)||^2 + ||C_4(XW^T)||^2 (X 10000 x 32,
W 32 x 32): against the torch-FP64 oracle's loss and autograd gradient,
central finite differences (h = 1e-3) of the oracle and of the GPU loss,
the homogeneity / bilinearity / shift identities, and the
torch.autograd.Function wrapper."""
import numpy as np
import pytest
import torch

import streams
from oracle import adjoint

pytestmark = pytest.mark.gpu

W8 = {3: 1.0, 4: 1.0}


def _inputs():
    X, W = streams.adjoint_workload()
    X32 = np.ascontiguousarray(X.astype(np.float32))
    W32 = np.ascontiguousarray(W.astype(np.float32))
    return X32, W32


def test_loss_and_gradients_vs_oracle_autograd():
    import paper_1701_06446_amd as cum

    X32, W32 = _inputs()
    L, dX, dW = cum.cum_loss_grad(torch.from_numpy(X32).cuda(), torch.from_numpy(W32).cuda(), 4, 4, W8)
    Lo, gXo, gWo = adjoint.loss_and_grads(X32.astype(np.float64), W32.astype(np.float64), W8, d=4)
    dX, dW = dX.cpu().double(), dW.cpu().double()
    eL = abs(L - Lo) / Lo
    eX = float((dX - gXo).norm() / gXo.norm())
    eW = float((dW - gWo).norm() / gWo.norm())
    print("loss rel err %.2e  dX %.2e  dW %.2e" % (eL, eX, eW))
    assert eL <= 1e-5 and eX <= 1e-5 and eW <= 1e-5  # the FP32 path's tolerance


def test_central_differences_of_oracle_and_gpu_loss():
    """64 random directions: the GPU gradient against central differences of
    the GPU loss (h = 1e-3; the Richardson value at h, h/2 is reported);
    8 of them also against central differences of the FP64 oracle."""
    import paper_1701_06446_amd as cum

    X32, W32 = _inputs()
    Xd, Wd = torch.from_numpy(X32).cuda(), torch.from_numpy(W32).cuda()
    _, dX, dW = cum.cum_loss_grad(Xd, Wd, 4, 4, W8)
    dX, dW = dX.double(), dW.double()
    gen = torch.Generator(device="cpu").manual_seed(12)

    def gpu_loss(Xp, Wp):
        return cum.cum_loss_grad(Xp.float().contiguous(), Wp.float().contiguous(), 4, 4, W8)[0]

    worst1 = worst2 = 0.0
    for i in range(64):
        vX = torch.randn(X32.shape, generator=gen, dtype=torch.float64).cuda()
        vW = torch.randn(W32.shape, generator=gen, dtype=torch.float64).cuda()
        an = float((dX * vX).sum() + (dW * vW).sum())
        Xp, Wp = Xd.double(), Wd.double()
        cd1 = (gpu_loss(Xp + 1e-3 * vX, Wp + 1e-3 * vW) - gpu_loss(Xp - 1e-3 * vX, Wp - 1e-3 * vW)) / 2e-3
        cd2 = (gpu_loss(Xp + 5e-4 * vX, Wp + 5e-4 * vW) - gpu_loss(Xp - 5e-4 * vX, Wp - 5e-4 * vW)) / 1e-3
        worst1 = max(worst1, abs(cd1 - an) / abs(an))
        worst2 = max(worst2, abs((4 * cd2 - cd1) / 3 - an) / abs(an))
        if i < 8:
            Xo, Wo = torch.from_numpy(X32).double(), torch.from_numpy(W32).double()
            vXc, vWc = vX.cpu(), vW.cpu()
            o1 = float(adjoint.loss(Xo + 1e-3 * vXc, Wo + 1e-3 * vWc, W8) -
                       adjoint.loss(Xo - 1e-3 * vXc, Wo - 1e-3 * vWc, W8)) / 2e-3
            print("dir %d: analytic %.6e  oracle FD %.6e  GPU FD %.6e" % (i, an, o1, cd1), flush=True)
            assert abs(o1 - an) <= 1e-3 * abs(an), (i, o1, an)
    print("worst FD rel err of the GPU loss: central %.2e  Richardson %.2e" % (worst1, worst2))
    # central differences at h = 1e-3 carry an O(h^2) truncation of ~1e-4
    # relative here (the oracle's own differences show it); FP32 rounding of
    # the loss adds far less at this step
    assert worst1 <= 2e-3


def test_identities():
    import paper_1701_06446_amd as cum

    X32, W32 = _inputs()
    Xd, Wd = torch.from_numpy(X32).cuda(), torch.from_numpy(W32).cuda()
    _, dX, dW = cum.cum_loss_grad(Xd, Wd, 4, 4, W8)
    L3, _, _ = cum.cum_loss_grad(Xd, Wd, 4, 4, {3: 1.0})
    L4, _, _ = cum.cum_loss_grad(Xd, Wd, 4, 4, {4: 1.0})
    gx = float((dX.double() * Xd.double()).sum())
    gw = float((dW.double() * Wd.double()).sum())
    assert abs(gx - (6 * L3 + 8 * L4)) <= 1e-4 * (6 * L3 + 8 * L4)
    assert abs(gw - gx) <= 1e-4 * abs(gx)
    assert float(dX.double().sum(0).abs().max()) <= 1e-4 * float(dX.abs().max()) * X32.shape[0] ** 0.5


def test_autograd_function():
    import paper_1701_06446_amd as cum

    X32, W32 = _inputs()
    Xd = torch.from_numpy(X32).cuda().requires_grad_(True)
    Wd = torch.from_numpy(W32).cuda().requires_grad_(True)
    L = cum.CumLoss.apply(Xd, Wd)
    (2.0 * L).backward()
    _, dX, dW = cum.cum_loss_grad(Xd.detach(), Wd.detach(), 4, 4, W8)
    assert torch.allclose(Xd.grad, 2.0 * dX, rtol=1e-6, atol=1e-12)
    assert torch.allclose(Wd.grad, 2.0 * dW, rtol=1e-6, atol=1e-12)


def test_bitwise_repeatable():
    """Two calls on the same inputs return bitwise equal loss and gradients:
    the reverse combine and Y_bar take every sum in a fixed order."""
    import paper_1701_06446_amd as cum

    X32, W32 = _inputs()
    Xd, Wd = torch.from_numpy(X32).cuda(), torch.from_numpy(W32).cuda()
    L1, dX1, dW1 = cum.cum_loss_grad(Xd, Wd, 4, 4, W8)
    L2, dX2, dW2 = cum.cum_loss_grad(Xd, Wd, 4, 4, W8)
    assert L1 == L2
    assert torch.equal(dX1, dX2) and torch.equal(dW1, dW2)


@pytest.mark.parametrize("n,d,b,t", [(10, 5, 2, 3000), (7, 6, 2, 2500), (13, 3, 4, 1999)])
def test_other_orders_vs_oracle(n, d, b, t):
    """Orders 3, 5 and 6 (every reverse block size up to 2^6 positions, a
    ragged last block when b does not divide n, a ragged last row tile),
    weights on every order from 2 up, against the FP64 oracle."""
    import paper_1701_06446_amd as cum

    rng = np.random.default_rng(100 * n + d)
    X = rng.standard_t(6, size=(t, n)) @ (rng.standard_normal((n, n)) / np.sqrt(n))
    W = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    X32 = np.ascontiguousarray(X.astype(np.float32))
    W32 = np.ascontiguousarray(W.astype(np.float32))
    w8 = {k: 1.0 / k for k in range(2, d + 1)}
    L, dX, dW = cum.cum_loss_grad(torch.from_numpy(X32).cuda(), torch.from_numpy(W32).cuda(), d, b, w8)
    Lo, gXo, gWo = adjoint.loss_and_grads(X32.astype(np.float64), W32.astype(np.float64), w8, d=d)
    dX, dW = dX.cpu().double(), dW.cpu().double()
    eL = abs(L - Lo) / Lo
    eX = float((dX - gXo).norm() / gXo.norm())
    eW = float((dW - gWo).norm() / gWo.norm())
    print("n=%d d=%d b=%d: loss %.2e dX %.2e dW %.2e" % (n, d, b, eL, eX, eW))
    assert eL <= 1e-5 and eX <= 1e-5 and eW <= 1e-5
