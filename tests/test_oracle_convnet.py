"""Pins of the FP64 conv-network reference (oracle.convnet): brute-force
loops on tiny grids, an independent library convolution (torch, FP64, CPU)
with circular/zero padding, gradients by finite differences, and the bf16
rounding against torch's bfloat16 cast."""
import numpy as np
import pytest

from oracle import convnet as C


def _brute(X, W, b, periodic):
    T, NX, NY, Ci = X.shape
    out = np.zeros((T, NX, NY, W.shape[1]))
    for t in range(T):
        for x in range(NX):
            for y in range(NY):
                acc = b.copy()
                for k, (a, bb, c) in enumerate(C.TAPS):
                    q = [t + a, x + bb, y + c]
                    ok = True
                    for ax, n in enumerate((T, NX, NY)):
                        if periodic[ax]:
                            q[ax] %= n
                        elif not 0 <= q[ax] < n:
                            ok = False
                    if ok:
                        acc = acc + W[k] @ X[q[0], q[1], q[2]]
                out[t, x, y] = acc
    return out


@pytest.mark.parametrize("periodic", [(False, True, True), (True, False, True), (False, False, False)])
def test_conv_fwd_brute_force(periodic):
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, 4, 5, 3))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(2)
    assert np.allclose(C.conv_fwd(X, W, b, periodic), _brute(X, W, b, periodic), atol=1e-12)


def test_conv_matches_torch():
    import torch
    import torch.nn.functional as F
    rng = np.random.default_rng(1)
    X = rng.standard_normal((5, 6, 7, 4))
    W = rng.standard_normal((27, 3, 4))
    b = rng.standard_normal(3)
    periodic = (False, True, True)
    xt = torch.from_numpy(X).permute(3, 0, 1, 2)[None]                      # N C T X Y
    xt = F.pad(xt, (1, 1, 1, 1, 0, 0), mode="circular")                     # y, x circular
    xt = F.pad(xt, (0, 0, 0, 0, 1, 1))                                      # t zero
    wt = torch.from_numpy(W.reshape(3, 3, 3, 3, 4)).permute(3, 4, 0, 1, 2)  # Co Ci kt kx ky
    ref = F.conv3d(xt, wt, torch.from_numpy(b))[0].permute(1, 2, 3, 0).numpy()
    assert np.allclose(C.conv_fwd(X, W, b, periodic), ref, atol=1e-12)


def test_net_gradients_fd():
    rng = np.random.default_rng(2)
    periodic = (False, True, True)
    X = rng.standard_normal((3, 4, 4, 2))
    layers = [(rng.standard_normal((27, 3, 2)) * 0.3, rng.standard_normal(3) * 0.1),
              (rng.standard_normal((27, 1, 3)) * 0.3, rng.standard_normal(1) * 0.1)]
    G = rng.standard_normal((3, 4, 4, 1))
    out, acts, pre = C.net_fwd(X, layers, periodic)
    grads, dX = C.net_bwd(G, acts, pre, layers, periodic)
    loss = lambda L, XX: float(np.sum(C.net_fwd(XX, L, periodic)[0] * G))
    eps = 1e-6
    for li, idx in [(0, (4, 1, 0)), (0, (13, 2, 1)), (1, (20, 0, 2))]:
        Lp = [(W.copy(), b.copy()) for W, b in layers]
        Lm = [(W.copy(), b.copy()) for W, b in layers]
        Lp[li][0][idx] += eps
        Lm[li][0][idx] -= eps
        fd = (loss(Lp, X) - loss(Lm, X)) / (2 * eps)
        assert np.isclose(grads[li][0][idx], fd, rtol=1e-5, atol=1e-8)
    Lp = [(W.copy(), b.copy()) for W, b in layers]; Lp[1][1][0] += eps
    Lm = [(W.copy(), b.copy()) for W, b in layers]; Lm[1][1][0] -= eps
    assert np.isclose(grads[1][1][0], (loss(Lp, X) - loss(Lm, X)) / (2 * eps), rtol=1e-5)
    Xp = X.copy(); Xp[1, 2, 3, 1] += eps
    Xm = X.copy(); Xm[1, 2, 3, 1] -= eps
    assert np.isclose(dX[1, 2, 3, 1], (loss(layers, Xp) - loss(layers, Xm)) / (2 * eps), rtol=1e-5, atol=1e-8)


def test_bf16_round_matches_torch():
    import torch
    a = np.random.default_rng(3).standard_normal(1000).astype(np.float32) * 10
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(C.bf16_round(a), ref)
