"""FP64 reference of the coarse-correction network (test infrastructure only).

The network is a stack of 3x3x3 convolutions over a (t, x, y) grid with
channels last, "same" output size, zero padding along non-periodic axes and
wrap-around along periodic ones:

    out[p, co] = bias[co] + sum_{tap, ci} W[tap, co, ci] * X[p + off(tap), ci]

with taps ordered (dt, dx, dy) in {-1,0,1}^3, dt slowest.  ReLU follows every
layer but the last.  Backward:

    dX[p, ci]        = sum_{tap, co} W[tap, co, ci] * dY[p - off(tap), co]
    dW[tap, co, ci]  = sum_p dY[p, co] * X[p + off(tap), ci]
    dbias[co]        = sum_p dY[p, co]

These are the plain definitions, written with numpy shifts; the pins in
tests/test_oracle_convnet.py compare them with brute-force loops and with an
independent library convolution.
"""

import numpy as np

TAPS = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]


def shift(X, off, periodic):
    """Y[p] = X[p + off] (zero outside non-periodic axes). X: [T, NX, NY, C]."""
    Y = X
    for ax, (o, per) in enumerate(zip(off, periodic)):
        if o == 0:
            continue
        if per:
            Y = np.roll(Y, -o, axis=ax)
        else:
            Z = np.zeros_like(Y)
            n = Y.shape[ax]
            src = [slice(None)] * Y.ndim
            dst = [slice(None)] * Y.ndim
            if o > 0:
                src[ax], dst[ax] = slice(o, n), slice(0, n - o)
            else:
                src[ax], dst[ax] = slice(0, n + o), slice(-o, n)
            Z[tuple(dst)] = Y[tuple(src)]
            Y = Z
    return Y


def conv_fwd(X, W, bias, periodic):
    """X [T,NX,NY,Ci], W [27,Co,Ci], bias [Co] -> [T,NX,NY,Co] (FP64)."""
    X = np.asarray(X, np.float64)
    out = np.broadcast_to(np.asarray(bias, np.float64), X.shape[:3] + (W.shape[1],)).copy()
    for k, off in enumerate(TAPS):
        out += shift(X, off, periodic) @ np.asarray(W[k], np.float64).T
    return out


def conv_bwd_data(dY, W, periodic):
    dY = np.asarray(dY, np.float64)
    dX = np.zeros(dY.shape[:3] + (W.shape[2],))
    for k, off in enumerate(TAPS):
        neg = tuple(-o for o in off)
        dX += shift(dY, neg, periodic) @ np.asarray(W[k], np.float64)
    return dX


def conv_bwd_weight(X, dY, periodic):
    X = np.asarray(X, np.float64)
    dY = np.asarray(dY, np.float64)
    Co, Ci = dY.shape[3], X.shape[3]
    dW = np.zeros((27, Co, Ci))
    for k, off in enumerate(TAPS):
        Xs = shift(X, off, periodic).reshape(-1, Ci)
        dW[k] = dY.reshape(-1, Co).T @ Xs
    return dW, dY.reshape(-1, Co).sum(axis=0)


def net_fwd(X, layers, periodic):
    """layers: list of (W, bias); ReLU between layers.  Returns output and the
    pre-activations needed for the backward pass."""
    acts, pre = [X], []
    h = X
    for i, (W, b) in enumerate(layers):
        z = conv_fwd(h, W, b, periodic)
        pre.append(z)
        h = np.maximum(z, 0.0) if i + 1 < len(layers) else z
        acts.append(h)
    return h, acts, pre


def net_bwd(dOut, acts, pre, layers, periodic):
    grads = [None] * len(layers)
    g = dOut
    for i in reversed(range(len(layers))):
        if i + 1 < len(layers):
            g = g * (pre[i] > 0)
        dW, db = conv_bwd_weight(acts[i], g, periodic)
        grads[i] = (dW, db)
        g = conv_bwd_data(g, layers[i][0], periodic)
    return grads, g


def bf16_round(a):
    """Round-to-nearest-even to bfloat16, returned as float64."""
    a = np.ascontiguousarray(np.asarray(a, np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)
