"""Learned coarse-grid correction: Python handle of the native network
(argument marshalling only; training steps, inference and the conv kernels
run in libmpde)."""
import ctypes

import numpy as np
import torch

from . import _native as N


class Net:
    def __init__(self, in_channels, seed=0):
        self._lib = N.load()
        h = ctypes.c_void_p()
        N.check(self._lib.mpde_net_create(in_channels, seed, ctypes.byref(h)))
        self._h = h
        self.in_channels = in_channels

    def train_step(self, problem, level, seed, lr):
        """Returns (loss of the learned correction, loss of the plain V-cycle)."""
        loss, plain = ctypes.c_double(), ctypes.c_double()
        N.check(self._lib.mpde_net_train_step(self._h, problem._h, level, seed, lr, ctypes.byref(loss),
                                              ctypes.byref(plain)))
        return loss.value, plain.value

    def attach(self, problem, level):
        N.check(self._lib.mpde_net_attach(problem._h, self._h, level))
        problem._net = self        # keep the weights alive while attached

    @staticmethod
    def detach(problem):
        N.check(N.load().mpde_net_attach(problem._h, None, 0))
        problem._net = None

    def get(self):
        a = np.zeros(N.NET_PARAMS, np.float32)
        N.check(self._lib.mpde_net_get(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))
        return a

    def set(self, a):
        a = np.ascontiguousarray(a, np.float32)
        N.check(self._lib.mpde_net_set(self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), a.size))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.mpde_net_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def conv3d(x_bf16, w_bf16, bias, periodic, relu=False, sign=1, want=("f32",)):
    """One conv layer on [batch, T, X, Y, 16] bf16 input; returns FP32 and/or
    bf16 outputs of the same shape."""
    lib = N.load()
    B, T, X, Y, C = x_bf16.shape
    assert C == 16 and x_bf16.dtype == torch.bfloat16 and w_bf16.dtype == torch.bfloat16
    y = torch.empty(x_bf16.shape, dtype=torch.float32, device=x_bf16.device) if "f32" in want else None
    yb = torch.empty_like(x_bf16) if "bf16" in want else None
    per = (ctypes.c_int32 * 3)(*[int(bool(p)) for p in periodic])
    s = torch.cuda.current_stream(x_bf16.device).cuda_stream
    N.check(lib.mpde_conv3d(x_bf16.data_ptr(), w_bf16.data_ptr(), bias.data_ptr() if bias is not None else None,
                            y.data_ptr() if y is not None else None, yb.data_ptr() if yb is not None else None,
                            int(relu), sign, B, T, X, Y, per, s))
    return y, yb


def conv3d_wgrad(x_bf16, dy_bf16, periodic):
    lib = N.load()
    B, T, X, Y, C = x_bf16.shape
    dw = torch.empty((27, 16, 16), dtype=torch.float32, device=x_bf16.device)
    per = (ctypes.c_int32 * 3)(*[int(bool(p)) for p in periodic])
    s = torch.cuda.current_stream(x_bf16.device).cuda_stream
    N.check(lib.mpde_conv3d_wgrad(x_bf16.data_ptr(), dy_bf16.data_ptr(), dw.data_ptr(), B, T, X, Y, per, s))
    return dw


def train(net, problems, level, steps, lr=1e-3, lr_final=1e-4, log_every=0, seed0=0):
    """Adam training of `net` on solver-generated problems (cycled), with a
    geometric learning-rate decay from lr to lr_final.  Returns the list of
    (step, loss, loss_plain)."""
    hist = []
    for k in range(steps):
        a = lr * (lr_final / lr) ** (k / max(1, steps - 1))
        loss, plain = net.train_step(problems[k % len(problems)], level, seed0 + k, a)
        hist.append((k, loss, plain))
        if log_every and (k % log_every == 0 or k == steps - 1):
            print(f"train step {k}: loss {loss:.5f} plain-MG {plain:.5f} lr {a:.2e}", flush=True)
    return hist
