"""Python binding of the MI355X NeuRLP-PDE solver (include/mpde.h).

Argument marshalling only: tensors are passed to the C ABI as device
pointers with the current torch stream; every step of the solve runs in the
library's HIP kernels.  There is no CPU fallback -- a missing library raises.
"""
import ctypes

import numpy as np
import torch

from . import _native as N

_TORCH_DT = {N.MPDE_F32: torch.float32, N.MPDE_F64: torch.float64}


def pack(instances, dtype=torch.float32, device="cuda"):
    """Concatenate a list of instance dicts (shape, step, bc, mset, coeff, rhs,
    bc_values; shared D, bc and mset) into the library's batch layout."""
    first = instances[0]
    D = len(first["shape"])
    for inst in instances:
        if len(inst["shape"]) != D or tuple(inst["bc"]) != tuple(first["bc"]) or \
                tuple(inst["mset"]) != tuple(first["mset"]):
            raise ValueError("all instances of a batch must share ndim, bc and mset")
    coeff = np.concatenate([np.asarray(i["coeff"]).reshape(-1) for i in instances])
    rhs = np.concatenate([np.asarray(i["rhs"]).reshape(-1) for i in instances])
    bcv = np.concatenate([np.asarray(i["bc_values"]).reshape(-1) for i in instances])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dtype)
    return dict(coeff=t(coeff), rhs=t(rhs), bc_values=t(bcv),
                shapes=[tuple(int(n) for n in i["shape"]) for i in instances],
                steps=[tuple(float(s) for s in i["step"]) for i in instances],
                bc=tuple(first["bc"]), mset=tuple(first["mset"]))


def default_options():
    o = N.Options()
    N.check(N.load().mpde_default_options(ctypes.byref(o)))
    return o


class Problem:
    """A built batch of PDE instances; owns the native handle."""

    def __init__(self, coeff, rhs, bc_values, shapes, steps, bc, mset, options=None, stream=None, **opt_kw):
        lib = N.load()
        if coeff.dtype not in (torch.float32, torch.float64):
            raise TypeError("coeff must be float32 or float64")
        for t in (coeff, rhs, bc_values):
            if not t.is_cuda or not t.is_contiguous() or t.dtype != coeff.dtype:
                raise ValueError("coeff, rhs, bc_values must be contiguous device tensors of one dtype")
        self.dtype = N.MPDE_F32 if coeff.dtype == torch.float32 else N.MPDE_F64
        self.D = len(shapes[0])
        self.B = len(shapes)
        self.V = 1 + 2 * self.D
        self.mset = tuple(mset)
        self.K = len(self.mset)
        self.shapes = [tuple(s) for s in shapes]
        self.npts = [int(np.prod(s)) for s in self.shapes]
        total = sum(self.npts)
        if rhs.numel() != total or bc_values.numel() != total or coeff.numel() != self.K * total:
            raise ValueError("tensor sizes do not match the shapes and mset")
        self.device = coeff.device
        self.torch_dtype = coeff.dtype
        o = options if options is not None else default_options()
        for k, v in opt_kw.items():
            setattr(o, k, v)
        self._opts = o
        self._shape_arr = (ctypes.c_int32 * (self.B * self.D))(*[n for s in self.shapes for n in s])
        self._step_arr = (ctypes.c_double * (self.B * self.D))(*[x for s in steps for x in s])
        d = N.Desc()
        d.dtype, d.ndim, d.batch = self.dtype, self.D, self.B
        d.shape = ctypes.cast(self._shape_arr, ctypes.POINTER(ctypes.c_int32))
        d.step = ctypes.cast(self._step_arr, ctypes.POINTER(ctypes.c_double))
        for a in range(3):
            lo, hi = bc[a] if a < self.D else ("none", "none")
            d.bc_lo[a], d.bc_hi[a] = N.BC_CODES[lo], N.BC_CODES[hi]
        d.mset = sum(1 << m for m in self.mset)
        d.coeff, d.rhs, d.bc_values = coeff.data_ptr(), rhs.data_ptr(), bc_values.data_ptr()
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        d.stream = s.cuda_stream
        d.opts = ctypes.pointer(o)
        self._stream = s
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            N.check(lib.mpde_build(ctypes.byref(d), ctypes.byref(h)))
        self._h = h
        self._lib = lib

    def _info(self):
        it = np.zeros(self.B, np.int32); ou = np.zeros(self.B, np.int32)
        rr = np.zeros(self.B, np.float64); stt = np.zeros(self.B, np.int32)
        info = N.Info()
        info.iters = it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        info.outer = ou.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        info.relres = rr.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        info.status = stt.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        return info, dict(iters=it, outer=ou, relres=rr, status=stt)

    def solve(self, out=None):
        """Return (z, info): z is the concatenated [V, N_b] blocks of all instances."""
        total = sum(self.npts)
        zdt = torch.float64 if self._opts.out_f64 else self.torch_dtype
        z = out if out is not None else torch.empty(self.V * total, dtype=zdt, device=self.device)
        if z.dtype != zdt or z.numel() != self.V * total:
            raise ValueError("out has the wrong dtype or size")
        info, res = self._info()
        with torch.cuda.device(self.device):
            code = N.check(self._lib.mpde_solve(self._h, z.data_ptr(), ctypes.byref(info)))
        res["code"], res["seconds"] = code, info.seconds
        return z, res

    def adjoint(self, g_z, want=("coeff", "rhs", "bc")):
        total = sum(self.npts)
        g_z = g_z.contiguous()
        if g_z.numel() != self.V * total or g_z.dtype != self.torch_dtype:
            raise ValueError("g_z must match z in size and dtype")
        mk = lambda n: torch.empty(n, dtype=self.torch_dtype, device=self.device)
        gc = mk(self.K * total) if "coeff" in want else None
        gf = mk(total) if "rhs" in want else None
        gw = mk(total) if "bc" in want else None
        ptr = lambda t: t.data_ptr() if t is not None else None
        info, res = self._info()
        with torch.cuda.device(self.device):
            code = N.check(self._lib.mpde_solve_adjoint(self._h, g_z.data_ptr(), ptr(gc), ptr(gf), ptr(gw),
                                                        ctypes.byref(info)))
        res["code"], res["seconds"] = code, info.seconds
        return gc, gf, gw, res

    def kernel_stats(self):
        """Finest-grid kernel timings of the last solve (options.profile=1)."""
        arr = (N.KStat * 4)()
        n = self._lib.mpde_kernel_stats(self._h, arr, 4)
        return {arr[i].name.decode(): dict(launches=int(arr[i].launches), ms=arr[i].ms, bytes=arr[i].bytes)
                for i in range(min(n, 4))}

    def time_operator(self, mode=2, reps=20):
        """Mean microseconds and algorithmic HBM bytes of one finest-grid
        operator pass in `mode` (0 apply, 1 residual, 2 Chebyshev step, 3
        apply with dot products, 4 the FP64 residual of the outer
        refinement), timed over `reps` back-to-back passes."""
        us, by = ctypes.c_double(), ctypes.c_double()
        N.check(self._lib.mpde_time_operator(self._h, mode, reps, ctypes.byref(us), ctypes.byref(by)))
        return us.value, by.value

    def levels(self, b=0):
        n = self._lib.mpde_levels(self._h, b, None)
        arr = (ctypes.c_int32 * (n * self.D))()
        self._lib.mpde_levels(self._h, b, arr)
        return [tuple(arr[l * self.D:(l + 1) * self.D]) for l in range(n)]

    def split(self, z):
        """List of per-instance [V, *shape] views of a concatenated z."""
        out, off = [], 0
        for s, n in zip(self.shapes, self.npts):
            out.append(z[off:off + self.V * n].view(self.V, *s))
            off += self.V * n
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._lib.mpde_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
