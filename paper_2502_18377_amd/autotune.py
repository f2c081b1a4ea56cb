"""Autotuned solver settings per shape class, cached in a JSON file.

The search itself (coordinate search over smoothing steps, inner Krylov
tolerance and iterations per captured graph, timing complete solves) runs in
the native library (mpde_autotune); this module only keys and stores the
results."""
import ctypes
import json
import math
import os

import torch

from . import _native as N


def shape_class(problem):
    """Key: ndim, dtype, boundary pattern, log2 buckets of the mean instance
    size and of the batch size."""
    mean_n = sum(problem.npts) / len(problem.npts)
    return (f"D{problem.D}-{'f32' if problem.dtype == N.MPDE_F32 else 'f64'}-K{problem.K}"
            f"-N{int(math.log2(max(mean_n, 1)))}-B{int(math.log2(max(problem.B, 1)))}")


def run(problem):
    """Autotune `problem` in place; returns the chosen settings."""
    lib = N.load()
    total = sum(problem.npts)
    z = torch.empty(problem.V * total, dtype=torch.float64 if problem._opts.out_f64 else problem.torch_dtype,
                    device=problem.device)
    chosen = (ctypes.c_int32 * 3)()
    best = ctypes.c_double()
    N.check(lib.mpde_autotune(problem._h, z.data_ptr(), chosen, ctypes.byref(best)))
    return {"nu": chosen[0], "check_every": chosen[1], "inner_tol": chosen[2] * 1e-9, "solve_ms": best.value}


def lookup(key, path):
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f).get(key)
    return None


def store(key, settings, path):
    data = {}
    if os.path.exists(path):
        with open(path) as f:
            data = json.load(f)
    data[key] = settings
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
