"""MI355X-native solver for the NeuRLP-PDE least-squares system of Mechanistic
PDE Networks (arXiv 2502.18377): batched multigrid-preconditioned Krylov
solve of the normal equations, with a backward pass through the KKT system.

Native library: libmpde.so (HIP, gfx950), C ABI in include/mpde.h.
"""
from . import _native  # noqa: F401


def __getattr__(name):
    if name in ("Problem", "pack", "default_options"):
        from . import api
        return getattr(api, name)
    if name in ("MPDESolve", "solve"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
