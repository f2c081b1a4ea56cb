"""Discretisation pins: manufactured solution of the 1D+time workload
(u* = exp(-t) sin(pi x)) and the 2D Laplace special case with an exact
harmonic solution.  The paper prints no order; we require the error to fall
monotonically under refinement with an observed order of at least 1.5, and the
Laplace error to fall 16 -> 32 -> 64 as in the paper's solver unit test."""
import numpy as np

import workloads as W
from oracle.system import assemble
from oracle.solve import solve_kkt
from tests.conftest import to_oracle


def _u_err(inst):
    A, d, _ = assemble(to_oracle(inst))
    z = solve_kkt(A, d)[0]
    N = int(np.prod(inst["shape"]))
    u = z[:N].reshape(inst["shape"])
    ue = inst["exact"][0]
    return np.sqrt(np.mean((u - ue) ** 2)) / np.sqrt(np.mean(ue ** 2))


def test_mms_rd1d_order():
    # smooth coefficients so the observed order reflects the discretisation
    errs = []
    for n in (16, 32, 64):
        inst = W.reaction_diffusion_1d(shape=(n, n))
        T, X = np.meshgrid(np.linspace(0, 1, n), np.linspace(0, 1, n), indexing="ij")
        a = 0.5 + 0.3 * np.sin(2 * np.pi * X) * np.cos(np.pi * T)
        u = np.exp(-T) * np.sin(np.pi * X)
        inst["coeff"][3] = -a
        inst["coeff"][2] = 0.0
        inst["coeff"][0] = 0.0
        inst["rhs"] = -u + a * np.pi ** 2 * u
        errs.append(_u_err(inst))
    assert errs[0] > errs[1] > errs[2]
    order = np.log2(errs[1] / errs[2])
    assert order >= 1.5, (errs, order)


def test_mms_rd1d_generator_converges():
    errs = [_u_err(W.reaction_diffusion_1d(shape=(n, n))) for n in (16, 32, 64)]
    assert errs[0] > errs[1] > errs[2]


def test_laplace_error_decreases():
    errs = [_u_err(W.laplace2d(n)) for n in (16, 32, 64)]
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-2
