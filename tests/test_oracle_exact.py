"""Exactness pins of the whole oracle (assembly + solve).

If u* is a tensor-product quadratic in every non-periodic axis (constant
along periodic axes), every Taylor row (Eqs. 6-7) and every 5-point
difference row (Eq. 5) holds exactly for the true derivatives, and with
f = sum_m c_m d_m u* and omega = u* the equation and boundary rows hold
too; then A z_exact = d, so the least-squares solution is z_exact.  A dropped
term, a wrong sign in a Taylor row, a wrong stencil weight or a wrong
neighbour index breaks this."""
import numpy as np
import pytest

import workloads as W
from oracle.system import assemble, exact_variables
from oracle.solve import solve_kkt, solve_dense_lstsq
from tests.conftest import to_oracle

IC = ("dirichlet", "none")
DIR = ("dirichlet", "dirichlet")
PER = ("periodic", "periodic")

CASES = [
    ((7, 6), (IC, DIR), (0, 1, 3, 4)),
    ((6, 8), (DIR, DIR), (0, 1, 2, 3, 4)),
    ((9, 5), (IC, ("none", "none")), (1, 4)),
    ((5, 6, 7), (IC, PER, PER), (0, 1, 3, 4, 5, 6)),
    ((6, 5, 6), (IC, DIR, PER), (0, 1, 2, 3, 4, 5, 6)),
]


def _z_exact(inst):
    D = len(inst["shape"])
    return np.concatenate([inst["exact"][v].reshape(-1) for v in range(1 + 2 * D)])


@pytest.mark.parametrize("shape,bc,mset", CASES)
def test_quadratic_exact(shape, bc, mset):
    inst = W.quadratic_exact(shape, bc, mset, seed=sum(shape))
    A, d, rows = assemble(to_oracle(inst))
    ze = _z_exact(inst)
    assert np.linalg.norm(A @ ze - d) <= 1e-10 * np.linalg.norm(d)
    z, lam, _ = solve_kkt(A, d)
    assert np.linalg.norm(z - ze) <= 1e-8 * np.linalg.norm(ze)
    assert np.linalg.norm(lam) <= 1e-8 * np.linalg.norm(d)


def test_quartic_difference_rows_exact():
    # 5-point difference rows are exact up to degree 4; Taylor rows are not.
    shape, step = (9, 8), (0.1, 0.2)
    funcs = [lambda t, x: t ** 4 - 2 * x ** 4 + t * x,
             lambda t, x: 4 * t ** 3 + x + 0 * t, lambda t, x: 12 * t ** 2 + 0 * x,
             lambda t, x: -8 * x ** 3 + t, lambda t, x: -24 * x ** 2 + 0 * t]
    z = exact_variables(shape, step, funcs)
    inst = W.random_instance(shape, (DIR, DIR), seed=3)
    inst["step"] = step
    A, d, rows = assemble(to_oracle(inst))
    r = A @ z
    for a in (0, 1):
        for k in ("C1", "C2"):
            assert np.abs(r[rows[(k, a)]]).max() < 1e-10
    assert np.abs(r[rows[("T+", 0)]]).max() > 1e-4


def test_dense_matches_kkt_quadratic():
    inst = W.quadratic_exact((5, 6), (IC, DIR), (0, 1, 3, 4), seed=5)
    A, d, _ = assemble(to_oracle(inst))
    assert np.allclose(solve_dense_lstsq(A, d), _z_exact(inst), atol=1e-9)
