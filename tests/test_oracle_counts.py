"""Pin of the constraint set against the sizes the paper prints
(Sec. "Scaling PDE Solving"): a 32x32 grid gives 5120 variables and 9212
constraints, 377 MB of dense FP64 storage and 99.9% zeros; 32x32x32 gives
about 220k variables (exactly 229,376 = 7 x 32^3), about 420k constraints
and about 780 GB of dense storage."""
import numpy as np

from oracle.system import OracleProblem, assemble

DIR = ("dirichlet", "dirichlet")


def _prob(shape):
    D = len(shape)
    V = 1 + 2 * D
    rng = np.random.default_rng(0)
    return OracleProblem(shape=shape, step=tuple(1.0 / (n - 1) for n in shape), bc=(DIR,) * D,
                         mset=tuple(range(V)), coeff=rng.uniform(0.5, 1, (V,) + shape),
                         rhs=np.zeros(shape), bc_values=np.zeros(shape))


def test_counts_32x32():
    A, d, rows = assemble(_prob((32, 32)))
    nc, nv = A.shape
    assert nv == 5120 and nc == 9212
    assert round(nv * nc * 8 / 1e6) == 377
    assert 1 - A.nnz / (nv * nc) >= 0.999
    # row families: 1024 equation, 124 boundary, 3968 Taylor, 4096 difference rows
    assert rows["E"].size == 1024 and rows["B"].size == 124
    assert sum(rows[(k, a)].size for k in ("T+", "T-") for a in (0, 1)) == 3968
    assert sum(rows[(k, a)].size for k in ("C1", "C2") for a in (0, 1)) == 4096


def test_counts_32cubed():
    A, d, rows = assemble(_prob((32, 32, 32)))
    nc, nv = A.shape
    assert nv == 229_376 and round(nv, -4) == 230_000      # paper: "220k"
    assert nc == 425_608 and round(nc, -4) == 430_000      # paper: "420k"
    assert round(nv * nc * 8 / 1e9, -1) == 780              # paper: "780GB"
    assert 1 - A.nnz / (nv * nc) >= 0.99997
