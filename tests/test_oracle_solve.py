"""Pins of the least-squares solve: brute force (dense lstsq) on tiny grids,
agreement of the saddle-point and normal-equation factorisations, least-squares
optimality, full column rank, and translation invariance along periodic axes."""
import numpy as np
import pytest

import workloads as W
from oracle.system import assemble
from oracle.solve import (solve_kkt, solve_normal_lu, solve_dense_lstsq, normal_residual,
                          dual, cg_normal)
from tests.conftest import to_oracle

IC, DIR, PER, NONE = ("dirichlet", "none"), ("dirichlet", "dirichlet"), ("periodic", "periodic"), ("none", "none")

TINY = [
    ((6, 6), (IC, DIR)),
    ((5, 7), (DIR, DIR)),
    ((6, 5), (IC, PER)),
    ((5, 5, 6), (IC, PER, PER)),
    ((5, 6, 5), (IC, DIR, DIR)),
]


@pytest.mark.parametrize("shape,bc", TINY)
def test_dense_brute_force(shape, bc):
    inst = W.random_instance(shape, bc, seed=len(shape) * 10 + shape[0])
    A, d, _ = assemble(to_oracle(inst))
    zd = solve_dense_lstsq(A, d)
    zk, lam, _ = solve_kkt(A, d)
    zn = solve_normal_lu(A, d)
    assert np.linalg.norm(zk - zd) <= 1e-9 * np.linalg.norm(zd)
    assert np.linalg.norm(zn - zd) <= 1e-7 * np.linalg.norm(zd)
    assert np.allclose(lam, dual(A, d, zk), atol=1e-10 * np.linalg.norm(d))
    # LS optimality: the residual is orthogonal to the columns of A ...
    assert normal_residual(A, d, zk) < 1e-10
    # ... and no perturbation does better.
    rng = np.random.default_rng(0)
    base = np.linalg.norm(A @ zk - d)
    for _ in range(5):
        assert np.linalg.norm(A @ (zk + 1e-3 * rng.standard_normal(zk.size)) - d) > base


@pytest.mark.parametrize("shape,bc", TINY)
def test_full_column_rank(shape, bc):
    inst = W.random_instance(shape, bc, seed=1)
    A, _, _ = assemble(to_oracle(inst))
    s = np.linalg.svd(A.toarray(), compute_uv=False)
    assert s[-1] > 1e-8 * s[0]


def test_generators_full_rank():
    for inst in (W.reaction_diffusion_1d(shape=(6, 6)), W.reaction_diffusion_1d_ragged(7, (6, 5)),
                 W.reaction_diffusion_2d(0, shape=(5, 6, 6)), W.advection_diffusion_2d(0, shape=(5, 6, 6))[0]):
        A, _, _ = assemble(to_oracle(inst))
        s = np.linalg.svd(A.toarray(), compute_uv=False)
        assert s[-1] > 1e-10 * s[0]


def test_periodic_translation_invariance():
    # Data independent of a periodic axis: the unique minimiser is independent
    # of it too, its derivative variables along that axis vanish, and it equals
    # the solution of the same problem without that axis.
    rng = np.random.default_rng(3)
    nt, nx, ny = 6, 7, 5
    mset2, mset3 = (0, 1, 3, 4), (0, 1, 3, 4)
    c2 = rng.uniform(-1, 1, (len(mset2), nt, nx))
    c2[1] = 1.0
    f2 = rng.standard_normal((nt, nx))
    w2 = rng.standard_normal((nt, nx))
    step2 = (0.2, 0.25)
    from oracle.system import OracleProblem
    p2 = OracleProblem((nt, nx), step2, (IC, DIR), mset2, c2, f2, w2)
    p3 = OracleProblem((nt, nx, ny), step2 + (0.3,), (IC, DIR, PER), mset3,
                       np.repeat(c2[..., None], ny, -1), np.repeat(f2[..., None], ny, -1),
                       np.repeat(w2[..., None], ny, -1))
    A2, d2, _ = assemble(p2)
    A3, d3, _ = assemble(p3)
    z2 = solve_kkt(A2, d2)[0].reshape(5, nt, nx)
    z3 = solve_kkt(A3, d3)[0].reshape(7, nt, nx, ny)
    for v in range(5):
        assert np.allclose(z3[v], z2[v][..., None], atol=1e-9 * np.abs(z2).max())
    assert np.abs(z3[5:]).max() < 1e-9 * np.abs(z2).max()


def test_cg_reference_matches_direct():
    inst = W.reaction_diffusion_1d(shape=(12, 12))
    A, d, _ = assemble(to_oracle(inst))
    zk = solve_kkt(A, d)[0]
    x, it, rel = cg_normal(A, A.T @ d, tol=1e-13, maxiter=50000)
    assert rel <= 1e-13
    assert np.linalg.norm(x - zk) <= 1e-5 * np.linalg.norm(zk)
