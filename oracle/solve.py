"""Least-squares solution of A z = d (Eqs. 8-10).

The method solves Eq. 8 in the least-squares sense through the normal
equations (Eq. 9) and obtains the dual variables from the saddle-point
system (Eq. 10)

    [ I   A ] [lambda*]   [d]
    [ A^T 0 ] [  z*   ] = [0]

whose solution is z* = argmin ||A z - d||^2 and lambda* = d - A z*.

* ``solve_kkt``        -- FP64 sparse LU (SuperLU) of the saddle-point matrix:
                          the primary oracle (conditioned like A, not A^T A).
* ``solve_normal_lu``  -- FP64 sparse LU of A^T A z = A^T d (cross-check).
* ``solve_dense_lstsq``-- dense numpy lstsq (brute force for tiny grids).
* ``cg_normal``        -- textbook Jacobi-preconditioned CG on the normal
                          equations in FP64, for sizes where a direct
                          factorisation does not fit in memory.
* ``normal_residual``  -- ||A^T(d - A z)|| / ||A^T d||, the relative residual
                          of the normal equations.

Oracle module: test infrastructure only.
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def kkt_matrix(A):
    nc, nv = A.shape
    return sp.bmat([[sp.identity(nc, format="csc"), A], [A.T, None]], format="csc")


def factor_kkt(A):
    """SuperLU factorisation of the saddle-point matrix of Eq. 10."""
    return spla.splu(kkt_matrix(A), permc_spec="COLAMD")


def solve_kkt(A, d, lu=None):
    """Return (z*, lambda*, lu) from the saddle-point system of Eq. 10."""
    nc, nv = A.shape
    if lu is None:
        lu = factor_kkt(A)
    sol = lu.solve(np.concatenate([d, np.zeros(nv)]))
    lam, z = sol[:nc], sol[nc:]
    return z, lam, lu


def solve_normal_lu(A, d):
    """z from a sparse LU of the normal equations (Eq. 9)."""
    AtA = (A.T @ A).tocsc()
    return spla.splu(AtA, permc_spec="COLAMD").solve(A.T @ d)


def solve_dense_lstsq(A, d):
    """Dense least squares (brute force, tiny systems only)."""
    z, *_ = np.linalg.lstsq(A.toarray(), d, rcond=None)
    return z


def dual(A, d, z):
    """lambda* = d - A z* (first block row of Eq. 10)."""
    return d - A @ z


def normal_residual(A, d, z):
    """Relative residual of the normal equations."""
    rhs = A.T @ d
    return float(np.linalg.norm(rhs - A.T @ (A @ z)) / np.linalg.norm(rhs))


def cg_normal(A, b, tol=1e-12, maxiter=200000, x0=None):
    """Jacobi-preconditioned conjugate gradients on A^T A x = b (FP64).

    Plain textbook PCG; ``b`` is the normal-equation right-hand side.
    Returns (x, iterations, final relative residual)."""
    diag = np.asarray(A.multiply(A).sum(axis=0)).ravel()
    minv = np.where(diag > 0, 1.0 / diag, 0.0)
    x = np.zeros(A.shape[1]) if x0 is None else x0.astype(np.float64).copy()
    r = b - A.T @ (A @ x)
    bn = np.linalg.norm(b)
    z = minv * r
    p = z.copy()
    rz = r @ z
    for it in range(1, maxiter + 1):
        q = A.T @ (A @ p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        rel = np.linalg.norm(r) / bn
        if rel <= tol:
            return x, it, rel
        z = minv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxiter, rel
