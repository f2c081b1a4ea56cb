"""Gradients through the least-squares solve (Eq. 11 and the formulas after
it, Sec. "Backward pass").

Given g_z = dl/dz*, the backward saddle-point system

    [ I   A ] [d_lambda]   [  0  ]
    [ A^T 0 ] [  d_z   ] = [ -g_z]

is solved with the same factorisation as the forward system; then

    dl/dA = d_lambda z*^T + lambda* d_z^T      (on the nonzeros of A)
    dl/dd = -d_lambda.

Chaining to the problem data of the canonical system: the coefficient
c_{m,p} is the entry of A in row E_p, column (m, p); the source f_p is
d[E_p]; omega_p is d[B_p].  Everything else in A depends only on the steps.

Oracle module: test infrastructure only.
"""

import numpy as np

from .solve import solve_kkt


def adjoint_kkt(A, lu, g_z):
    """Solve Eq. 11 with the LU of the forward saddle-point matrix."""
    nc, nv = A.shape
    sol = lu.solve(np.concatenate([np.zeros(nc), -np.asarray(g_z, np.float64)]))
    return sol[:nc], sol[nc:]          # d_lambda, d_z


def grad_A_entries(A, z, lam, dlam, dz):
    """dl/dA restricted to the sparsity pattern of A, as a CSR matrix with
    the same pattern: entry (r, k) = dlam_r z_k + lam_r dz_k."""
    G = A.copy().tocsr()
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    G.data = dlam[rows] * z[A.indices] + lam[rows] * dz[A.indices]
    return G


def chain_gradients(prob, A, rows, z, lam, dlam, dz):
    """Gradients of l w.r.t. (coeff [K,*shape], rhs [*shape], bc_values
    [*shape]) from the gradient w.r.t. A and d."""
    N = prob.npoints
    G = grad_A_entries(A, z, lam, dlam, dz)
    e_rows = rows["E"]
    flat = np.arange(N)
    gc = np.stack([np.asarray(G[e_rows, m * N + flat]).ravel() for m in prob.mset])
    gd = -dlam
    gf = gd[e_rows]
    gw = np.zeros(N)
    gw[rows["Bpoint"]] = gd[rows["B"]]
    return (gc.reshape((len(prob.mset),) + tuple(prob.shape)),
            gf.reshape(prob.shape), gw.reshape(prob.shape))


def fd_gradient(loss_of_param, x0, eps):
    """Central finite differences of a scalar function of a flat array."""
    x0 = np.asarray(x0, np.float64)
    g = np.zeros_like(x0)
    for i in range(x0.size):
        xp = x0.copy(); xp[i] += eps
        xm = x0.copy(); xm[i] -= eps
        g[i] = (loss_of_param(xp) - loss_of_param(xm)) / (2 * eps)
    return g


def solve_value(A, d):
    """Convenience: z* only (forward solve through Eq. 10)."""
    return solve_kkt(A, d)[0]
