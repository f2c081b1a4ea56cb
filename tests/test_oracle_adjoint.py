"""Pins of the backward pass (Eq. 11 and the gradient formulas after it)
against central finite differences of the FP64 oracle loss."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle.system import assemble
from oracle.solve import solve_kkt, factor_kkt
from oracle.adjoint import adjoint_kkt, grad_A_entries, chain_gradients, fd_gradient
from tests.conftest import to_oracle


def test_scalar_case():
    # A = [c], d = [f]: z* = f/c, l = z*  ->  dl/dc = -f/c^2, dl/dd = 1/c.
    c, f = 1.7, 0.6
    A = sp.csr_matrix([[c]])
    d = np.array([f])
    z, lam, lu = solve_kkt(A, d)
    dlam, dz = adjoint_kkt(A, lu, np.array([1.0]))
    G = grad_A_entries(A, z, lam, dlam, dz)
    assert np.isclose(G.toarray()[0, 0], -f / c ** 2)
    assert np.isclose(-dlam[0], 1 / c)


def test_random_overdetermined_ls():
    rng = np.random.default_rng(0)
    A = sp.random(9, 5, density=0.6, random_state=1, format="csr") + sp.eye(9, 5)
    A = A.tocsr()
    d = rng.standard_normal(9)
    g = rng.standard_normal(5)
    z, lam, lu = solve_kkt(A, d)
    dlam, dz = adjoint_kkt(A, lu, g)
    G = grad_A_entries(A, z, lam, dlam, dz)
    r, k = A.nonzero()

    def loss_A(vals):
        B = sp.csr_matrix((vals, (r, k)), shape=A.shape)
        return g @ solve_kkt(B, d)[0]
    vals0 = np.asarray(A[r, k]).ravel()
    fd = fd_gradient(loss_A, vals0, 1e-6)
    assert np.allclose(np.asarray(G[r, k]).ravel(), fd, rtol=1e-6, atol=1e-8)
    fdd = fd_gradient(lambda dd: g @ solve_kkt(A, dd)[0], d, 1e-6)
    assert np.allclose(-dlam, fdd, rtol=1e-6, atol=1e-9)


def test_pde_gradients_vs_fd():
    inst = W.reaction_diffusion_2d(0, shape=(5, 6, 5), dt=0.1)
    prob = to_oracle(inst)
    rng = np.random.default_rng(2)
    target = rng.standard_normal(prob.npoints * 7)
    # loss ~ 4e5: a step of 1e-3 keeps FD round-off below its O(eps^2) truncation

    def loss_of(p):
        A, d, _ = assemble(p)
        z = solve_kkt(A, d)[0]
        return 0.5 * np.sum((z - target) ** 2)

    A, d, rows = assemble(prob)
    z, lam, lu = solve_kkt(A, d)
    dlam, dz = adjoint_kkt(A, lu, z - target)
    gc, gf, gw = chain_gradients(prob, A, rows, z, lam, dlam, dz)
    idx = [(k, 1, 2, 3) for k in range(6)] + [(1, 4, 0, 1), (3, 0, 5, 4)]
    for (k, t, x, y) in idx:
        def lc(v, k=k, t=t, x=x, y=y):
            c = prob.coeff.copy(); c[k, t, x, y] = v[0]
            p = to_oracle(dict(inst, coeff=c))
            return loss_of(p)
        fd = fd_gradient(lc, [prob.coeff[k, t, x, y]], 1e-3)[0]
        assert np.isclose(gc[k, t, x, y], fd, rtol=1e-5, atol=1e-8), (k, t, x, y)
    for (t, x, y) in [(0, 0, 0), (2, 3, 1)]:
        def lf(v, t=t, x=x, y=y):
            f = prob.rhs.copy(); f[t, x, y] = v[0]
            return loss_of(to_oracle(dict(inst, rhs=f)))
        assert np.isclose(gf[t, x, y], fd_gradient(lf, [prob.rhs[t, x, y]], 1e-3)[0], rtol=1e-5, atol=1e-8)
        def lw(v, t=t, x=x, y=y):
            w = prob.bc_values.copy(); w[t, x, y] = v[0]
            return loss_of(to_oracle(dict(inst, bc_values=w)))
        assert np.isclose(gw[t, x, y], fd_gradient(lw, [prob.bc_values[t, x, y]], 1e-3)[0], rtol=1e-5, atol=1e-8)
    assert np.all(gw[1:] == 0)      # only the initial face is constrained
