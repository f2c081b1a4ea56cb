"""Assembly of the NeuRLP-PDE constraint system A z = d (Eq. 8).

Grid and variables (Sec. "Discretization" and "Variables"):
  * D axes, axis 0 is time; axis a has n_a points at spacing s_a (point i_a
    sits at i_a * s_a), flattened in C order (last axis fastest).
  * every grid point carries V = 1 + 2D variables, in the order
        u, u_{a0}, u_{a0 a0}, u_{a1}, u_{a1 a1}, ...
    i.e. variable 0 is u and variables 1+2a / 2+2a are the first / second
    derivative along axis a.  z is stored variable-major: column v*N + p.
  * the multi-index set M is given as the sorted list of variable indices
    that carry a coefficient field (``mset``); phi (u itself) is index 0.

Rows, every row with weight 1 (residual form "A z - d"):
  E_p      (Eq. 3)  at every point:       sum_{m in M} c_{m,p} z_{m,p} - f_p
  B_p      (Eq. 4)  at every point of a Dirichlet face (once per point):
                                          z_{u,p} - omega_p
  T+_{a,p} (Eq. 6)  where p+e_a exists (always on a periodic axis):
                     z_{u,p} + s z_{a,p} + s^2/2 z_{aa,p} - z_{u,p+e_a}
  T-_{a,p} (Eq. 7)  where p-e_a exists:
                     z_{u,p} - s z_{a,p} + s^2/2 z_{aa,p} - z_{u,p-e_a}
  C1_{a,p} (Eq. 5)  at every point:       s z_{a,p}    - sum_k w1_k z_{u,p+o_k e_a}
  C2_{a,p} (Eq. 5)  at every point:       s^2 z_{aa,p} - sum_k w2_k z_{u,p+o_k e_a}
with the 5-point windows of ``stencil.window_offsets``.  Rows are ordered
E, B, then per axis T+, T-, C1, C2.

Oracle module: test infrastructure only.
"""

from dataclasses import dataclass, field
import numpy as np
import scipy.sparse as sp

from .stencil import fd_weights, window_offsets

NONE, DIRICHLET, PERIODIC = "none", "dirichlet", "periodic"


def variable_count(ndim):
    """V = 1 + 2D variables per grid point."""
    return 1 + 2 * ndim


@dataclass
class OracleProblem:
    shape: tuple            # points per axis, axis 0 = time
    step: tuple             # uniform spacing per axis
    bc: tuple               # per axis (lo, hi) in {"none","dirichlet","periodic"}
    mset: tuple             # sorted variable indices carrying a coefficient
    coeff: np.ndarray       # [K, *shape] float64
    rhs: np.ndarray         # [*shape]    float64 (the paper's b)
    bc_values: np.ndarray   # [*shape]    float64 (omega; read on Dirichlet faces)
    meta: dict = field(default_factory=dict)

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def npoints(self):
        return int(np.prod(self.shape))

    def periodic(self, a):
        lo, hi = self.bc[a]
        if (lo == PERIODIC) != (hi == PERIODIC):
            raise ValueError("periodic must be set on both ends of an axis")
        return lo == PERIODIC

    def boundary_mask(self):
        """Points on any Dirichlet face (each counted once)."""
        mask = np.zeros(self.shape, dtype=bool)
        for a, (lo, hi) in enumerate(self.bc):
            idx = [slice(None)] * self.ndim
            if lo == DIRICHLET:
                idx[a] = 0
                mask[tuple(idx)] = True
            if hi == DIRICHLET:
                idx[a] = self.shape[a] - 1
                mask[tuple(idx)] = True
        return mask


def _check(prob):
    D = prob.ndim
    if len(prob.step) != D or len(prob.bc) != D:
        raise ValueError("shape, step and bc must have one entry per axis")
    V = variable_count(D)
    if any(m < 0 or m >= V for m in prob.mset) or list(prob.mset) != sorted(set(prob.mset)):
        raise ValueError("mset must be sorted distinct variable indices")
    K = len(prob.mset)
    if prob.coeff.shape != (K,) + tuple(prob.shape):
        raise ValueError("coeff must be [K, *shape]")
    for a in range(D):
        prob.periodic(a)
        if prob.shape[a] < 5:
            raise ValueError("every axis needs at least 5 points")


def assemble(prob):
    """Return (A, d, rows) with A a scipy CSR matrix [n_c, n_v], d float64
    [n_c] and ``rows`` a dict of row-index arrays per row kind:
    rows["E"][p] is the E row of point p (all points), rows["B"] the B rows
    and rows["Bpoint"] the flat point each B row belongs to."""
    _check(prob)
    D, N, V = prob.ndim, prob.npoints, variable_count(prob.ndim)
    shape = tuple(prob.shape)
    pts = np.arange(N).reshape(shape)
    coords = np.indices(shape).reshape(D, N)     # coords[a][p] = i_a
    flat = pts.reshape(N)

    R, C, X = [], [], []     # COO triplets
    d_parts = []
    rows = {}
    nrow = 0

    def add(row_ids, col_ids, vals):
        R.append(np.asarray(row_ids, dtype=np.int64))
        C.append(np.asarray(col_ids, dtype=np.int64))
        X.append(np.asarray(vals, dtype=np.float64))

    # E rows (Eq. 3): one per point.
    e_rows = nrow + flat
    for k, m in enumerate(prob.mset):
        add(e_rows, m * N + flat, prob.coeff[k].reshape(N))
    d_parts.append(prob.rhs.reshape(N).astype(np.float64))
    rows["E"] = e_rows
    nrow += N

    # B rows (Eq. 4): one per constrained point.
    bpts = flat[prob.boundary_mask().reshape(N)]
    b_rows = nrow + np.arange(bpts.size)
    add(b_rows, bpts, np.ones(bpts.size))
    d_parts.append(prob.bc_values.reshape(N)[bpts].astype(np.float64))
    rows["B"], rows["Bpoint"] = b_rows, bpts
    nrow += bpts.size

    for a in range(D):
        n, s, per = shape[a], float(prob.step[a]), prob.periodic(a)
        ia = coords[a]
        va, vaa = 1 + 2 * a, 2 + 2 * a

        def shifted(off):
            """Flat index of p + off*e_a (wrapped on periodic axes)."""
            j = ia + off
            if per:
                j = j % n
            return flat + (j - ia) * (N // np.prod(shape[: a + 1])), j

        # T+ (Eq. 6) and T- (Eq. 7)
        for sign in (+1, -1):
            nb, j = shifted(sign)
            ok = np.ones(N, bool) if per else (j >= 0) & (j < n)
            p = flat[ok]
            r = nrow + np.arange(p.size)
            add(r, p, np.ones(p.size))
            add(r, va * N + p, np.full(p.size, sign * s))
            add(r, vaa * N + p, np.full(p.size, 0.5 * s * s))
            add(r, nb[ok], -np.ones(p.size))
            d_parts.append(np.zeros(p.size))
            rows[("T+" if sign > 0 else "T-", a)] = r
            nrow += p.size

        # C1 / C2 (Eq. 5): every point, 5-point windows.
        for q, vq in ((1, va), (2, vaa)):
            r = nrow + flat
            add(r, vq * N + flat, np.full(N, s ** q))
            for i in range(n):
                offs = window_offsets(i, n, per)
                w = fd_weights(offs, q)
                sel = flat[ia == i]
                for o, wk in zip(offs, w):
                    if wk == 0.0:
                        continue
                    j = (i + o) % n if per else i + o
                    add(r[sel], sel + (j - i) * (N // np.prod(shape[: a + 1])),
                        np.full(sel.size, -wk))
            d_parts.append(np.zeros(N))
            rows[("C1" if q == 1 else "C2", a)] = r
            nrow += N

    A = sp.coo_matrix((np.concatenate(X), (np.concatenate(R), np.concatenate(C))),
                      shape=(nrow, V * N)).tocsr()
    A.sum_duplicates()
    d = np.concatenate(d_parts)
    return A, d, rows


def exact_variables(shape, step, funcs):
    """Stack grid samples of (u, u_a, u_aa, ...) given callables
    funcs[v](*coords) -> array, in variable order; returns z [V*N]."""
    D = len(shape)
    grids = np.meshgrid(*[np.arange(n) * s for n, s in zip(shape, step)], indexing="ij")
    V = variable_count(D)
    return np.concatenate([np.broadcast_to(funcs[v](*grids), shape).reshape(-1)
                           for v in range(V)]).astype(np.float64)
