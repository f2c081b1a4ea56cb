"""Seeded synthetic PDE instances for the NeuRLP-PDE solve.

This module only builds inputs (grids, coefficient fields, sources, initial
and boundary data, manufactured solutions); it holds none of the solver's
arithmetic (no constraint rows, no stencils, no least squares).  Both the
FP64 oracle and the GPU path consume its output, and nothing else is shared
between them.

An instance is a dict:
    shape      tuple of points per axis, axis 0 = time (D = len(shape))
    step       tuple of uniform spacings
    bc         tuple per axis of (lo, hi) in {"none","dirichlet","periodic"}
    mset       sorted variable indices with a coefficient field; variable 0 is
               u, 1+2a / 2+2a the first / second derivative along axis a
    coeff      float64 [K, *shape], in mset order
    rhs        float64 [*shape]  (the source b of the linear PDE)
    bc_values  float64 [*shape]  (omega; read on Dirichlet faces only)
    exact      optional dict var-index -> float64 [*shape] of a known
               continuous solution and its derivatives
All randomness comes from numpy.random.Generator(PCG64(seed)).

Workloads (the five shapes of the benchmark suite):
  reaction_diffusion_1d   1D+time, 32x32, variable-coefficient reaction-advection-diffusion
            with manufactured u* = exp(-t) sin(pi x); Dirichlet in x, initial
            data at t = 0.
  reaction_diffusion_2d   2D+time, 32x64x64, periodic space, Fourier-mode coefficient
            fields, Gaussian-random-field initial data, zero source.
  reaction_diffusion_1d_ragged   reaction_diffusion_1d with each axis drawn from {16,24,32,48,64}.
  advection_diffusion_2d   2D+time advection-diffusion with a divergence-free velocity from
            a 16-mode random streamfunction, 32x128x128.
  reaction_diffusion_2d_large   the reaction_diffusion_2d generator at 64x128x128.
"""

import numpy as np

VAR_NAMES2 = ("u", "u_t", "u_tt", "u_x", "u_xx")
VAR_NAMES3 = ("u", "u_t", "u_tt", "u_x", "u_xx", "u_y", "u_yy")
RAGGED_SIZES = (16, 24, 32, 48, 64)


def rng_for(family, instance):
    return np.random.Generator(np.random.PCG64(1000 * family + instance))


def _box5(a, axis):
    """Separable 5-point box mean along one axis, 'nearest' edge padding."""
    pad = [(0, 0)] * a.ndim
    pad[axis] = (2, 2)
    ap = np.pad(a, pad, mode="edge")
    n = a.shape[axis]
    return sum(np.take(ap, np.arange(k, k + n), axis=axis) for k in range(5)) / 5.0


def _grid(shape, step):
    return np.meshgrid(*[np.arange(n) * s for n, s in zip(shape, step)], indexing="ij")


# ------------------------------------------- 1D + time reaction-diffusion
def reaction_diffusion_1d(seed=None, shape=(32, 32), rng=None):
    """u_t = a u_xx + b u_x + c u + f on [0,1]^2 (t, x), Dirichlet in x and
    initial data at t = 0, with f manufactured from u* = exp(-t) sin(pi x)."""
    rng = rng if rng is not None else rng_for(1, 0 if seed is None else seed)
    nt, nx = shape
    step = (1.0 / (nt - 1), 1.0 / (nx - 1))
    a = rng.uniform(0.1, 1.0, shape)
    b = _box5(_box5(rng.uniform(-1.0, 1.0, shape), 0), 1)
    c = _box5(_box5(rng.uniform(-1.0, 1.0, shape), 0), 1)
    T, X = _grid(shape, step)
    u = np.exp(-T) * np.sin(np.pi * X)
    ut = -u
    ux = np.pi * np.exp(-T) * np.cos(np.pi * X)
    uxx = -np.pi ** 2 * u
    f = ut - a * uxx - b * ux - c * u
    mset = (0, 1, 3, 4)                       # phi, t, x, xx
    coeff = np.stack([-c, np.ones(shape), -b, -a])
    return dict(shape=tuple(shape), step=step,
                bc=(("dirichlet", "none"), ("dirichlet", "dirichlet")),
                mset=mset, coeff=coeff, rhs=f, bc_values=u.copy(),
                exact={0: u, 1: ut, 2: u, 3: ux, 4: uxx})


def ragged_shapes(count=256, seed=0):
    rng = rng_for(3, 10_000 + seed)
    return [tuple(int(v) for v in rng.choice(RAGGED_SIZES, size=2)) for _ in range(count)]


def reaction_diffusion_1d_ragged(instance, shape):
    """One instance of the 1D + time workload of the given (n_t, n_x)."""
    return reaction_diffusion_1d(shape=shape, rng=rng_for(3, instance))


# ------------------------------------------- 2D + time reaction-diffusion
def _fourier_field(rng, shape, step, nmodes=8, kmax=3, time_modes=True):
    T, X, Y = _grid(shape, step)
    tf = max((shape[0] - 1) * step[0], 1e-30)
    S = np.zeros(shape)
    for _ in range(nmodes):
        alpha = rng.uniform(-0.5, 0.5)
        kx, ky = rng.integers(-kmax, kmax + 1, size=2)
        kt = rng.integers(0, 2) if time_modes else 0
        th = rng.uniform(0, 2 * np.pi)
        S += alpha * np.cos(2 * np.pi * (kx * X + ky * Y + kt * T / tf) + th)
    return S


def gaussian_random_field(rng, shape, length=0.1):
    """Periodic squared-exponential Gaussian random field on [0,1)^d with
    the given length scale, normalised to zero mean and unit variance."""
    w = rng.standard_normal(shape)
    ks = np.meshgrid(*[np.fft.fftfreq(n, d=1.0 / n) for n in shape], indexing="ij")
    k2 = sum(k * k for k in ks)
    amp = np.exp(-(2 * np.pi * length) ** 2 * k2 / 4.0)
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
    g -= g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def reaction_diffusion_2d(instance=0, shape=(32, 64, 64), family=2, dt=None):
    """u_t = D (u_xx + u_yy) + v . grad u + r u on (t, x, y), x, y periodic on
    [0,1), initial data a Gaussian random field (length 0.1), zero source."""
    rng = rng_for(family, instance)
    nt, nx, ny = shape
    sx, sy = 1.0 / nx, 1.0 / ny
    st = dt if dt is not None else sx        # time step equal to the space step
    step = (st, sx, sy)
    SD = _fourier_field(rng, shape, step)
    Dc = 1.0 + 0.5 * SD / max(np.abs(SD).max(), 1e-30)
    vx = _fourier_field(rng, shape, step)
    vy = _fourier_field(rng, shape, step)
    r = _fourier_field(rng, shape, step)
    ic = gaussian_random_field(rng, (nx, ny), 0.1)
    omega = np.zeros(shape)
    omega[0] = ic
    mset = (0, 1, 3, 4, 5, 6)                 # phi, t, x, xx, y, yy
    coeff = np.stack([-r, np.ones(shape), -vx, -Dc, -vy, -Dc])
    return dict(shape=tuple(shape), step=step,
                bc=(("dirichlet", "none"), ("periodic", "periodic"), ("periodic", "periodic")),
                mset=mset, coeff=coeff, rhs=np.zeros(shape), bc_values=omega)


def reaction_diffusion_2d_large(instance=0, shape=(64, 128, 128), dt=None):
    return reaction_diffusion_2d(instance, shape=shape, family=5, dt=dt)


# ------------------------------------------- 2D + time advection-diffusion
def advection_diffusion_2d(instance=0, shape=(32, 128, 128), dt=None):
    """u_t + v . grad u = kappa (u_xx + u_yy) + f, v = (psi_y, -psi_x) from a
    16-mode random streamfunction scaled to max|v| = 1; kappa ~ U[0.005,0.05]
    per instance; f an 8-mode field; returns (instance, target field)."""
    rng = rng_for(4, instance)
    nt, nx, ny = shape
    sx, sy = 1.0 / nx, 1.0 / ny
    st = dt if dt is not None else sx
    step = (st, sx, sy)
    T, X, Y = _grid(shape, step)
    ks = [(kx, ky) for kx in range(-4, 5) for ky in range(-4, 5) if (kx, ky) != (0, 0)]
    pick = rng.choice(len(ks), size=16, replace=False)
    psix = np.zeros(shape)
    psiy = np.zeros(shape)
    for idx in pick:
        kx, ky = ks[idx]
        al = rng.uniform(-0.5, 0.5)
        th = rng.uniform(0, 2 * np.pi)
        sarg = np.sin(2 * np.pi * (kx * X + ky * Y) + th)
        psix += -al * 2 * np.pi * kx * sarg
        psiy += -al * 2 * np.pi * ky * sarg
    vx, vy = psiy, -psix
    vmax = max(np.sqrt(vx * vx + vy * vy).max(), 1e-30)
    vx, vy = vx / vmax, vy / vmax
    kappa = rng.uniform(0.005, 0.05)
    f = _fourier_field(rng, shape, step)
    ic = gaussian_random_field(rng, (nx, ny), 0.1)
    omega = np.zeros(shape)
    omega[0] = ic
    target = gaussian_random_field(rng, shape, 0.1)
    mset = (0, 1, 3, 4, 5, 6)
    kap = np.full(shape, kappa)
    coeff = np.stack([np.zeros(shape), np.ones(shape), vx, -kap, vy, -kap])
    inst = dict(shape=tuple(shape), step=step,
                bc=(("dirichlet", "none"), ("periodic", "periodic"), ("periodic", "periodic")),
                mset=mset, coeff=coeff, rhs=f, bc_values=omega, kappa=kappa)
    return inst, target


# ------------------------------------------------------- manufactured cases
def quadratic_exact(shape, bc, mset, seed=0, step=None):
    """Random coefficients and a solution that is a tensor-product quadratic
    in every non-periodic axis and constant along periodic axes, with the
    source f = sum_m c_m d_m u* and omega = u* taken from it exactly."""
    rng = np.random.Generator(np.random.PCG64(777 + seed))
    D = len(shape)
    step = step if step is not None else tuple(1.0 / (n - 1) for n in shape)
    grids = _grid(shape, step)
    per = [bc[a][0] == "periodic" for a in range(D)]
    degs = [0 if per[a] else 2 for a in range(D)]
    # u = sum over multi-degrees alpha of c_alpha prod x_a^alpha_a
    terms = []
    for alpha in np.ndindex(*[d + 1 for d in degs]):
        terms.append((alpha, rng.uniform(-1, 1)))

    def deriv(axis, order):
        out = np.zeros(shape)
        for alpha, ca in terms:
            if axis is not None and alpha[axis] < order:
                continue
            val = np.full(shape, ca)
            for a in range(D):
                p = alpha[a] - (order if a == axis else 0)
                coef = 1.0
                if a == axis:
                    for k in range(order):
                        coef *= alpha[a] - k
                val = val * coef * grids[a] ** p
            out += val
        return out

    exact = {0: deriv(None, 0)}
    for a in range(D):
        exact[1 + 2 * a] = deriv(a, 1)
        exact[2 + 2 * a] = deriv(a, 2)
    coeff = rng.uniform(-1, 1, (len(mset),) + tuple(shape))
    f = sum(coeff[k] * exact[m] for k, m in enumerate(mset))
    return dict(shape=tuple(shape), step=step, bc=tuple(bc), mset=tuple(mset),
                coeff=coeff, rhs=f, bc_values=exact[0].copy(), exact=exact)


def laplace2d(n):
    """Laplace u_xx + u_yy = 0 on [0,1]^2 (no time axis; axis 0 plays x),
    all faces Dirichlet, exact u = sin(pi x) sinh(pi y) / sinh(pi)."""
    shape = (n, n)
    step = (1.0 / (n - 1), 1.0 / (n - 1))
    X, Y = _grid(shape, step)
    u = np.sin(np.pi * X) * np.sinh(np.pi * Y) / np.sinh(np.pi)
    return dict(shape=shape, step=step,
                bc=(("dirichlet", "dirichlet"), ("dirichlet", "dirichlet")),
                mset=(2, 4), coeff=np.ones((2,) + shape), rhs=np.zeros(shape),
                bc_values=u.copy(), exact={0: u})


def random_instance(shape, bc, mset=None, seed=0):
    """Generic random instance (uniform coefficients in [-1,1], with the
    highest time/space derivative coefficients kept away from zero)."""
    rng = np.random.Generator(np.random.PCG64(4242 + seed))
    D = len(shape)
    V = 1 + 2 * D
    mset = tuple(range(V)) if mset is None else tuple(mset)
    coeff = rng.uniform(-1, 1, (len(mset),) + tuple(shape))
    step = tuple((1.0 / shape[a]) if bc[a][0] == "periodic" else 1.0 / (shape[a] - 1)
                 for a in range(D))
    return dict(shape=tuple(shape), step=step, bc=tuple(bc), mset=mset, coeff=coeff,
                rhs=rng.standard_normal(shape), bc_values=rng.standard_normal(shape))
