/*
 * mpde.h -- C ABI of the MI355X (gfx950) solver for the NeuRLP-PDE
 * least-squares system of Mechanistic PDE Networks (arXiv 2502.18377).
 *
 * Problem (Sec. "Mechanistic PDE Networks", Eq. 1 and Eq. 2; Sec. "Linear PDE
 * Solving With Differentiable Optimization", Eqs. 3-10):
 *   a batch of linear space-time PDEs  sum_{m in M} c_m(t,x) u_m = b(t,x)
 *   with initial/boundary data u = omega on a set of faces, on a Cartesian
 *   grid of D axes (axis 0 = time, the last axis varies fastest in memory).
 *   Each grid point carries V = 1 + 2D unknowns, in the order
 *       u, u_{a0}, u_{a0 a0}, u_{a1}, u_{a1 a1}, ...
 *   (variable 1+2a / 2+2a = first / second derivative along axis a).
 *   The constraint rows -- equation rows at every point (Eq. 3), boundary
 *   rows on Dirichlet faces (Eq. 4), 5-point central-difference rows with
 *   one-sided windows at non-periodic edges (Eq. 5) and forward/backward
 *   Taylor rows (Eqs. 6-7) -- form A z = d (Eq. 8); the library returns the
 *   least-squares solution z* of the normal equations A^T A z = A^T d (Eq. 9)
 *   and gradients through it from the backward saddle-point system (Eq. 11).
 *
 * Memory and ownership: every pointer argument is owned by the caller.
 * Pointers documented "device" must be device memory on the current HIP
 * device; "host" pointers are host memory.  mpde_build copies what it needs
 * (coefficients, source, boundary data) into a library-owned hierarchy, so
 * the caller may free or overwrite its inputs after mpde_build returns.  The
 * problem handle owns that device memory until mpde_free.
 *
 * Batches may be ragged: all instances share D, the boundary types and the
 * multi-index set, but each has its own shape and steps.  Per-instance
 * blocks are concatenated in instance order:
 *   coeff     [sum_b K*N_b]   instance b: K planes of N_b points (mset order)
 *   rhs       [sum_b N_b]
 *   bc_values [sum_b N_b]     read on Dirichlet faces only
 *   z_out     [sum_b V*N_b]   instance b: V planes of N_b points
 * where N_b = prod_a shape[b][a] and K = popcount(mset).
 *
 * Return codes: 0 = success; > 0 = warning (MPDE_WARN_NOT_CONVERGED: at
 * least one instance did not reach the tolerance, see info.status);
 * < 0 = error (no partial results).  Arguments are validated on the host
 * before any device work; no C++ exception crosses this interface.  The last
 * error message of the calling thread is available from mpde_last_error().
 * Calls are synchronous with respect to the host: they enqueue on the given
 * stream and wait for it before returning.  One problem handle must not be
 * used from two threads at once.
 */
#ifndef MPDE_H
#define MPDE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  MPDE_OK = 0,
  MPDE_WARN_NOT_CONVERGED = 1,
  MPDE_ERR_INVALID_ARG = -1,
  MPDE_ERR_UNSUPPORTED = -2,
  MPDE_ERR_OUT_OF_MEMORY = -3,
  MPDE_ERR_HIP = -4,
  MPDE_ERR_NO_DEVICE = -5,
  MPDE_ERR_BAD_STATE = -6,
  MPDE_ERR_NONFINITE = -7
};

enum { MPDE_F32 = 0, MPDE_F64 = 1 };

enum { MPDE_BC_NONE = 0, MPDE_BC_DIRICHLET = 1, MPDE_BC_PERIODIC = 2 };

enum { MPDE_STATUS_CONVERGED = 0, MPDE_STATUS_NOT_CONVERGED = 1, MPDE_STATUS_NONFINITE = 2 };

/* Solver options (multigrid-preconditioned Krylov solve of the normal
 * equations, Sec. "An Iterative Sparse Multigrid Solver" and the V-cycle
 * algorithm of the appendix).  Fill with mpde_default_options first. */
typedef struct {
  double tol;            /* target relative residual of the normal equations,
                            ||A^T(d - A z)|| / ||A^T d||, per instance (1e-6) */
  double inner_tol;      /* relative reduction of each inner Krylov solve;
                            0 (default): per instance and outer step, the
                            reduction still needed (0.3 tol / relres),
                            clamped to [max(1e-4, sqrt(0.3 tol)), 0.1] in
                            F32 and [1e-10, 0.1] in F64 */
  int32_t max_outer;     /* outer refinement steps with an FP64 residual (30) */
  int32_t max_inner;     /* Krylov iterations per outer step (200) */
  int32_t nu;            /* smoothing steps before and after each coarse
                            correction (2) */
  int32_t coarse_min;    /* smallest coarsened periodic axis (8; axes go on
                            to 4 while the coarsest grid would exceed 4096
                            points); a non-periodic axis stops at >= 5 */
  int32_t check_every;   /* Krylov iterations between host convergence checks (2) */
  int32_t max_levels;    /* cap on grid levels including the finest (16) */
  int32_t profile;       /* nonzero: time the finest-grid operator kernels of
                            mpde_solve with HIP events (see mpde_kernel_stats) */
  int32_t out_f64;       /* nonzero: mpde_solve writes z_out as FP64 (the FP64
                            iterate) even for an MPDE_F32 problem (0) */
  int32_t graph;         /* nonzero: replay the Krylov iterations between
                            host convergence checks as captured HIP graphs
                            (1; ignored while profiling or with a network) */
  int32_t fused;         /* nonzero: FP32 levels with three axes (t, x, y), x
                            and y periodic, use the one-pass operator kernel
                            that evaluates every row once (1); zero: the
                            two-pass kernels (same operator, other rounding) */
  int32_t time_chunks;   /* one-pass operator: time chunks per tile, each
                            with two halo row planes per side (same sums):
                            0 = tiles and chunks chosen per launch from a
                            cost model (default), 1 = whole time axis, 2 or
                            4 = that many where the time axis allows */
  int32_t reserved[3];
} mpde_options;

/* Problem description (the encoder outputs of Eq. 2 with uniform steps). */
typedef struct {
  int32_t dtype;          /* MPDE_F32 or MPDE_F64: element type of coeff, rhs,
                             bc_values, z_out, g_z and the gradient outputs */
  int32_t ndim;           /* D = 2 or 3 axes, axis 0 = time */
  int32_t batch;          /* B >= 1 instances */
  const int32_t *shape;   /* host [B][D] points per axis; every axis >= 5 */
  const double *step;     /* host [B][D] uniform step per axis, > 0 */
  int32_t bc_lo[3];       /* per axis, face at index 0: MPDE_BC_*  */
  int32_t bc_hi[3];       /* per axis, face at index n-1; PERIODIC must be set
                             on both faces of an axis or on neither */
  uint32_t mset;          /* bit v set = variable v has a coefficient field in
                             the equation row; bits >= V must be clear; at
                             least one bit set */
  const void *coeff;      /* device, see layout above */
  const void *rhs;        /* device, the source b of Eq. 1 */
  const void *bc_values;  /* device, omega of Eq. 4 */
  void *stream;           /* hipStream_t to run on (NULL = null stream) */
  const mpde_options *opts; /* host, NULL = defaults */
} mpde_desc;

/* Per-call report; every array is host memory of length >= batch, or NULL. */
typedef struct {
  int32_t *iters;         /* total inner Krylov iterations per instance */
  int32_t *outer;         /* outer refinement steps per instance */
  double *relres;         /* final relative residual of the normal equations */
  int32_t *status;        /* MPDE_STATUS_* */
  double seconds;         /* wall time of the call (output) */
} mpde_info;

typedef struct mpde_problem mpde_problem;   /* opaque, library-owned */

/* Fill *o with the defaults above.  Returns MPDE_ERR_INVALID_ARG if o is NULL. */
int mpde_default_options(mpde_options *o);

/* Validate *d (host only), plan the grid hierarchy (each spatial axis is
 * halved while it stays at or above the minimum size; time is never
 * coarsened), copy and coarsen the coefficient fields to every level and
 * factor the coarsest-level operators.  On success *out receives a new
 * handle that the caller releases with mpde_free.  Errors: INVALID_ARG,
 * UNSUPPORTED, OUT_OF_MEMORY, HIP, NO_DEVICE.  Sec. "An Iterative Sparse
 * Multigrid Solver" (coarse grids by halving with doubled steps, coefficients
 * coarsened by interpolation). */
int mpde_build(const mpde_desc *d, mpde_problem **out);

/* Solve A^T A z = A^T d (Eq. 9) for every instance and write z* to z_out
 * (device, [sum_b V*N_b], dtype of the problem, or FP64 if options.out_f64).  Keeps an internal copy of
 * u* for mpde_solve_adjoint.  info may be NULL.  Returns 0, or
 * MPDE_WARN_NOT_CONVERGED (z_out holds the best iterate), or an error. */
int mpde_solve(mpde_problem *p, void *z_out, mpde_info *info);

/* Backward pass (Eq. 11 and the gradient formulas after it): given
 * g_z = dl/dz* (device, [sum_b V*N_b]) solve A^T A d_z = g_z, form
 * d_lambda = -A d_z and lambda* = d - A z*, and write
 *   grad_coeff [sum_b K*N_b] = d_lambda_E z*_m + lambda*_E d_z_m  (per point)
 *   grad_rhs   [sum_b N_b]   = -d_lambda_E
 *   grad_bc    [sum_b N_b]   = -d_lambda_B on constrained points, 0 elsewhere
 * Any of the three outputs may be NULL.  Requires a prior successful
 * mpde_solve on p (else MPDE_ERR_BAD_STATE). */
int mpde_solve_adjoint(mpde_problem *p, const void *g_z, void *grad_coeff,
                       void *grad_rhs, void *grad_bc, mpde_info *info);

/* Release the handle and its device memory; NULL is a no-op. */
void mpde_free(mpde_problem *p);

/* Message of the last error on the calling thread ("" if none). */
const char *mpde_last_error(void);

/* Kernel statistics of the last mpde_solve run with options.profile set:
 * one record per kernel family on the finest grid ("gamma": the per-point
 * projection pass, "gather": the operator/smoother pass of the two-pass
 * kernels, "apply3": the one-pass three-axis operator), with launches,
 * summed device time in ms (HIP events on the problem's stream) and the
 * algorithmic HBM bytes those launches must move (inputs read once, outputs
 * written once).  Writes at most max records to out (host) and returns the
 * number of records available (0 if p is NULL or profiling was off). */
typedef struct {
  char name[32];
  int64_t launches;
  double ms;
  double bytes;
} mpde_kstat;
int mpde_kernel_stats(const mpde_problem *p, mpde_kstat *out, int32_t max);

/* Timing of the finest-grid operator pass (the matrix-free normal-equation
 * operator of Eq. 9 in reduced form, fused with the epilogue `mode`: 0 y = S u,
 * 1 residual, 2 Chebyshev smoothing step, 3 y = S u with per-block u.y
 * partial sums, 4 the FP64 residual r = b - S u of the outer refinement, in
 * FP64 arithmetic on FP64 vectors): `reps` launches back to back on the
 * problem's stream on the library's own level-0 work vectors, between two HIP
 * events.  Writes the mean duration per launch in microseconds and the
 * algorithmic HBM bytes of one launch (inputs read once, outputs written
 * once).  Overwrites only library scratch vectors: a later mpde_solve or
 * mpde_solve_adjoint is unaffected.  Returns MPDE_ERR_INVALID_ARG for a NULL
 * problem or output, mode outside 0..4 or reps < 1, and
 * MPDE_ERR_UNSUPPORTED for mode 4 on a problem without a fused FP64 pass
 * (FP64 coefficients, fused operator off, or a level shape it does not
 * cover). */
int mpde_time_operator(mpde_problem *p, int32_t mode, int32_t reps, double *us_per_launch,
                       double *bytes_per_launch);

/* ---------------------------------------------------------------------
 * Learned coarse-grid correction (an addition to the paper's solver): a
 * 3-layer 3x3x3 convolution network, 16 channels, BF16 weights with FP32
 * accumulation, mapping the normalised restricted residual plus the
 * coefficient fields of a grid level to the coarse-grid correction, used in
 * place of the recursive V-cycle below that level inside flexible CG.  It
 * is trained on systems built by mpde_build with the solver's own operator:
 * the loss is the energy-norm error o^T S o - 2 o^T r of the prediction o for
 * a unit residual r (minimised by o = S^-1 r).
 * ------------------------------------------------------------------- */
typedef struct mpde_net mpde_net;   /* opaque, library-owned weights + Adam state */

/* Parameters of a network: 3 layers x (27*16*16 weights [tap][out][in] +
 * 16 biases), FP32 master copy. */
#define MPDE_NET_PARAMS (3 * (27 * 16 * 16 + 16))

/* New network on the current device with seeded (He-scaled) weights; the
 * last layer starts at zero (an untrained network is plain multigrid).  in_channels (2..16) = 2 + K: the normalised
 * residual, the plain V-cycle's coarse correction (Jacobi units) and the K
 * coefficient fields of the level.  The network refines the plain
 * correction: e = V(r) + D^-1 N(r, V(r), c) ||r||, so N = 0 is plain MG. */
int mpde_net_create(int32_t in_channels, uint64_t seed, mpde_net **out);

/* One Adam step (learning rate lr) on residual samples drawn from problem p
 * at grid level `level` (>= 1): a random right-hand side per instance is
 * smoothed on the finer levels and restricted, exactly as in a V-cycle.
 * The loss of a coarse correction o is the energy on the next finer level
 * f = level - 1 of its prolongation, (P o)^T S_f (P o) - 2 (P o)^T r_f, with
 * r_f the pre-smoothed finer residual, both normalised by ||R r_f||; its
 * minimiser is the Galerkin coarse correction (P^T S_f P)^-1 P^T r_f, which
 * the rediscretised coarse operator only approximates.  *loss and
 * *loss_plain (host, may be NULL) receive the mean loss of the learned
 * correction and of the plain V-cycle's on the same samples (lower is
 * better).
 * Errors: INVALID_ARG (bad level / mismatched channels), UNSUPPORTED (FP64
 * problem), HIP. */
int mpde_net_train_step(mpde_net *net, mpde_problem *p, int32_t level, uint64_t seed, double lr, double *loss,
                        double *loss_plain);

/* Use net (borrowed; it must outlive its use) for the coarse correction of
 * level `level` in later mpde_solve / mpde_solve_adjoint calls on p; the
 * Krylov method becomes flexible CG.  net == NULL restores plain multigrid. */
int mpde_net_attach(mpde_problem *p, const mpde_net *net, int32_t level);

/* Copy the FP32 master parameters out of / into a network (host arrays of
 * n >= MPDE_NET_PARAMS floats). */
int mpde_net_get(const mpde_net *net, float *host, int64_t n);
int mpde_net_set(mpde_net *net, const float *host, int64_t n);
void mpde_net_free(mpde_net *net);

/* One convolution layer (parity and training building block).  x_bf16:
 * device [batch][T][X][Y][16] bf16; w_bf16: device [27][16][16] bf16 indexed
 * [tap][out][in] for sign = +1 (forward) or [tap][in][out] (the transposed
 * weights) with sign = -1 (data gradient: taps mirrored); bias: device [16]
 * FP32 or NULL; outputs y (device FP32, same shape) and/or y_bf16 (bf16 of
 * relu(y) if relu != 0, else of y); either may be NULL.  Taps are ordered
 * (dt, dx, dy) in {-1,0,1}^3 with dt slowest; periodic[a] selects
 * wrap-around, otherwise zero padding. */
int mpde_conv3d(const void *x_bf16, const void *w_bf16, const float *bias, float *y, void *y_bf16,
                int32_t relu, int32_t sign, int32_t batch, int32_t T, int32_t X, int32_t Y,
                const int32_t *periodic, void *stream);

/* Weight gradient of one layer: dw[27][16][16] (device FP32) =
 * sum over points of dy[p][out] * x[p + off(tap)][in]. */
int mpde_conv3d_wgrad(const void *x_bf16, const void *dy_bf16, float *dw, int32_t batch, int32_t T, int32_t X,
                      int32_t Y, const int32_t *periodic, void *stream);

/* Autotuner: time complete solves of p for candidate settings of the
 * smoothing steps (nu), the inner Krylov tolerance and the number of Krylov
 * iterations per captured graph / host check, by coordinate search, and keep
 * the fastest in p's options.  chosen (host, may be NULL) receives
 * {nu, check_every, inner_tol * 1e9} of the winner (inner_tol 0: the
 * adaptive default); *best_ms its solve time.
 * The solution state of p is overwritten (call mpde_solve afterwards). */
int mpde_autotune(mpde_problem *p, void *z_scratch, int32_t *chosen, double *best_ms);

/* Grid levels planned for instance b (0 if p is NULL or b out of range);
 * if shapes is not NULL it receives levels*D points-per-axis values. */
int mpde_levels(const mpde_problem *p, int32_t b, int32_t *shapes);

#ifdef __cplusplus
}
#endif

#endif /* MPDE_H */
