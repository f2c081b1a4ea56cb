// Internal declarations shared by the host runtime and the kernels of the
// MI355X NeuRLP-PDE solver.  Not part of the public ABI (include/mpde.h).
//
// Formulation used by every kernel (exact block elimination of the normal
// equations of Eq. 9):
//   The derivative unknowns of a grid point appear only in that point's own
//   constraint rows (equation row Eq. 3, Taylor rows Eqs. 6-7 and the two
//   central-difference rows Eq. 5 of every axis).  For a fixed field u they
//   are therefore the solution of a small local least-squares problem, and
//   A^T A z = A^T d reduces exactly to  S u = g  with the Schur complement
//       S = A_u^T Pi A_u,   Pi_i = I - A_w,i (A_w,i^T A_w,i)^-1 A_w,i^T,
//   a scalar-field operator.  Krylov iterations and multigrid run on u; the
//   derivative unknowns are recovered pointwise at the end.  Inside a point,
//   the derivative unknowns of axis a are carried in scaled form
//       p_a = s_a u_a,  q_a = s_a^2 u_aa,
//   so that the Taylor and difference rows have O(1) entries:
//       T+ : wT (u_i + p + q/2 - u_{i+e})      T- : wT (u_i - p + q/2 - u_{i-e})
//       C1 : wC1 (p - sum_k w1_k u_{i+o_k})    C2 : wC2 (q - sum_k w2_k u_{i+o_k})
//       E  : c_phi u_i + sum_a (c_a/s_a) p_a + (c_aa/s_a^2) q_a - f_i
//       B  : u_i - omega_i
//   (row weights wT = wC1 = wC2 = 1 on the finest grid; coarse grids use
//   level weights, see mpde_api.hip).  A_w,i^T A_w,i = G + c^ c^^T with G
//   block diagonal (2x2 per axis, depending only on which Taylor rows exist)
//   is inverted by Sherman-Morrison, so Pi_i couples the axes through one
//   scalar per point, gamma_i = (rho_E - sum_a c^_a.g_a) / kappa.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mpde {

constexpr int kMaxD = 3;
constexpr int kBlock = 256;

// One instance on one grid level.
struct LInst {
  int n[kMaxD];        // points per axis (unused axes: 1)
  int str[kMaxD];      // element stride of each axis
  int N;               // points of this instance on this level
  int per[kMaxD];      // periodic axis
  int dlo[kMaxD];      // Dirichlet face at index 0
  int dhi[kMaxD];      // Dirichlet face at index n-1
  int coarsest;        // this level is the instance's coarsest
  int ncoarsened;      // axes halved from the next finer level to this one
  int pad;
  double s[kMaxD];     // steps
  double is1[kMaxD];   // 1 / s
  double is2[kMaxD];   // 1 / s^2
  double wT[kMaxD], wC1[kMaxD], wC2[kMaxD];   // row weights per axis
  // Inverse of the per-axis 2x2 Gram block G_a for the three row classes
  // (0: both Taylor rows, 1: no T- (first point), 2: no T+ (last point)),
  // entries (i11, i12, i22); filled by the host.
  double gi[kMaxD][3][3];
  double cheb_theta, cheb_delta;              // Chebyshev interval of D^-1 S
  long long voff;      // offset (points) of this instance in level vectors
  long long coff;      // offset (elements) of its coefficient block (K planes)
  long long doff;      // offset (elements) of its dense coarsest inverse
  // Krylov gate: the instance's active flag in the copy of the level's
  // descriptors that the Krylov iterations launch with (kernels of an
  // iteration return at once for a converged instance); null elsewhere.
  const int* act;
  // FP32 copies of per-axis constants for the fused operator (FK_* indices):
  // wT^2, wT^2 / 2, wC1^2, wC2^2, 1/s, 1/s^2, the Gram inverses and
  // wC1^2 / 12, wC2^2 / 12.
  float fk[kMaxD][16];
};

__host__ __device__ inline bool gated_off(const LInst& L) { return L.act != nullptr && *L.act == 0; }

// Indices into LInst::fk.  Class 0 (both Taylor rows) has a diagonal Gram
// block, so only its two diagonal entries are kept.
enum FConst {
  FK_A = 0,     // wT^2
  FK_AH = 1,    // wT^2 / 2
  FK_B1 = 2,    // wC1^2
  FK_B2 = 3,    // wC2^2
  FK_S1 = 4,    // 1 / s
  FK_S2 = 5,    // 1 / s^2
  FK_G0 = 6,    // class 0: i11, i22
  FK_G1 = 8,    // class 1: i11, i12, i22
  FK_G2 = 11,   // class 2: i11, i12, i22
  FK_B1D = 14,  // wC1^2 / 12 (the centred 5-point weights are multiples of 1/12)
  FK_B2D = 15,  // wC2^2 / 12
};

// Variable -> coefficient plane (-1 = no field).
struct CIdx {
  int k[1 + 2 * kMaxD];
  int K;
};

// Block work item: instance id and first point handled by the block.
struct Work {
  int inst;
  int start;
};

enum GatherMode {
  G_STORE = 0,      // out = S u (- g when sigma = 1)
  G_RESID = 1,      // out = b - y (b may be null), d = dinv*out/theta if d != null
  G_CHEB = 2,       // Chebyshev step on (x, r, d = u): x += d, r -= y, d' = a d + c dinv r;
                    // d' must not alias u (neighbours of u are still being read)
  G_STORE_DOT = 3,  // out = y and per-block partial sum of u*y
};

}  // namespace mpde
