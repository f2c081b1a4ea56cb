// HIP kernels (gfx950) of the NeuRLP-PDE solver: the matrix-free reduced
// normal-equation operator, Chebyshev smoothing, grid transfers, the dense
// coarsest-grid solve, Krylov reductions and vector updates, the output of
// all derivative unknowns, and the backward-pass kernels.
//
// Every kernel is thread-per-grid-point over a table of (instance, first
// point) work items, so uniform and ragged batches share one launch per
// stage; blocks never straddle two instances, which keeps every per-instance
// reduction in a fixed order (two-stage, no floating-point atomics).
#include "mpde_internal.hpp"
#include "mpde_kernels.hpp"
#include "mpde_fused.hpp"

namespace mpde {

// 5-point difference weights, [window position][k], window offsets
// k - position; filled by the host from the moment conditions (Eq. 5).
__constant__ double c_W1[5][5];
__constant__ double c_W2[5][5];
__constant__ float c_W1f[5][5];
__constant__ float c_W2f[5][5];

hipError_t upload_stencils(const double w1[5][5], const double w2[5][5]) {
  float f1[5][5], f2[5][5];
  for (int i = 0; i < 5; ++i)
    for (int k = 0; k < 5; ++k) { f1[i][k] = (float)w1[i][k]; f2[i][k] = (float)w2[i][k]; }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_W1), w1, sizeof(double) * 25);
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_W2), w2, sizeof(double) * 25);
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_W1f), f1, sizeof(float) * 25);
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_W2f), f2, sizeof(float) * 25);
  return e;
}

template <typename TA> __device__ __forceinline__ TA W1(int p, int k);
template <typename TA> __device__ __forceinline__ TA W2(int p, int k);
template <> __device__ __forceinline__ float W1<float>(int p, int k) { return c_W1f[p][k]; }
template <> __device__ __forceinline__ float W2<float>(int p, int k) { return c_W2f[p][k]; }
template <> __device__ __forceinline__ double W1<double>(int p, int k) { return c_W1[p][k]; }
template <> __device__ __forceinline__ double W2<double>(int p, int k) { return c_W2[p][k]; }

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ void axis_class(int i, int n, int per, int& tp, int& tm, int& wp) {
  if (per) { tp = 1; tm = 1; wp = 2; return; }
  tp = (i + 1 < n);
  tm = (i >= 1);
  int st = i - 2;
  st = st < 0 ? 0 : st;
  st = st > n - 5 ? n - 5 : st;
  wp = i - st;
}

// Flat index of the point o steps from p along an axis (wrapping if periodic).
__device__ __forceinline__ long long nbr(long long p, int ia, int o, int n, int str, int per) {
  int j = ia + o;
  if (per) { if (j < 0) j += n; else if (j >= n) j -= n; }
  return p + (long long)(j - ia) * str;
}

template <int D>
__device__ __forceinline__ void coords(const LInst& L, int p, int* c) {
  if (D == 2) { c[0] = p / L.n[1]; c[1] = p - c[0] * L.n[1]; }
  else { int q = p / L.n[2]; c[2] = p - q * L.n[2]; c[0] = q / L.n[1]; c[1] = q - c[0] * L.n[1]; }
}

template <typename TC>
__device__ __forceinline__ double coef(const TC* c, const LInst& L, int k, long long p) {
  return k < 0 ? 0.0 : (double)c[L.coff + (long long)k * L.N + p];
}

// Row residuals of axis a at point (p, ia) for field u (weighted), plus the
// class of the point on that axis.  u values at the 5-point window are loaded
// once; the Taylor neighbours are window[wp-1] and window[wp+1].
template <typename TA, typename TV>
struct AxisRows {
  TA rTp, rTm, rC1, rC2;
  int tp, tm, wp;
};

template <typename TA, typename TV>
__device__ __forceinline__ AxisRows<TA, TV> axis_rows(const LInst& L, int a, const TV* u,
                                                      long long p, int ia, TA ui) {
  AxisRows<TA, TV> R;
  const int n = L.n[a], st = L.str[a], per = L.per[a];
  axis_class(ia, n, per, R.tp, R.tm, R.wp);
  TA w[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    int o = k - R.wp;
    w[k] = (o == 0) ? ui : (TA)u[nbr(p, ia, o, n, st, per)];
  }
  TA s1 = 0, s2 = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    s1 += W1<TA>(R.wp, k) * w[k];
    s2 += W2<TA>(R.wp, k) * w[k];
  }
  const TA wT = (TA)L.wT[a];
  TA up = (R.wp < 4) ? w[R.wp + 1] : (TA)0;
  TA um = (R.wp > 0) ? w[R.wp - 1] : (TA)0;
  R.rTp = R.tp ? wT * (ui - up) : (TA)0;
  R.rTm = R.tm ? wT * (ui - um) : (TA)0;
  R.rC1 = -(TA)L.wC1[a] * s1;
  R.rC2 = -(TA)L.wC2[a] * s2;
  return R;
}

// 2x2 inverse of the per-axis Gram block G_a (depends on tp, tm and weights).
template <typename TA>
__device__ __forceinline__ void ginv(const LInst& L, int a, int tp, int tm, TA& i11, TA& i12, TA& i22) {
  const int cls = tm ? (tp ? 0 : 2) : 1;
  i11 = (TA)L.gi[a][cls][0]; i12 = (TA)L.gi[a][cls][1]; i22 = (TA)L.gi[a][cls][2];
}

// Periodic wrap for |o| <= n (no integer division).
__device__ __forceinline__ int wrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// Scaled equation-row coefficients of axis a's derivative unknowns at p.
template <typename TA, typename TC>
__device__ __forceinline__ void chat(const LInst& L, const CIdx& ci, const TC* c, int a, long long p,
                                     TA& ca, TA& caa) {
  const int k1 = ci.k[1 + 2 * a], k2 = ci.k[2 + 2 * a];
  ca = k1 < 0 ? (TA)0 : (TA)c[L.coff + (long long)k1 * L.N + p] * (TA)L.is1[a];
  caa = k2 < 0 ? (TA)0 : (TA)c[L.coff + (long long)k2 * L.N + p] * (TA)L.is2[a];
}

// gamma at point p: the projected equation-row residual (see header).
template <int D, typename TA, typename TV, typename TC>
__device__ __forceinline__ TA gamma_at(const LInst& L, const CIdx& ci, const TV* u, const TC* c,
                                       const TC* f, int sigma, long long p, const int* ic) {
  const TA ui = (TA)u[L.voff + p];
  TA rhoE = (ci.k[0] < 0 ? (TA)0 : (TA)c[L.coff + (long long)ci.k[0] * L.N + p]) * ui;
  if (sigma) rhoE -= (TA)f[L.voff + p];
  TA kappa = 1, num = rhoE;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    AxisRows<TA, TV> R = axis_rows<TA, TV>(L, a, u + L.voff, p, ic[a], ui);
    TA i11, i12, i22;
    ginv<TA>(L, a, R.tp, R.tm, i11, i12, i22);
    const TA wT = (TA)L.wT[a];
    const TA b1 = wT * (R.rTp - R.rTm) + (TA)L.wC1[a] * R.rC1;
    const TA b2 = wT * (R.rTp + R.rTm) * (TA)0.5 + (TA)L.wC2[a] * R.rC2;
    const TA g1 = i11 * b1 + i12 * b2, g2 = i12 * b1 + i22 * b2;
    TA ca, caa;
    chat<TA, TC>(L, ci, c, a, p, ca, caa);
    const TA h1 = i11 * ca + i12 * caa, h2 = i12 * ca + i22 * caa;
    kappa += ca * h1 + caa * h2;
    num -= ca * g1 + caa * g2;
  }
  return num / kappa;
}

// Projected axis-a rows q = rho + A_w,a x* at point (pi, ia) given gamma_i.
template <typename TA, typename TV, typename TC>
__device__ __forceinline__ void q_axis(const LInst& L, const CIdx& ci, const TV* u, const TC* c,
                                       const TV* gam, int a, long long pi, int ia, TA& qTp, TA& qTm,
                                       TA& qC1, TA& qC2, int& tp, int& tm, int& wp) {
  const TA ui = (TA)u[pi];
  AxisRows<TA, TV> R = axis_rows<TA, TV>(L, a, u, pi, ia, ui);
  tp = R.tp; tm = R.tm; wp = R.wp;
  TA i11, i12, i22;
  ginv<TA>(L, a, R.tp, R.tm, i11, i12, i22);
  const TA wT = (TA)L.wT[a];
  const TA b1 = wT * (R.rTp - R.rTm) + (TA)L.wC1[a] * R.rC1;
  const TA b2 = wT * (R.rTp + R.rTm) * (TA)0.5 + (TA)L.wC2[a] * R.rC2;
  TA ca, caa;
  chat<TA, TC>(L, ci, c, a, pi, ca, caa);
  const TA g = (TA)gam[pi];
  const TA x1 = -(i11 * (b1 + ca * g) + i12 * (b2 + caa * g));
  const TA x2 = -(i12 * (b1 + ca * g) + i22 * (b2 + caa * g));
  qTp = R.tp ? R.rTp + wT * (x1 + (TA)0.5 * x2) : (TA)0;
  qTm = R.tm ? R.rTm + wT * (-x1 + (TA)0.5 * x2) : (TA)0;
  qC1 = R.rC1 + (TA)L.wC1[a] * x1;
  qC2 = R.rC2 + (TA)L.wC2[a] * x2;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Fixed-order block sum (256 threads = 4 waves); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double part[kBlock / 64];
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += part[w];
  }
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------- kernels
template <int D, typename TA, typename TV, typename TC>
__global__ void __launch_bounds__(kBlock) k_gamma(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                  CIdx ci, const TV* __restrict__ u, const TC* __restrict__ c,
                                                  const TC* __restrict__ f, int sigma, TV* __restrict__ gam) {
  const Work w = work[blockIdx.x];
  const LInst& L = li[w.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const int p = w.start + threadIdx.x;
  if (p >= L.N) return;
  int ic[kMaxD];
  coords<D>(L, p, ic);
  gam[L.voff + p] = (TV)gamma_at<D, TA, TV, TC>(L, ci, u, c, f, sigma, p, ic);
}

// y_j = (A_u^T Pi (A_u u - sigma d))_j, then the epilogue of `mode`.
template <int D, typename TA, typename TV, typename TC>
__global__ void __launch_bounds__(kBlock) k_gather(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                   CIdx ci, const TV* __restrict__ u, const TV* __restrict__ gam,
                                                   const TC* __restrict__ c, const TC* __restrict__ w,
                                                   int sigma, int mode, TV* __restrict__ out,
                                                   const TV* __restrict__ bvec, TV* __restrict__ xv,
                                                   TV* __restrict__ rv, TV* __restrict__ dv,
                                                   const TV* __restrict__ dinv, int cheb_step,
                                                   double* __restrict__ partial) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const int j = wk.start + threadIdx.x;
  const bool live = j < L.N;
  TA y = 0, uj = 0;
  if (live) {
    int ic[kMaxD];
    coords<D>(L, j, ic);
    const TV* U = u + L.voff;
    const TV* G = gam + L.voff;
    uj = (TA)U[j];
    y = (ci.k[0] < 0 ? (TA)0 : (TA)c[L.coff + (long long)ci.k[0] * L.N + j]) * (TA)G[j];  // equation row (q_E = gamma)
    bool onB = false;
#pragma unroll
    for (int a = 0; a < D; ++a)
      onB |= (L.dlo[a] && ic[a] == 0) || (L.dhi[a] && ic[a] == L.n[a] - 1);
    if (onB) y += uj - (sigma ? (TA)w[L.voff + j] : (TA)0);  // boundary row
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int n = L.n[a], st = L.str[a], per = L.per[a], ia = ic[a];
      const TA wT = (TA)L.wT[a], wC1 = (TA)L.wC1[a], wC2 = (TA)L.wC2[a];
      if ((per && n >= 5) || (ia >= 5 && ia <= n - 6)) {
        // Interior fast path: the five candidate rows i = j-2..j+2 are all
        // centred rows with both Taylor rows (G_a diagonal), and no edge row
        // reaches j; the 9-point line of u around j covers every window.
        TA ul[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) ul[k] = (k == 4) ? uj : (TA)U[nbr(j, ia, k - 4, n, st, per)];
        const TA ig1 = (TA)L.gi[a][0][0], ig2 = (TA)L.gi[a][0][2];
        const int k1 = ci.k[1 + 2 * a], k2 = ci.k[2 + 2 * a];
#pragma unroll
        for (int o = -2; o <= 2; ++o) {
          const long long pi = (o == 0) ? (long long)j : nbr(j, ia, o, n, st, per);
          const TA rTp = wT * (ul[o + 4] - ul[o + 5]);
          const TA rTm = wT * (ul[o + 4] - ul[o + 3]);
          TA s1 = 0, s2 = 0;
#pragma unroll
          for (int m = 0; m < 5; ++m) {
            s1 += W1<TA>(2, m) * ul[o + 2 + m];
            s2 += W2<TA>(2, m) * ul[o + 2 + m];
          }
          const TA rC1 = -wC1 * s1, rC2 = -wC2 * s2;
          const TA ca = k1 < 0 ? (TA)0 : (TA)c[L.coff + (long long)k1 * L.N + pi] * (TA)L.is1[a];
          const TA caa = k2 < 0 ? (TA)0 : (TA)c[L.coff + (long long)k2 * L.N + pi] * (TA)L.is2[a];
          const TA g = (TA)G[pi];
          const TA x1 = -ig1 * (wT * (rTp - rTm) + wC1 * rC1 + ca * g);
          const TA x2 = -ig2 * (wT * (rTp + rTm) * (TA)0.5 + wC2 * rC2 + caa * g);
          const TA qC1 = rC1 + wC1 * x1, qC2 = rC2 + wC2 * x2;
          y -= wC1 * W1<TA>(2, 2 - o) * qC1 + wC2 * W2<TA>(2, 2 - o) * qC2;
          if (o == 0) y += wT * (rTp + wT * (x1 + (TA)0.5 * x2) + rTm + wT * (-x1 + (TA)0.5 * x2));
          else if (o == -1) y -= wT * (rTp + wT * (x1 + (TA)0.5 * x2));
          else if (o == 1) y -= wT * (rTm + wT * (-x1 + (TA)0.5 * x2));
        }
        continue;
      }
      const int R = per ? 2 : 4;
      for (int o = -R; o <= R; ++o) {       // candidate row owner i = j + o e_a
        const int ii = ia + o;
        if (!per && (ii < 0 || ii >= n)) continue;
        const int iw = per ? wrap(ii, n) : ii;
        int tp, tm, wp;
        axis_class(iw, n, per, tp, tm, wp);
        const int k = wp - o;               // position of j in row i's window
        const bool inC = (k >= 0 && k <= 4);
        const bool inT = (o >= -1 && o <= 1);
        if (!inC && !inT) continue;
        const long long pi = nbr(j, ia, o, n, st, per);
        TA qTp, qTm, qC1, qC2;
        q_axis<TA, TV, TC>(L, ci, U, c, G, a, pi, iw, qTp, qTm, qC1, qC2, tp, tm, wp);
        if (inC) y -= wC1 * W1<TA>(wp, k) * qC1 + wC2 * W2<TA>(wp, k) * qC2;
        if (o == 0) y += wT * (qTp + qTm);
        else if (o == -1) y -= wT * qTp;    // T+ of j - e_a ends at j
        else if (o == 1) y -= wT * qTm;     // T- of j + e_a ends at j
      }
    }
  }
  const long long gj = L.voff + j;
  if (mode == G_STORE) {
    if (live) out[gj] = (TV)y;
  } else if (mode == G_RESID) {
    if (live) {
      TA r = (bvec ? (TA)bvec[gj] : (TA)0) - y;
      out[gj] = (TV)r;
      if (dv) dv[gj] = (TV)((TA)dinv[gj] * r / (TA)L.cheb_theta);
    }
  } else if (mode == G_CHEB) {
    if (live) {
      // Chebyshev recurrence on [lo, hi] of D^-1 S: rho_0 = 1/sigma1,
      // rho_k = 1/(2 sigma1 - rho_{k-1}); d_k = rho_k rho_{k-1} d + 2 rho_k/delta D^-1 r.
      const double th = L.cheb_theta, de = L.cheb_delta, s1 = th / de;
      double rp = 1.0 / s1, rn = 0;
      for (int s = 0; s <= cheb_step; ++s) { rn = 1.0 / (2.0 * s1 - rp); if (s < cheb_step) rp = rn; }
      const TA d = uj;
      xv[gj] = (TV)((TA)xv[gj] + d);
      const TA r = (TA)rv[gj] - y;
      rv[gj] = (TV)r;
      dv[gj] = (TV)((TA)(rn * rp) * d + (TA)(2.0 * rn / de) * (TA)dinv[gj] * r);
    }
  } else {  // G_STORE_DOT
    if (live) out[gj] = (TV)y;
    double s = block_sum(live ? (double)uj * (double)y : 0.0);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

// Diagonal of S (inverse stored): sum over the rows touching u_j of a^T Pi a.
template <int D, typename TV, typename TC>
__global__ void __launch_bounds__(kBlock) k_diag(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                 CIdx ci, const TC* __restrict__ c, TV* __restrict__ dinv) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  int ic[kMaxD];
  coords<D>(L, j, ic);
  double diag = 0;
  bool onB = false;
  for (int a = 0; a < D; ++a) onB |= (L.dlo[a] && ic[a] == 0) || (L.dhi[a] && ic[a] == L.n[a] - 1);
  if (onB) diag += 1.0;
  // Per-point quantities of a row owner i: kappa_i, h_b(i) for all axes.
  auto kappa_at = [&](long long pi, const int* ii) {
    double kap = 1;
    for (int b = 0; b < D; ++b) {
      int tp, tm, wp;
      axis_class(ii[b], L.n[b], L.per[b], tp, tm, wp);
      double i11, i12, i22, ca, caa;
      ginv<double>(L, b, tp, tm, i11, i12, i22);
      chat<double, TC>(L, ci, c, b, pi, ca, caa);
      kap += ca * (i11 * ca + i12 * caa) + caa * (i12 * ca + i22 * caa);
    }
    return kap;
  };
  // Self rows (owner i = j): all axes plus the equation row.
  {
    double rhoE = coef(c, L, ci.k[0], j), num = rhoE, kap = 1;
    double ra[kMaxD][4], g1[kMaxD], g2[kMaxD], h1[kMaxD], h2[kMaxD];
    for (int a = 0; a < D; ++a) {
      int tp, tm, wp;
      axis_class(ic[a], L.n[a], L.per[a], tp, tm, wp);
      double wT = L.wT[a];
      ra[a][0] = tp ? wT : 0; ra[a][1] = tm ? wT : 0;
      ra[a][2] = -L.wC1[a] * c_W1[wp][wp]; ra[a][3] = -L.wC2[a] * c_W2[wp][wp];
      double i11, i12, i22, ca, caa;
      ginv<double>(L, a, tp, tm, i11, i12, i22);
      double b1 = wT * (ra[a][0] - ra[a][1]) + L.wC1[a] * ra[a][2];
      double b2 = wT * (ra[a][0] + ra[a][1]) * 0.5 + L.wC2[a] * ra[a][3];
      g1[a] = i11 * b1 + i12 * b2; g2[a] = i12 * b1 + i22 * b2;
      chat<double, TC>(L, ci, c, a, j, ca, caa);
      h1[a] = i11 * ca + i12 * caa; h2[a] = i12 * ca + i22 * caa;
      kap += ca * h1[a] + caa * h2[a];
      num -= ca * g1[a] + caa * g2[a];
    }
    double gam = num / kap;
    diag += rhoE * gam;
    for (int a = 0; a < D; ++a) {
      double wT = L.wT[a];
      double x1 = -(g1[a] + h1[a] * gam), x2 = -(g2[a] + h2[a] * gam);
      double q0 = ra[a][0] != 0 ? ra[a][0] + wT * (x1 + 0.5 * x2) : 0;
      double q1 = ra[a][1] != 0 ? ra[a][1] + wT * (-x1 + 0.5 * x2) : 0;
      double q2 = ra[a][2] + L.wC1[a] * x1, q3 = ra[a][3] + L.wC2[a] * x2;
      diag += ra[a][0] * q0 + ra[a][1] * q1 + ra[a][2] * q2 + ra[a][3] * q3;
    }
  }
  // Rows of other owners along each axis.
  for (int a = 0; a < D; ++a) {
    const int n = L.n[a], per = L.per[a], ia = ic[a];
    const int R = per ? 2 : 4;
    for (int o = -R; o <= R; ++o) {
      if (o == 0) continue;
      const int ii = ia + o;
      if (!per && (ii < 0 || ii >= n)) continue;
      const int iw = per ? wrap(ii, n) : ii;
      if (per && n == 4 && o == -2) continue;      // same owner as o = +2, merged below
      int tp, tm, wp;
      axis_class(iw, n, per, tp, tm, wp);
      double a4[4] = {0, 0, 0, 0};
      int k = wp - o;
      if (k >= 0 && k <= 4) { a4[2] = -L.wC1[a] * c_W1[wp][k]; a4[3] = -L.wC2[a] * c_W2[wp][k]; }
      if (per && n == 4 && o == 2) {               // the o = -2 window entry of the same owner
        int k2 = wp + 2;
        a4[2] += -L.wC1[a] * c_W1[wp][k2]; a4[3] += -L.wC2[a] * c_W2[wp][k2];
      }
      if (o == -1 && tp) a4[0] = -L.wT[a];
      if (o == 1 && tm) a4[1] = -L.wT[a];
      if (a4[0] == 0 && a4[1] == 0 && a4[2] == 0 && a4[3] == 0) continue;
      const long long pi = nbr(j, ia, o, n, L.str[a], per);
      int ii3[kMaxD];
      for (int b = 0; b < D; ++b) ii3[b] = ic[b];
      ii3[a] = iw;
      double kap = kappa_at(pi, ii3);
      double i11, i12, i22, ca, caa;
      ginv<double>(L, a, tp, tm, i11, i12, i22);
      double wT = L.wT[a];
      double b1 = wT * (a4[0] - a4[1]) + L.wC1[a] * a4[2];
      double b2 = wT * (a4[0] + a4[1]) * 0.5 + L.wC2[a] * a4[3];
      double g1 = i11 * b1 + i12 * b2, g2 = i12 * b1 + i22 * b2;
      chat<double, TC>(L, ci, c, a, pi, ca, caa);
      double h1 = i11 * ca + i12 * caa, h2 = i12 * ca + i22 * caa;
      double gam = -(ca * g1 + caa * g2) / kap;
      double x1 = -(g1 + h1 * gam), x2 = -(g2 + h2 * gam);
      double q0 = tp ? a4[0] + wT * (x1 + 0.5 * x2) : 0;
      double q1 = tm ? a4[1] + wT * (-x1 + 0.5 * x2) : 0;
      double q2 = a4[2] + L.wC1[a] * x1, q3 = a4[3] + L.wC2[a] * x2;
      diag += a4[0] * q0 + a4[1] * q1 + a4[2] * q2 + a4[3] * q3;
    }
  }
  dinv[L.voff + j] = (TV)(1.0 / diag);
}

// Chebyshev start from x = 0: x = 0, r = b, d = D^-1 b / theta.
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_cheb_init(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                      const TV* __restrict__ b, const TV* __restrict__ dinv,
                                                      TV* __restrict__ x, TV* __restrict__ r, TV* __restrict__ d) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  const long long g = L.voff + j;
  const TV bb = b[g];
  x[g] = (TV)0;
  r[g] = bb;
  d[g] = (TV)((double)dinv[g] * (double)bb / L.cheb_theta);
}

// Restriction r_c = P^T r_f / 2^(coarsened axes) over coarse points; P is
// linear interpolation along the halved (spatial) axes.
// One-dimensional transfer stencils along one axis.  Restriction (full
// weighting, the transpose of linear interpolation): coarse X gathers fine
// 2X (weight 1) and 2X-1, 2X+1 (weight 1/2; periodic wrap; on a non-periodic
// axis the last fine point, extrapolated as a constant, gives its whole
// weight).  Prolongation: fine i = 2X copies coarse X, i = 2X+1 averages X
// and X+1 (wrap; constant extrapolation past the last coarse point).  An
// axis that is not coarsened is the identity.  Entries with weight 0 carry a
// valid index, so every load stays in bounds.
struct Tap3 {
  int i[3];
  float w[3];
};
__device__ __forceinline__ Tap3 restrict_taps(int X, int nf, int ncn, int per, bool halved) {
  Tap3 t;
  if (!halved) {
    t.i[0] = t.i[1] = t.i[2] = X;
    t.w[0] = 1.f; t.w[1] = t.w[2] = 0.f;
    return t;
  }
  t.i[0] = 2 * X;
  t.w[0] = 1.f;
  if (per) {
    t.i[1] = 2 * X - 1 < 0 ? nf - 1 : 2 * X - 1;
    t.i[2] = 2 * X + 1 >= nf ? 0 : 2 * X + 1;
    t.w[1] = t.w[2] = 0.5f;
  } else {
    t.i[1] = X >= 1 ? 2 * X - 1 : 2 * X;
    t.w[1] = X >= 1 ? 0.5f : 0.f;
    const bool in = 2 * X + 1 < nf;
    t.i[2] = in ? 2 * X + 1 : 2 * X;
    t.w[2] = in ? ((X + 1 < ncn) ? 0.5f : 1.f) : 0.f;
  }
  return t;
}
struct Tap2 {
  int i[2];
  float w[2];
};
__device__ __forceinline__ Tap2 prolong_taps(int i, int ncn, int per, bool halved) {
  Tap2 t;
  if (!halved) { t.i[0] = t.i[1] = i; t.w[0] = 1.f; t.w[1] = 0.f; return t; }
  const int X = i >> 1;
  t.i[0] = X;
  if ((i & 1) == 0) { t.i[1] = X; t.w[0] = 1.f; t.w[1] = 0.f; }
  else if (per) { t.i[1] = X + 1 >= ncn ? 0 : X + 1; t.w[0] = t.w[1] = 0.5f; }
  else if (X + 1 < ncn) { t.i[1] = X + 1; t.w[0] = t.w[1] = 0.5f; }
  else { t.i[1] = X; t.w[0] = 1.f; t.w[1] = 0.f; }
  return t;
}

// Restriction of fine residuals to coarse points: rc = P^T rf / 2^k, k =
// number of halved axes.  Axis 0 (time) is never halved, so the stencil is
// the tensor product of the two (or one) spatial axes.
// With xc != null the coarse level's Chebyshev start (as k_cheb_init) is
// written too, on instances for which the coarse level is smoothed (not
// their coarsest): xc = 0, r = rc, d = D^-1 rc / theta.
template <int D, typename TV>
__global__ void __launch_bounds__(kBlock) k_restrict(const Work* __restrict__ work, const LInst* __restrict__ lf,
                                                     const LInst* __restrict__ lc, const TV* __restrict__ rf,
                                                     TV* __restrict__ rc, const TV* __restrict__ dinv,
                                                     TV* __restrict__ xc, TV* __restrict__ r0, TV* __restrict__ d0) {
  const Work wk = work[blockIdx.x];
  const LInst& C = lc[wk.inst];
  const LInst& F = lf[wk.inst];
  if (gated_off(C)) return;   // converged instance (Krylov iterations only)
  const int jc = wk.start + threadIdx.x;
  if (jc >= C.N) return;
  int cc[kMaxD];
  coords<D>(C, jc, cc);
  const TV* R = rf + F.voff + (long long)cc[0] * F.str[0];
  const Tap3 a1 = restrict_taps(cc[1], F.n[1], C.n[1], F.per[1], C.n[1] != F.n[1]);
  float acc = 0.f;
  if (D == 2) {
#pragma unroll
    for (int u = 0; u < 3; ++u) acc += a1.w[u] * (float)R[a1.i[u]];
  } else {
    const Tap3 a2 = restrict_taps(cc[2], F.n[2], C.n[2], F.per[2], C.n[2] != F.n[2]);
#pragma unroll
    for (int u = 0; u < 3; ++u) {
      const TV* Ru = R + (long long)a1.i[u] * F.str[1];
      float s = 0.f;
#pragma unroll
      for (int v = 0; v < 3; ++v) s += a2.w[v] * (float)Ru[a2.i[v]];
      acc += a1.w[u] * s;
    }
  }
  const TV v = (TV)(acc * (1.f / (float)(1 << C.ncoarsened)));
  const long long g = C.voff + jc;
  rc[g] = v;
  if (xc && !C.coarsest) {
    xc[g] = (TV)0;
    r0[g] = v;
    d0[g] = (TV)((double)dinv[g] * (double)v / C.cheb_theta);
  }
}

// Prolongation and correction x_f += P e_c over fine points.
template <int D, typename TV>
__global__ void __launch_bounds__(kBlock) k_prolong_add(const Work* __restrict__ work, const LInst* __restrict__ lf,
                                                        const LInst* __restrict__ lc, const TV* __restrict__ ec,
                                                        TV* __restrict__ xf) {
  const Work wk = work[blockIdx.x];
  const LInst& F = lf[wk.inst];
  const LInst& C = lc[wk.inst];
  if (gated_off(C)) return;   // converged instance (Krylov iterations only)
  const int jf = wk.start + threadIdx.x;
  if (jf >= F.N) return;
  int fc[kMaxD];
  coords<D>(F, jf, fc);
  const TV* E = ec + C.voff + (long long)fc[0] * C.str[0];
  const Tap2 a1 = prolong_taps(fc[1], C.n[1], F.per[1], C.n[1] != F.n[1]);
  float acc = 0.f;
  if (D == 2) {
    acc = a1.w[0] * (float)E[a1.i[0]] + a1.w[1] * (float)E[a1.i[1]];
  } else {
    const Tap2 a2 = prolong_taps(fc[2], C.n[2], F.per[2], C.n[2] != F.n[2]);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const TV* Eu = E + (long long)a1.i[u] * C.str[1];
      acc += a1.w[u] * (a2.w[0] * (float)Eu[a2.i[0]] + a2.w[1] * (float)Eu[a2.i[1]]);
    }
  }
  const long long g = F.voff + jf;
  xf[g] = (TV)((float)xf[g] + acc);
}

// Coefficient coarsening: normalised full weighting along halved axes.
template <int D, typename TC>
__global__ void __launch_bounds__(kBlock) k_coarsen_coef(const Work* __restrict__ work, const LInst* __restrict__ lf,
                                                         const LInst* __restrict__ lc, int K,
                                                         const TC* __restrict__ cf, TC* __restrict__ cc) {
  const Work wk = work[blockIdx.x];
  const LInst& C = lc[wk.inst];
  const LInst& F = lf[wk.inst];
  const int jc = wk.start + threadIdx.x;
  if (jc >= C.N) return;
  int cq[kMaxD];
  coords<D>(C, jc, cq);
  int fi[kMaxD][3];
  double fw[kMaxD][3];
  int cnt[kMaxD];
  for (int a = 0; a < D; ++a) {
    if (C.n[a] == F.n[a]) { cnt[a] = 1; fi[a][0] = cq[a]; fw[a][0] = 1; continue; }
    const int nf = F.n[a], X = cq[a];
    int m = 0;
    double tw = 0;
    fi[a][m] = 2 * X; fw[a][m++] = 0.5;
    if (F.per[a] || 2 * X - 1 >= 0) { fi[a][m] = (2 * X - 1 + nf) % nf; fw[a][m++] = 0.25; }
    if (F.per[a] || 2 * X + 1 < nf) { fi[a][m] = (2 * X + 1) % nf; fw[a][m++] = 0.25; }
    for (int q = 0; q < m; ++q) tw += fw[a][q];
    for (int q = 0; q < m; ++q) fw[a][q] /= tw;
    cnt[a] = m;
  }
  const int tot = cnt[0] * cnt[1] * (D == 3 ? cnt[2] : 1);
  for (int k = 0; k < K; ++k) {
    double acc = 0;
    for (int t = 0; t < tot; ++t) {
      int rem = t, idx[kMaxD];
      for (int a = D - 1; a >= 0; --a) { idx[a] = rem % cnt[a]; rem /= cnt[a]; }
      long long off = 0;
      double wgt = 1;
      for (int a = 0; a < D; ++a) { off += (long long)fi[a][idx[a]] * F.str[a]; wgt *= fw[a][idx[a]]; }
      acc += wgt * (double)cf[F.coff + (long long)k * F.N + off];
    }
    cc[C.coff + (long long)k * C.N + jc] = (TC)acc;
  }
}

// Unit columns for probing the coarsest operator: probe instance q holds the
// unit vector of its own column, U[voff(q) + col(q)] = 1 (U zero-filled).
__global__ void __launch_bounds__(kBlock) k_set_unit(const LInst* __restrict__ probe, const int* __restrict__ col,
                                                     int nprobe, double* __restrict__ U) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nprobe) U[probe[q].voff + col[q]] = 1.0;
}

// Time-coloured probe vectors for the coarsest operator, whose couplings
// reach at most 4 time steps: probe (c, s) has ones at the points (t, s) with
// t = c (mod 9), so every operator column is recovered from one probe.
__global__ void __launch_bounds__(kBlock) k_set_probe(const LInst* __restrict__ probe, const int* __restrict__ pc,
                                                      const int* __restrict__ ps, int nprobe, int ncolor,
                                                      double* __restrict__ U) {
  const int q = blockIdx.x;
  const LInst& L = probe[q];
  const int m = L.N / L.n[0];
  for (int t = pc[q] + (int)threadIdx.x * ncolor; t < L.n[0]; t += (int)blockDim.x * ncolor)
    U[L.voff + (long long)t * m + ps[q]] = 1.0;
}

// Scatter probe responses into the dense column-major matrix:
// S[i][j] = Y_(c(j), s(j))[i] for |t(i) - t(j)| <= 4.
__global__ void __launch_bounds__(kBlock) k_extract_probe(const Work* __restrict__ work, const LInst* __restrict__ probe,
                                                          const int* __restrict__ pc, const int* __restrict__ ps,
                                                          const long long* __restrict__ dout, int ncolor,
                                                          const double* __restrict__ Y, double* __restrict__ S) {
  const Work wk = work[blockIdx.x];
  const LInst& L = probe[wk.inst];
  const int i = wk.start + threadIdx.x;
  if (i >= L.N) return;
  const int m = L.N / L.n[0];
  const int tr = i / m;
  const int c = pc[wk.inst], sc = ps[wk.inst];
  // the column time t = c (mod ncolor) within [tr - 4, tr + 4]; with a time
  // axis no longer than the colour count each probe is a single time step
  int t;
  if (L.n[0] <= ncolor) {
    t = c;
  } else {
    const int lo = tr - 4;
    t = lo + ((c - lo) % ncolor + ncolor) % ncolor;
    if (t > tr + 4 || t >= L.n[0] || t < 0) return;
  }
  const long long j = (long long)t * m + sc;
  S[dout[wk.inst] + j * L.N + i] = Y[L.voff + i];
}

// ------------------------------------------------ block-banded coarsest solve
// The coarsest operator, in time-major order, is block banded: blocks are
// spatial planes of m <= 64 points and only blocks with |t - t'| <= 4 are
// nonzero.  Lower blocks are stored per instance as Lb[t][k] = block
// (t, t - k), k = 0..4, row-major m x m.  The factor keeps the off-diagonal
// blocks of L and the inverses of its diagonal blocks.
constexpr int kBBMax = 64;

__device__ __forceinline__ long long bb_at(long long base, int t, int k, int m) {
  return base + ((long long)t * 5 + k) * m * m;
}

// Probe instances of the coarsest-level probing, generated on the device.
// Source k (a probed instance) owns probes pstart .. pstart + nc * plane - 1
// in (colour c, plane point sp) order, c-major; each probe is a copy of the
// instance's level descriptor whose vector offset points at its probe
// vector (yoff + (c * plane + sp) * n).  Work items: ceil(n / kBlock) per
// probe from wstart; fused-operator tiles: tpp per probe from tstart, with
// origins torg[toff ..].  Sources are ordered, so the owner of an index is
// found by binary search on the prefix starts.
template <typename F>
__device__ __forceinline__ int probe_owner(const ProbeSrc* src, int nsrc, long long i, F start) {
  int lo = 0, hi = nsrc - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start(src[mid]) <= i) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}
__global__ void __launch_bounds__(kBlock) k_probe_lists(const LInst* __restrict__ lc, const ProbeSrc* __restrict__ src,
                                                        int nsrc, long long nvq, long long nwk, long long ntile,
                                                        const int2* __restrict__ torg, LInst* __restrict__ vq,
                                                        int* __restrict__ pc, int* __restrict__ ps,
                                                        long long* __restrict__ bo, Work* __restrict__ wk,
                                                        FTile* __restrict__ tiles) {
  const long long i = (long long)blockIdx.x * kBlock + threadIdx.x;
  if (i < nvq) {
    const ProbeSrc& S = src[probe_owner(src, nsrc, i, [](const ProbeSrc& x) { return x.pstart; })];
    const long long loc = i - S.pstart;
    const int c = (int)(loc / S.plane), sp = (int)(loc - (long long)c * S.plane);
    LInst q = lc[S.b];
    q.voff = S.yoff + ((long long)c * S.plane + sp) * S.n;
    vq[i] = q;
    pc[i] = c;
    ps[i] = sp;
    bo[i] = S.boff;
  }
  if (i < nwk) {
    const ProbeSrc& S = src[probe_owner(src, nsrc, i, [](const ProbeSrc& x) { return x.wstart; })];
    const long long loc = i - S.wstart;
    const long long wpp = (S.n + kBlock - 1) / kBlock;
    wk[i] = Work{(int)(S.pstart + loc / wpp), (int)(loc % wpp) * kBlock};
  }
  if (tiles && i < ntile) {
    const ProbeSrc& S = src[probe_owner(src, nsrc, i, [](const ProbeSrc& x) { return x.tstart; })];
    const long long loc = i - S.tstart;
    const int2 o = torg[S.toff + (int)(loc % S.tpp)];
    tiles[i] = FTile{(int)(S.pstart + loc / S.tpp), o.x, o.y, (int)i};
  }
}

void launch_probe_lists(hipStream_t st, const LInst* lc, const ProbeSrc* src, int nsrc, long long nvq, long long nwk,
                        long long ntile, const int2* torg, LInst* vq, int* pc, int* ps, long long* bo, Work* wk,
                        FTile* tiles) {
  const long long n = std::max(nvq, std::max(nwk, tiles ? ntile : 0LL));
  if (n <= 0) return;
  hipLaunchKernelGGL(k_probe_lists, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, lc, src, nsrc,
                     nvq, nwk, ntile, torg, vq, pc, ps, bo, wk, tiles);
}

// Probe responses into the lower band blocks.
__global__ void __launch_bounds__(kBlock) k_extract_band(const Work* __restrict__ work, const LInst* __restrict__ probe,
                                                         const int* __restrict__ pc, const int* __restrict__ ps,
                                                         const long long* __restrict__ bout, int ncolor,
                                                         const double* __restrict__ Y, double* __restrict__ Lb) {
  const Work wk = work[blockIdx.x];
  const LInst& L = probe[wk.inst];
  const int i = wk.start + threadIdx.x;
  if (i >= L.N) return;
  const int m = L.N / L.n[0];
  const int tr = i / m, sr = i - tr * m;
  const int c = pc[wk.inst], sc = ps[wk.inst];
  int t;
  if (L.n[0] <= ncolor) {
    t = c;
  } else {
    const int lo = tr - 4;
    t = lo + ((c - lo) % ncolor + ncolor) % ncolor;
    if (t > tr + 4 || t >= L.n[0] || t < 0) return;
  }
  const int k = tr - t;
  if (k < 0 || k > 4) return;
  Lb[bb_at(bout[wk.inst], tr, k, m) + (long long)sr * m + sc] = Y[L.voff + i];
}

// Block Cholesky, one block of threads per instance, FP64.  The block
// products (the off-diagonal blocks L_ij = B_ij L_jj^-T and the trailing
// updates B_ik -= L_ij L_kj^T) run as 64 x 64 x 64 products C = A B^T with
// both operands staged transposed in LDS and a 4 x 4 register tile per
// thread (256 threads cover the 64 x 64 result); blocks of a smaller plane
// are zero-padded to 64.  The block has two such groups of 256 threads,
// which take two products of a plane at a time (they share the B operand:
// L_jj^-T for the off-diagonal blocks, L_kj for the updates of column k).
constexpr int kBBT = kBBMax + 4;   // staged operand stride (keeps 4-double groups 16-byte aligned)
constexpr int kBBGroups = 2;
constexpr int kBBThreads = kBBGroups * kBlock;

// Stage the m x m row-major block G into T transposed and zero-padded,
// T[q][r] = G[r][q], by the threads lt = 0 .. nth - 1 of the caller.
__device__ __forceinline__ void bb_stage_t(double* __restrict__ T, const double* G, int m, int gstride, int lt,
                                           int nth) {
  for (int e = lt; e < kBBMax * kBBMax; e += nth) {
    const int r = e >> 6, q = e & 63;
    T[q * kBBT + r] = (r < m && q < m) ? G[r * gstride + q] : 0.0;
  }
}

// acc[a][b] = sum_q At[q][4tr + a] * Bt[q][4tc + b] for the tile of the
// group's thread lt < 256.
__device__ __forceinline__ void bb_tile_abt(const double* __restrict__ At, const double* __restrict__ Bt,
                                            double (&acc)[4][4], int lt) {
  const int tr = lt >> 4, tc = lt & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 4
  for (int q = 0; q < kBBMax; ++q) {
    const double2 a01 = *reinterpret_cast<const double2*>(At + q * kBBT + 4 * tr);
    const double2 a23 = *reinterpret_cast<const double2*>(At + q * kBBT + 4 * tr + 2);
    const double2 b01 = *reinterpret_cast<const double2*>(Bt + q * kBBT + 4 * tc);
    const double2 b23 = *reinterpret_cast<const double2*>(Bt + q * kBBT + 4 * tc + 2);
    const double av[4] = {a01.x, a01.y, a23.x, a23.y}, bv[4] = {b01.x, b01.y, b23.x, b23.y};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
  }
}

__global__ void __launch_bounds__(kBBThreads) k_bb_factor(double* __restrict__ Lb, const long long* __restrict__ boff,
                                                      const int* __restrict__ Tn, const int* __restrict__ mn,
                                                      int* __restrict__ fail) {
  const long long base = boff[blockIdx.x];
  const int T = Tn[blockIdx.x], m = mn[blockIdx.x];
  __shared__ double Ls[kBBMax][kBBMax + 1];            // Ls[k][r] = L[r][k], the factor's columns
  __shared__ double col[2][kBBMax], xr[2][kBBMax];     // broadcast pivot column / inverse row
  __shared__ __align__(16) double S1[kBBGroups][kBBMax * kBBT];   // staged A^T, one per group
  __shared__ __align__(16) double S2[kBBMax * kBBT];              // staged B^T, shared
  const int tid = threadIdx.x;
  const int grp = tid / kBlock, lt = tid % kBlock;   // product group and thread within it
  const int tr = lt >> 4, tc = lt & 15;
  const bool g0 = grp == 0;                          // the diagonal factor runs on group 0
  // diagonal-block factor and inverse: thread (r, cb) keeps columns
  // c = cb + 4 i (i < 16) of row r in registers; a plane of m < 64 points
  // is padded with an identity block
  // (group 1 mirrors group 0's indices so that its reads stay in range;
  // every write of the diagonal factor is group 0's)
  const int r = lt >> 2, cb = lt & 3;
  for (int j = 0; j < T; ++j) {
    double* Bjj = Lb + bb_at(base, j, 0, m);
    double a[16], x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int c = cb + 4 * i;
      a[i] = (g0 && r < m && c < m) ? Bjj[r * m + c] : (r == c ? 1.0 : 0.0);
      x[i] = (r == c) ? 1.0 : 0.0;
    }
    // right-looking Cholesky, one barrier per pivot: the owners of column k
    // publish its current values, then every row r > k applies
    // a[r][c] -= a[r][k] a[c][k] / a[k][k] (k < c <= r) and column k is
    // scaled into Ls
#pragma unroll
    for (int k = 0; k < kBBMax; ++k) {
      double* ck = col[k & 1];
      if (g0 && cb == (k & 3)) ck[r] = a[k >> 2];
      __syncthreads();
      double akk = ck[k];
      if (!(akk > 0)) {
        if (tid == 0) fail[blockIdx.x] = 1;
        akk = 1.0;
      }
      const double piv = sqrt(akk), rinv = 1.0 / akk;
      const double ark = ck[r];
      if (g0 && cb == (k & 3)) Ls[k][r] = r >= k ? (r == k ? piv : ark / piv) : 0.0;
      if (g0 && r > k) {
        const double f = ark * rinv;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int c = cb + 4 * i;
          if (4 * i + 3 > k && c > k && c <= r) a[i] = fma(-f, ck[c], a[i]);
        }
      }
    }
    // inverse X = L^-1 (lower), right-looking: row k of X is final once
    // divided by L[k][k]; rows r > k then subtract L[r][k] X[k][:]
#pragma unroll
    for (int k = 0; k < kBBMax; ++k) {
      double* xk = xr[k & 1];
      const double dk = 1.0 / Ls[k][k];
      if (g0 && r == k) {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          x[i] *= dk;
          xk[cb + 4 * i] = x[i];
        }
      }
      __syncthreads();
      if (g0 && r > k) {
        const double lrk = Ls[k][r];
#pragma unroll
        for (int i = 0; i < 16; ++i)
          if (4 * i <= k + 3 && cb + 4 * i <= k) x[i] = fma(-lrk, xk[cb + 4 * i], x[i]);
      }
    }
    // Linv row-major into the diagonal block (k_bb_solve* read the inverse
    // there), and transposed into S2 (S2[c][r] = Linv[r][c]), the staged B^T
    // of the products B_ij Linv^T below
    if (g0) {
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int c = cb + 4 * i;
        if (r < m && c < m) Bjj[r * m + c] = x[i];
        S2[c * kBBT + r] = x[i];
      }
    }
    // B^T operand of L_ij = B_ij Linv^T is Linv^T[q][c] = Linv[c][q] = S2[q][c]: in place.
    __syncthreads();
    const int ie = min(T - 1, j + 4);
    // off-diagonal blocks, two at a time (group g takes block i0 + g)
    for (int i0 = j + 1; i0 <= ie; i0 += kBBGroups) {
      const int i = i0 + grp;
      double* Bij = Lb + bb_at(base, min(i, ie), min(i, ie) - j, m);
      if (i <= ie) bb_stage_t(S1[grp], Bij, m, m, lt, kBlock);
      __syncthreads();
      if (i <= ie) {
        double acc[4][4];
        bb_tile_abt(S1[grp], S2, acc, lt);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            const int r = 4 * tr + a, cc = 4 * tc + b;
            if (r < m && cc < m) Bij[r * m + cc] = acc[a][b];
          }
      }
      __syncthreads();
    }
    // trailing update: B_ik -= L_ij L_kj^T for j < k <= i <= j + 4, the
    // blocks i of one column k two at a time
    for (int k = j + 1; k <= ie; ++k) {
      const double* Lkj = Lb + bb_at(base, k, k - j, m);
      bb_stage_t(S2, Lkj, m, m, tid, kBBThreads);
      for (int i0 = k; i0 <= ie; i0 += kBBGroups) {
        const int i = i0 + grp;
        const double* Lij = Lb + bb_at(base, min(i, ie), min(i, ie) - j, m);
        if (i <= ie) bb_stage_t(S1[grp], Lij, m, m, lt, kBlock);
        __syncthreads();
        if (i <= ie) {
          double acc[4][4];
          bb_tile_abt(S1[grp], S2, acc, lt);
          double* Bik = Lb + bb_at(base, i, i - k, m);
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
              const int r = 4 * tr + a, cc = 4 * tc + b;
              if (r < m && cc < m) Bik[r * m + cc] -= acc[a][b];
            }
        }
        __syncthreads();
      }
    }
  }
}

// x = S^-1 b on the coarsest level by block forward / backward substitution;
// one block of threads per instance (its rows in the work table).
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_bb_solve(const int* __restrict__ inst_list, const LInst* __restrict__ li,
                                                     const TV* __restrict__ Lb, const TV* __restrict__ bvec,
                                                     TV* __restrict__ xvec) {
  const LInst& L = li[inst_list[blockIdx.x]];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const int T = L.n[0], m = L.N / T;
  const long long base = L.doff;
  __shared__ double ys[kBBMax * kBBMax];  // y then x (T * m <= 4096)
  __shared__ double acc[kBBMax];
  __shared__ double part[kBlock];
  const int tid = threadIdx.x;
  const int lanes = kBlock / m;             // threads per row (m <= 64, so >= 4)
  const int r = tid / lanes, sub = tid % lanes;
  const TV* B = bvec + L.voff;
  TV* X = xvec + L.voff;
  // forward: y_t = Dinv_t (b_t - sum_k L[t][k] y_{t-k})
  for (int t = 0; t < T; ++t) {
    double s = 0;
    if (r < m) {
      if (sub == 0) s = (double)B[(long long)t * m + r];
      for (int k = 1; k <= 4 && k <= t; ++k) {
        const TV* Lk = Lb + bb_at(base, t, k, m) + (long long)r * m;
        const double* yk = ys + (t - k) * m;
        for (int cc = sub; cc < m; cc += lanes) s -= (double)Lk[cc] * (double)yk[cc];
      }
    }
    part[tid] = s;
    __syncthreads();
    if (r < m && sub == 0) {
      double a = 0;
      for (int q = 0; q < lanes; ++q) a += part[r * lanes + q];
      acc[r] = a;
    }
    __syncthreads();
    if (r < m) {
      const TV* Di = Lb + bb_at(base, t, 0, m) + (long long)r * m;
      double v = 0;
      for (int cc = sub; cc <= r; cc += lanes) v += (double)Di[cc] * acc[cc];
      part[tid] = v;
    } else {
      part[tid] = 0;
    }
    __syncthreads();
    if (r < m && sub == 0) {
      double a = 0;
      for (int q = 0; q < lanes; ++q) a += part[r * lanes + q];
      ys[t * m + r] = a;
    }
    __syncthreads();
  }
  // backward: x_t = Dinv_t^T (y_t - sum_k L[t+k][k]^T x_{t+k})
  for (int t = T - 1; t >= 0; --t) {
    double s = 0;
    if (r < m) {
      if (sub == 0) s = (double)ys[t * m + r];
      for (int k = 1; k <= 4 && t + k < T; ++k) {
        const TV* Lk = Lb + bb_at(base, t + k, k, m);
        const double* xk = ys + (t + k) * m;
        for (int q = sub; q < m; q += lanes) s -= (double)Lk[(long long)q * m + r] * (double)xk[q];
      }
    }
    part[tid] = s;
    __syncthreads();
    if (r < m && sub == 0) {
      double a = 0;
      for (int q = 0; q < lanes; ++q) a += part[r * lanes + q];
      acc[r] = a;
    }
    __syncthreads();
    if (r < m) {
      const TV* Di = Lb + bb_at(base, t, 0, m);
      double v = 0;
      for (int q = r + sub; q < m; q += lanes) v += (double)Di[(long long)q * m + r] * acc[q];
      part[tid] = v;
    } else {
      part[tid] = 0;
    }
    __syncthreads();
    if (r < m && sub == 0) {
      double a = 0;
      for (int q = 0; q < lanes; ++q) a += part[r * lanes + q];
      ys[t * m + r] = a;
      X[(long long)t * m + r] = (TV)a;
    }
    __syncthreads();
  }
}

// In-place Gauss-Jordan inverse of one SPD matrix per block (FP64, no
// pivoting: the coarsest operator is symmetric positive definite).
__global__ void __launch_bounds__(1024) k_gauss_jordan(double* __restrict__ A, const long long* __restrict__ off,
                                                       const int* __restrict__ nn, int* __restrict__ fail) {
  double* M = A + off[blockIdx.x];
  const int n = nn[blockIdx.x];
  __shared__ double prow[2048];
  __shared__ double pcol[2048];
  __shared__ double piv;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      piv = M[(long long)k * n + k];
      if (!(piv > 0)) fail[blockIdx.x] = 1;
    }
    __syncthreads();
    const double ip = 1.0 / piv;
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
      prow[c] = M[(long long)k * n + c] * ip;
      pcol[c] = M[(long long)c * n + k];
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) prow[c] = (c == k) ? ip : prow[c];
    __syncthreads();
    for (long long e = threadIdx.x; e < (long long)n * n; e += blockDim.x) {
      const int r = (int)(e / n), c = (int)(e - (long long)r * n);
      if (r == k) M[e] = prow[c];
      else {
        const double f = pcol[r];
        M[e] = (c == k ? 0.0 : M[e]) - f * prow[c];
      }
    }
    __syncthreads();
  }
}

// Banded Cholesky in place (FP64), one block per matrix.  A is column-major
// N x N, symmetric positive definite, with A[i][j] = 0 for |i - j| > band
// (the coarsest operator couples points at most 4 time steps apart, so in
// time-major order the half-band is 5 * plane - 1).  The lower factor L
// overwrites the lower band of A.
__global__ void __launch_bounds__(kBlock) k_band_chol(double* __restrict__ A, const long long* __restrict__ off,
                                                      const int* __restrict__ nn, const int* __restrict__ bw,
                                                      int* __restrict__ fail) {
  double* M = A + off[blockIdx.x];
  const int n = nn[blockIdx.x], b = bw[blockIdx.x];
  __shared__ double dk;
  for (int k = 0; k < n; ++k) {
    if (threadIdx.x == 0) {
      const double a = M[(long long)k * n + k];
      if (!(a > 0)) fail[blockIdx.x] = 1;
      dk = a > 0 ? sqrt(a) : 1.0;
      M[(long long)k * n + k] = dk;
    }
    __syncthreads();
    const int hi = min(n - 1, k + b);
    const double inv = 1.0 / dk;
    for (int i = k + 1 + threadIdx.x; i <= hi; i += blockDim.x) M[(long long)k * n + i] *= inv;
    __syncthreads();
    // trailing update of the band: A[i][j] -= L[i][k] L[j][k], k < j <= i <= hi
    const int m = hi - k;
    for (int e = threadIdx.x; e < m * m; e += blockDim.x) {
      const int ii = e / m, jj = e - ii * m;
      if (jj > ii) continue;
      const int i = k + 1 + ii, j = k + 1 + jj;
      M[(long long)j * n + i] -= M[(long long)k * n + i] * M[(long long)k * n + j];
    }
    __syncthreads();
  }
}

// Dense inverse from a banded Cholesky factor: thread c solves L L^T x = e_c
// and writes x as row c of X (X symmetric, so this is also column c); rows
// are interleaved so that consecutive threads write consecutive addresses.
__global__ void __launch_bounds__(kBlock) k_band_inverse(const double* __restrict__ Lf, double* __restrict__ X,
                                                         const long long* __restrict__ off,
                                                         const int* __restrict__ nn, const int* __restrict__ bw,
                                                         const int* __restrict__ mat_of_block,
                                                         const int* __restrict__ col0_of_block) {
  const int mtx = mat_of_block[blockIdx.x];
  const int n = nn[mtx], b = bw[mtx];
  const int c = col0_of_block[blockIdx.x] + threadIdx.x;
  if (c >= n) return;
  const double* L = Lf + off[mtx];
  double* Y = X + off[mtx];                 // Y[i * n + c] holds y_i then x_i
  for (int i = 0; i < n; ++i) {             // forward: L y = e_c
    double acc = (i == c) ? 1.0 : 0.0;
    const int j0 = max(0, i - b);
    if (i >= c)
      for (int j = max(j0, c); j < i; ++j) acc -= L[(long long)j * n + i] * Y[(long long)j * n + c];
    Y[(long long)i * n + c] = (i >= c) ? acc / L[(long long)i * n + i] : 0.0;
  }
  for (int i = n - 1; i >= 0; --i) {        // backward: L^T x = y
    double acc = Y[(long long)i * n + c];
    const int j1 = min(n - 1, i + b);
    for (int j = i + 1; j <= j1; ++j) acc -= L[(long long)i * n + j] * Y[(long long)j * n + c];
    Y[(long long)i * n + c] = acc / L[(long long)i * n + i];
  }
}

template <typename TV>
__global__ void __launch_bounds__(kBlock) k_convert_dense(const double* __restrict__ src, TV* __restrict__ dst, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (TV)src[i];
}

// e = Sinv r for coarsest instances: one thread per row; Sinv symmetric, so
// row r is read as column r (coalesced across threads).
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_dense_apply(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                        const TV* __restrict__ Sinv, const TV* __restrict__ r,
                                                        TV* __restrict__ e) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int row = wk.start + threadIdx.x;
  const int n = L.N;
  const TV* M = Sinv + L.doff;
  const TV* rr = r + L.voff;
  __shared__ TV rs[kBlock];
  double acc = 0;
  for (int c0 = 0; c0 < n; c0 += kBlock) {
    __syncthreads();
    if (c0 + (int)threadIdx.x < n) rs[threadIdx.x] = rr[c0 + threadIdx.x];
    __syncthreads();
    const int cmax = (n - c0) < kBlock ? (n - c0) : kBlock;
    if (row < n)
      for (int cc = 0; cc < cmax; ++cc) acc += (double)M[(long long)(c0 + cc) * n + row] * (double)rs[cc];
  }
  if (row < n) e[L.voff + row] = (TV)acc;
}

// ---------------------------------------------------------------- Krylov
// Per-work-item partial sums of a.b: one wavefront per work item of kBlock
// points, each lane summing kBlock / 64 points in a fixed order, then a
// fixed cross-lane tree (no LDS, no barrier).
constexpr int kDotLanes = 64;
template <typename TA, typename TV>
__global__ void __launch_bounds__(kDotLanes) k_dot(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                   const TV* __restrict__ a, const TV* __restrict__ b,
                                                   double* __restrict__ partial) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  double v = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kDotLanes; ++i) {
    const int j = wk.start + threadIdx.x + kDotLanes * i;
    if (j < L.N) v = fma((double)a[L.voff + j], (double)b[L.voff + j], v);
  }
#pragma unroll
  for (int off = kDotLanes / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kDotLanes);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// Per-instance fixed-order sum of block partials: out[b] = sum partial[bs[b]..bs[b+1]);
// one block per instance, strided per-thread sums then a fixed tree.
__global__ void __launch_bounds__(kBlock) k_finish_sum(const double* __restrict__ partial,
                                                       const int* __restrict__ bstart, int B,
                                                       double* __restrict__ out) {
  const int b = blockIdx.x;
  double s = 0;
  for (int i = bstart[b] + threadIdx.x; i < bstart[b + 1]; i += kBlock) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[b] = s;
}

// Scalar updates of PCG, one thread per instance.
//   op 0: beta = active ? (first ? 0 : rz_new/rz) : 0; rz = rz_new
//   op 1: alpha = active ? rz/pq : 0
//   op 2: convergence test of rnorm2 against tol2[b]*r0norm2; counts iterations
__global__ void k_pcg_scalars(int op, int B, int first, const double* __restrict__ tol2, double* __restrict__ rz_new,
                              double* __restrict__ rz, double* __restrict__ beta, double* __restrict__ pq,
                              double* __restrict__ alpha, double* __restrict__ rn2, double* __restrict__ r0n2,
                              int* __restrict__ active, int* __restrict__ iters) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  if (op == 0) {
    const double v = rz_new[b];
    beta[b] = (active[b] && !first && rz[b] != 0.0) ? v / rz[b] : 0.0;
    rz[b] = v;
  } else if (op == 1) {
    const double d = pq[b];
    alpha[b] = (active[b] && d > 0.0 && isfinite(d)) ? rz[b] / d : 0.0;
  } else if (op == 3) {
    // flexible (Polak-Ribiere) beta; pq carries r.z_prev
    const double v = rz_new[b];
    beta[b] = (active[b] && !first && rz[b] != 0.0) ? (v - pq[b]) / rz[b] : 0.0;
    rz[b] = v;
  } else {
    if (active[b]) {
      iters[b] += 1;
      const double r = rn2[b];
      if (!(r > tol2[b] * r0n2[b])) active[b] = 0;   // converged or non-finite
    }
  }
}

// k_finish_sum into out (one of rz_new, pq, rn2), then the scalar update
// of k_pcg_scalars op 0, 1 or 2 of the same instance from that sum, by the
// thread that holds it (one launch instead of two).  The sum is handed to
// the update as a value: out is not read back.
__global__ void __launch_bounds__(kBlock) k_finish_scalars(const double* __restrict__ partial,
                                                           const int* __restrict__ bstart, double* __restrict__ out,
                                                           int op, int first, const double* __restrict__ tol2,
                                                           double* __restrict__ rz, double* __restrict__ beta,
                                                           double* __restrict__ alpha,
                                                           const double* __restrict__ r0n2, int* __restrict__ active,
                                                           int* __restrict__ iters) {
  const int b = blockIdx.x;
  double s = 0;
  for (int i = bstart[b] + threadIdx.x; i < bstart[b + 1]; i += kBlock) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x != 0) return;
  out[b] = s;
  if (op == 0) {   // s = r.z
    beta[b] = (active[b] && !first && rz[b] != 0.0) ? s / rz[b] : 0.0;
    rz[b] = s;
  } else if (op == 1) {   // s = p.q
    alpha[b] = (active[b] && s > 0.0 && isfinite(s)) ? rz[b] / s : 0.0;
  } else if (active[b]) {   // s = ||r||^2
    iters[b] += 1;
    if (!(s > tol2[b] * r0n2[b])) active[b] = 0;   // converged or non-finite
  }
}

// p = z + beta p
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_update_p(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                     const double* __restrict__ beta, const TV* __restrict__ z,
                                                     TV* __restrict__ p) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  const long long g = L.voff + j;
  const double bt = beta[wk.inst];
  p[g] = (TV)((double)z[g] + bt * (double)p[g]);
}

// p = z + beta p and q = S p without an operator pass: S z = r - rv, where
// rv = r - S z is the preconditioner's own final residual (the V-cycle's
// smoother keeps it), so q = (r - rv) + beta q; partial p.q
template <typename TV>
// (one wavefront per work item, like k_dot: kBlock / 64 points per lane and
// a cross-lane tree for the partial sum)
__global__ void __launch_bounds__(kDotLanes) k_update_pq(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                         const double* __restrict__ beta, const TV* __restrict__ z,
                                                         const TV* __restrict__ r, const TV* __restrict__ rv,
                                                         TV* __restrict__ p, TV* __restrict__ q,
                                                         double* __restrict__ partial) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const double bt = beta[wk.inst];
  double v = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kDotLanes; ++i) {
    const int j = wk.start + threadIdx.x + kDotLanes * i;
    if (j < L.N) {
      const long long g = L.voff + j;
      // (beta = 0 starts the recurrences: the old p and q are not read)
      const double po = bt != 0.0 ? (double)p[g] : 0.0, qo = bt != 0.0 ? (double)q[g] : 0.0;
      const TV pn = (TV)((double)z[g] + bt * po);
      const TV qn = (TV)(((double)r[g] - (double)rv[g]) + bt * qo);
      p[g] = pn;
      q[g] = qn;
      v = fma((double)pn, (double)qn, v);
    }
  }
#pragma unroll
  for (int off = kDotLanes / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kDotLanes);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// x += alpha p; r -= alpha q; partial ||r||^2.  With z0 != null also the
// Chebyshev start of the next preconditioner application on this level
// (as k_cheb_init with b = the new r), on instances for which the level is
// smoothed: z0 = 0, r0 = r, d0 = D^-1 r / theta.
template <typename TV>
__global__ void __launch_bounds__(kDotLanes) k_update_xr(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                         const double* __restrict__ alpha, const TV* __restrict__ p,
                                                         const TV* __restrict__ q, TV* __restrict__ x,
                                                         TV* __restrict__ r, double* __restrict__ partial,
                                                         const TV* __restrict__ dinv, TV* __restrict__ z0,
                                                         TV* __restrict__ r0, TV* __restrict__ d0) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const double al = alpha[wk.inst];
  const bool start = z0 && !L.coarsest;
  double v = 0;
#pragma unroll
  for (int i = 0; i < kBlock / kDotLanes; ++i) {
    const int j = wk.start + threadIdx.x + kDotLanes * i;
    if (j < L.N) {
      const long long g = L.voff + j;
      x[g] = (TV)((double)x[g] + al * (double)p[g]);
      const TV rr = (TV)((double)r[g] - al * (double)q[g]);
      r[g] = rr;
      v = fma((double)rr, (double)rr, v);
      if (start) {
        z0[g] = (TV)0;
        r0[g] = rr;
        d0[g] = (TV)((double)dinv[g] * (double)rr / L.cheb_theta);
      }
    }
  }
#pragma unroll
  for (int off = kDotLanes / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kDotLanes);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// Elementwise helpers for the refinement loop.
template <typename TS, typename TD>
__global__ void __launch_bounds__(kBlock) k_copy_scale(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                       const TS* __restrict__ s, TD* __restrict__ d,
                                                       const double* __restrict__ scale, int add) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  const long long g = L.voff + j;
  const double sc = scale ? scale[wk.inst] : 1.0;
  const double v = sc * (double)s[g];
  d[g] = add ? (TD)((double)d[g] + v) : (TD)v;
}

template <typename TV>
__global__ void __launch_bounds__(kBlock) k_fill(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                 TV* __restrict__ d, double v) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  d[L.voff + j] = (TV)v;
}

// ||A^T d||^2 partials: (A^T d)_u = c_phi f + [B] omega, (A^T d)_m = c_m f.
template <int D, typename TC>
__global__ void __launch_bounds__(kBlock) k_atd_norm(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                     CIdx ci, const TC* __restrict__ c, const TC* __restrict__ f,
                                                     const TC* __restrict__ w, double* __restrict__ partial) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  double v = 0;
  if (j < L.N) {
    int ic[kMaxD];
    coords<D>(L, j, ic);
    bool onB = false;
    for (int a = 0; a < D; ++a) onB |= (L.dlo[a] && ic[a] == 0) || (L.dhi[a] && ic[a] == L.n[a] - 1);
    const double fj = (double)f[L.voff + j];
    double tu = coef(c, L, ci.k[0], j) * fj + (onB ? (double)w[L.voff + j] : 0.0);
    v = tu * tu;
    for (int m = 1; m < 1 + 2 * D; ++m) {
      const double t = coef(c, L, ci.k[m], j) * fj;
      v += t * t;
    }
  }
  v = block_sum(v);
  if (threadIdx.x == 0) partial[blockIdx.x] = v;
}

// Local optimum of the derivative unknowns at p given u (and sigma*d); writes
// the scaled values xs[2a] = p_a, xs[2a+1] = q_a.  rhs_w (optional) adds a
// right-hand side in the scaled derivative unknowns (backward pass).
template <int D>
__device__ void local_derivs(const LInst& L, const CIdx& ci, const double* u, const double* cpl,
                             double fterm, const double* rw, long long p, const int* ic, double* xs,
                             double* rhoE_out, double ui) {
  // cpl: coefficient values at p per variable (0 if absent)
  double rhoE = cpl[0] * ui - fterm;
  double b1[kMaxD], b2[kMaxD], i11[kMaxD], i12[kMaxD], i22[kMaxD], ca[kMaxD], caa[kMaxD];
  double kap = 1, num = rhoE;
  for (int a = 0; a < D; ++a) {
    AxisRows<double, double> R = axis_rows<double, double>(L, a, u, p, ic[a], ui);
    ginv<double>(L, a, R.tp, R.tm, i11[a], i12[a], i22[a]);
    const double wT = L.wT[a];
    // A_w^T rho with rho = rows of u; the backward pass subtracts a rhs.
    b1[a] = wT * (R.rTp - R.rTm) + L.wC1[a] * R.rC1;
    b2[a] = wT * (R.rTp + R.rTm) * 0.5 + L.wC2[a] * R.rC2;
    if (rw) { b1[a] -= rw[2 * a]; b2[a] -= rw[2 * a + 1]; }
    ca[a] = cpl[1 + 2 * a] / L.s[a];
    caa[a] = cpl[2 + 2 * a] / (L.s[a] * L.s[a]);
  }
  // M x = -(c^ rhoE + b)  with M = G + c^ c^^T  (Sherman-Morrison)
  double g1[kMaxD], g2[kMaxD], h1[kMaxD], h2[kMaxD];
  for (int a = 0; a < D; ++a) {
    g1[a] = i11[a] * b1[a] + i12[a] * b2[a];
    g2[a] = i12[a] * b1[a] + i22[a] * b2[a];
    h1[a] = i11[a] * ca[a] + i12[a] * caa[a];
    h2[a] = i12[a] * ca[a] + i22[a] * caa[a];
    kap += ca[a] * h1[a] + caa[a] * h2[a];
    num -= ca[a] * g1[a] + caa[a] * g2[a];
  }
  const double gam = num / kap;
  for (int a = 0; a < D; ++a) {
    xs[2 * a] = -(g1[a] + h1[a] * gam);
    xs[2 * a + 1] = -(g2[a] + h2[a] * gam);
  }
  if (rhoE_out) *rhoE_out = gam;
}

// z_out (all V planes, physical units) from u (FP64).
template <int D, typename TC, typename TO>
__global__ void __launch_bounds__(kBlock) k_output(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                   CIdx ci, const double* __restrict__ u, const TC* __restrict__ c,
                                                   const TC* __restrict__ f, TO* __restrict__ z,
                                                   const long long* __restrict__ zoff) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  int ic[kMaxD];
  coords<D>(L, j, ic);
  double cpl[1 + 2 * kMaxD];
  for (int v = 0; v < 1 + 2 * D; ++v) cpl[v] = coef(c, L, ci.k[v], j);
  double xs[2 * kMaxD];
  const double ui = u[L.voff + j];
  local_derivs<D>(L, ci, u + L.voff, cpl, (double)f[L.voff + j], nullptr, j, ic, xs, nullptr, ui);
  TO* Z = z + zoff[wk.inst];
  Z[j] = (TO)ui;
  for (int a = 0; a < D; ++a) {
    Z[(long long)(1 + 2 * a) * L.N + j] = (TO)(xs[2 * a] / L.s[a]);
    Z[(long long)(2 + 2 * a) * L.N + j] = (TO)(xs[2 * a + 1] / (L.s[a] * L.s[a]));
  }
}

// Backward pass, step 1: v_i = M_i^-1 g~_w,i  (scaled derivative rhs) stored
// as 2D planes; g~_p = g_{u_a}/s_a, g~_q = g_{u_aa}/s_a^2.
template <int D, typename TC, typename TG>
__global__ void __launch_bounds__(kBlock) k_adj_local(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                      CIdx ci, const TC* __restrict__ c, const TG* __restrict__ gz,
                                                      const long long* __restrict__ zoff, double* __restrict__ vloc) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  int ic[kMaxD];
  coords<D>(L, j, ic);
  const TG* G = gz + zoff[wk.inst];
  double r1[kMaxD], r2[kMaxD], i11[kMaxD], i12[kMaxD], i22[kMaxD], ca[kMaxD], caa[kMaxD];
  double kap = 1, num = 0;
  double g1[kMaxD], g2[kMaxD], h1[kMaxD], h2[kMaxD];
  for (int a = 0; a < D; ++a) {
    int tp, tm, wp;
    axis_class(ic[a], L.n[a], L.per[a], tp, tm, wp);
    ginv<double>(L, a, tp, tm, i11[a], i12[a], i22[a]);
    r1[a] = (double)G[(long long)(1 + 2 * a) * L.N + j] / L.s[a];
    r2[a] = (double)G[(long long)(2 + 2 * a) * L.N + j] / (L.s[a] * L.s[a]);
    chat<double, TC>(L, ci, c, a, j, ca[a], caa[a]);
    g1[a] = i11[a] * r1[a] + i12[a] * r2[a];
    g2[a] = i12[a] * r1[a] + i22[a] * r2[a];
    h1[a] = i11[a] * ca[a] + i12[a] * caa[a];
    h2[a] = i12[a] * ca[a] + i22[a] * caa[a];
    kap += ca[a] * h1[a] + caa[a] * h2[a];
    num += ca[a] * g1[a] + caa[a] * g2[a];
  }
  const double t = num / kap;
  double* V = vloc + (long long)2 * D * L.voff;
  for (int a = 0; a < D; ++a) {
    V[(long long)(2 * a) * L.N + j] = g1[a] - h1[a] * t;
    V[(long long)(2 * a + 1) * L.N + j] = g2[a] - h2[a] * t;
  }
}

// Backward pass, step 2: g^_j = g_u,j - (A_u^T A_w v)_j.
template <int D, typename TC, typename TG>
__global__ void __launch_bounds__(kBlock) k_adj_rhs(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                    CIdx ci, const TC* __restrict__ c, const TG* __restrict__ gz,
                                                    const long long* __restrict__ zoff,
                                                    const double* __restrict__ vloc, double* __restrict__ ghat) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  int ic[kMaxD];
  coords<D>(L, j, ic);
  const double* V = vloc + (long long)2 * D * L.voff;
  double zE = 0;
  for (int a = 0; a < D; ++a) {
    double ca, caa;
    chat<double, TC>(L, ci, c, a, j, ca, caa);
    zE += ca * V[(long long)(2 * a) * L.N + j] + caa * V[(long long)(2 * a + 1) * L.N + j];
  }
  double y = coef(c, L, ci.k[0], j) * zE;
  for (int a = 0; a < D; ++a) {
    const int n = L.n[a], st = L.str[a], per = L.per[a], ia = ic[a];
    const double wT = L.wT[a];
    const int R = per ? 2 : 4;
    for (int o = -R; o <= R; ++o) {
      const int ii = ia + o;
      if (!per && (ii < 0 || ii >= n)) continue;
      const int iw = per ? wrap(ii, n) : ii;
      int tp, tm, wp;
      axis_class(iw, n, per, tp, tm, wp);
      const int k = wp - o;
      const bool inC = (k >= 0 && k <= 4);
      const bool inT = (o >= -1 && o <= 1);
      if (!inC && !inT) continue;
      const long long pi = nbr(j, ia, o, n, st, per);
      const double vp = V[(long long)(2 * a) * L.N + pi], vq = V[(long long)(2 * a + 1) * L.N + pi];
      const double zTp = tp ? wT * (vp + 0.5 * vq) : 0, zTm = tm ? wT * (-vp + 0.5 * vq) : 0;
      const double zC1 = L.wC1[a] * vp, zC2 = L.wC2[a] * vq;
      if (inC) y -= L.wC1[a] * c_W1[wp][k] * zC1 + L.wC2[a] * c_W2[wp][k] * zC2;
      if (o == 0) y += wT * (zTp + zTm);
      else if (o == -1) y -= wT * zTp;
      else if (o == 1) y -= wT * zTm;
    }
  }
  const TG* G = gz + zoff[wk.inst];
  ghat[L.voff + j] = (double)G[j] - y;
}

// Backward pass, step 3: d_z from d_u, the dual variables and the gradients.
template <int D, typename TC, typename TG>
__global__ void __launch_bounds__(kBlock) k_adj_grad(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                     CIdx ci, const TC* __restrict__ c, const TC* __restrict__ f,
                                                     const double* __restrict__ ustar, const double* __restrict__ du,
                                                     const TG* __restrict__ gz, const long long* __restrict__ zoff,
                                                     TG* __restrict__ gc, TG* __restrict__ gf, TG* __restrict__ gw) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  int ic[kMaxD];
  coords<D>(L, j, ic);
  double cpl[1 + 2 * kMaxD];
  for (int v = 0; v < 1 + 2 * D; ++v) cpl[v] = coef(c, L, ci.k[v], j);
  const double fj = (double)f[L.voff + j];
  // z* at j (physical units)
  double xs[2 * kMaxD], zs[1 + 2 * kMaxD];
  const double us = ustar[L.voff + j];
  local_derivs<D>(L, ci, ustar + L.voff, cpl, fj, nullptr, j, ic, xs, nullptr, us);
  zs[0] = us;
  for (int a = 0; a < D; ++a) { zs[1 + 2 * a] = xs[2 * a] / L.s[a]; zs[2 + 2 * a] = xs[2 * a + 1] / (L.s[a] * L.s[a]); }
  // d_z at j: derivative unknowns minimise the local rows with rhs g~_w
  const TG* G = gz + zoff[wk.inst];
  double rw[2 * kMaxD];
  for (int a = 0; a < D; ++a) {
    rw[2 * a] = (double)G[(long long)(1 + 2 * a) * L.N + j] / L.s[a];
    rw[2 * a + 1] = (double)G[(long long)(2 + 2 * a) * L.N + j] / (L.s[a] * L.s[a]);
  }
  double dx[2 * kMaxD], dzv[1 + 2 * kMaxD];
  const double duj = du[L.voff + j];
  local_derivs<D>(L, ci, du + L.voff, cpl, 0.0, rw, j, ic, dx, nullptr, duj);
  dzv[0] = duj;
  for (int a = 0; a < D; ++a) { dzv[1 + 2 * a] = dx[2 * a] / L.s[a]; dzv[2 + 2 * a] = dx[2 * a + 1] / (L.s[a] * L.s[a]); }
  double Az = 0, Adz = 0;
  for (int v = 0; v < 1 + 2 * D; ++v) { Az += cpl[v] * zs[v]; Adz += cpl[v] * dzv[v]; }
  const double lamE = fj - Az;       // lambda* on the equation row
  const double dlamE = -Adz;         // d_lambda = -A d_z on the equation row
  if (gc) {
    TG* GC = gc + L.coff;
    for (int v = 0; v < 1 + 2 * D; ++v) {
      const int k = ci.k[v];
      if (k < 0) continue;
      GC[(long long)k * L.N + j] = (TG)(dlamE * zs[v] + lamE * dzv[v]);
    }
  }
  if (gf) gf[L.voff + j] = (TG)(-dlamE);
  if (gw) {
    bool onB = false;
    for (int a = 0; a < D; ++a) onB |= (L.dlo[a] && ic[a] == 0) || (L.dhi[a] && ic[a] == L.n[a] - 1);
    gw[L.voff + j] = (TG)(onB ? duj : 0.0);
  }
}

// Non-finite scan of an input array: flag[0] |= any element is NaN/Inf.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_nonfinite(const T* __restrict__ a, long long n, int* __restrict__ flag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !isfinite((double)a[i])) flag[0] = 1;
}

// ---------------------------------------------------------------- launchers
#define GRID(nb) dim3((unsigned)(nb)), dim3(kBlock), 0, st

template <typename TA, typename TV, typename TC>
void launch_gamma(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TV* u,
                  const TC* c, const TC* f, int sigma, TV* gam) {
  if (nb <= 0) return;
  if (D == 2) hipLaunchKernelGGL((k_gamma<2, TA, TV, TC>), GRID(nb), w, li, ci, u, c, f, sigma, gam);
  else hipLaunchKernelGGL((k_gamma<3, TA, TV, TC>), GRID(nb), w, li, ci, u, c, f, sigma, gam);
}

template <typename TA, typename TV, typename TC>
void launch_gather(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TV* u,
                   const TV* gam, const TC* c, const TC* bw, int sigma, int mode, TV* out, const TV* bvec,
                   TV* x, TV* r, TV* d, const TV* dinv, int cheb_step, double* partial) {
  if (nb <= 0) return;
  if (D == 2)
    hipLaunchKernelGGL((k_gather<2, TA, TV, TC>), GRID(nb), w, li, ci, u, gam, c, bw, sigma, mode, out, bvec, x, r,
                       d, dinv, cheb_step, partial);
  else
    hipLaunchKernelGGL((k_gather<3, TA, TV, TC>), GRID(nb), w, li, ci, u, gam, c, bw, sigma, mode, out, bvec, x, r,
                       d, dinv, cheb_step, partial);
}

template <typename TV, typename TC>
void launch_diag(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c, TV* dinv) {
  if (nb <= 0) return;
  if (D == 2) hipLaunchKernelGGL((k_diag<2, TV, TC>), GRID(nb), w, li, ci, c, dinv);
  else hipLaunchKernelGGL((k_diag<3, TV, TC>), GRID(nb), w, li, ci, c, dinv);
}

template <typename TV>
void launch_cheb_init(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* b, const TV* dinv, TV* x,
                      TV* r, TV* d) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_cheb_init<TV>), GRID(nb), w, li, b, dinv, x, r, d);
}

template <typename TV>
void launch_restrict(int D, hipStream_t st, const Work* w, int nb, const LInst* lf, const LInst* lc, const TV* rf,
                     TV* rc, const TV* dinv, TV* xc, TV* r0, TV* d0) {
  if (nb <= 0) return;
  if (D == 2) hipLaunchKernelGGL((k_restrict<2, TV>), GRID(nb), w, lf, lc, rf, rc, dinv, xc, r0, d0);
  else hipLaunchKernelGGL((k_restrict<3, TV>), GRID(nb), w, lf, lc, rf, rc, dinv, xc, r0, d0);
}

template <typename TV>
void launch_prolong_add(int D, hipStream_t st, const Work* w, int nb, const LInst* lf, const LInst* lc,
                        const TV* ec, TV* xf) {
  if (nb <= 0) return;
  if (D == 2) hipLaunchKernelGGL((k_prolong_add<2, TV>), GRID(nb), w, lf, lc, ec, xf);
  else hipLaunchKernelGGL((k_prolong_add<3, TV>), GRID(nb), w, lf, lc, ec, xf);
}

template <typename TC>
void launch_coarsen_coef(int D, hipStream_t st, const Work* w, int nb, const LInst* lf, const LInst* lc, int K,
                         const TC* cf, TC* cc) {
  if (nb <= 0) return;
  if (D == 2) hipLaunchKernelGGL((k_coarsen_coef<2, TC>), GRID(nb), w, lf, lc, K, cf, cc);
  else hipLaunchKernelGGL((k_coarsen_coef<3, TC>), GRID(nb), w, lf, lc, K, cf, cc);
}

void launch_set_unit(hipStream_t st, const LInst* probe, const int* col, int nprobe, double* U) {
  if (nprobe <= 0) return;
  hipLaunchKernelGGL(k_set_unit, dim3((nprobe + 255) / 256), dim3(256), 0, st, probe, col, nprobe, U);
}

void launch_gauss_jordan(hipStream_t st, int nmat, double* A, const long long* off, const int* n, int* fail) {
  if (nmat <= 0) return;
  hipLaunchKernelGGL(k_gauss_jordan, dim3(nmat), dim3(1024), 0, st, A, off, n, fail);
}

void launch_set_probe(hipStream_t st, const LInst* probe, const int* pc, const int* ps, int nprobe, int ncolor,
                      double* U) {
  if (nprobe <= 0) return;
  hipLaunchKernelGGL(k_set_probe, dim3(nprobe), dim3(64), 0, st, probe, pc, ps, nprobe, ncolor, U);
}

void launch_extract_probe(hipStream_t st, const Work* w, int nb, const LInst* probe, const int* pc, const int* ps,
                          const long long* dout, int ncolor, const double* Y, double* S) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_extract_probe, dim3(nb), dim3(kBlock), 0, st, w, probe, pc, ps, dout, ncolor, Y, S);
}

void launch_extract_band(hipStream_t st, const Work* w, int nb, const LInst* probe, const int* pc, const int* ps,
                         const long long* bout, int ncolor, const double* Y, double* Lb) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_extract_band, dim3(nb), dim3(kBlock), 0, st, w, probe, pc, ps, bout, ncolor, Y, Lb);
}

void launch_bb_factor(hipStream_t st, int nmat, double* Lb, const long long* boff, const int* T, const int* m,
                      int* fail) {
  if (nmat <= 0) return;
  hipLaunchKernelGGL(k_bb_factor, dim3(nmat), dim3(kBBThreads), 0, st, Lb, boff, T, m, fail);
}

// Specialisation for 64-point planes: thread (r, h) owns 16 consecutive
// columns h*16..h*16+15 of row r in every block; the four off-diagonal
// blocks of the next step are prefetched into registers while the current
// step's reductions run.
// Sum over the four lanes of a quad (lanes 4i..4i+3) by two DPP quad
// permutations (lane ^ 1, then lane ^ 2) on the two halves of the double:
// register moves within the wavefront, no LDS round trip.
template <int CTRL>
__device__ __forceinline__ double dpp_quad(double v) {
  int2 h = __builtin_bit_cast(int2, v);
  h.x = __builtin_amdgcn_update_dpp(0, h.x, CTRL, 0xF, 0xF, false);
  h.y = __builtin_amdgcn_update_dpp(0, h.y, CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, h);
}
__device__ __forceinline__ double quad_sum(double v) {
  v += dpp_quad<0xB1>(v);   // quad_perm [1, 0, 3, 2]
  v += dpp_quad<0x4E>(v);   // quad_perm [2, 3, 0, 1]
  return v;
}

template <typename TV>
__global__ void __launch_bounds__(kBlock) k_bb_solve64(const int* __restrict__ inst_list,
                                                       const LInst* __restrict__ li, const TV* __restrict__ Lb,
                                                       const TV* __restrict__ bvec, TV* __restrict__ xvec) {
  constexpr int M = 64, CW = 16;
  const LInst& L = li[inst_list[blockIdx.x]];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const int T = L.n[0];
  const long long base = L.doff;
  __shared__ double ys[4096];
  __shared__ double acc[M];
  const int tid = threadIdx.x, r = tid >> 2, h = tid & 3, c0 = h * CW;
  const TV* B = bvec + L.voff;
  TV* X = xvec + L.voff;
  // The five blocks of a plane (k = 0: the diagonal-block inverse, k = 1..4
  // the sub-diagonal blocks) are loaded DEP planes ahead into DEP + 1
  // register sets used in rotation (two planes ahead for FP32 factors; the
  // FP64 sets are twice as large, so one plane); the loops are unrolled by
  // DEP + 1 so that every set keeps fixed registers.
  constexpr int DEP = sizeof(TV) == 4 ? 2 : 1;
  TV pre[DEP + 1][5][CW];
  TV bpre[DEP + 1];
  // Every load is unconditional: the plane index is clamped to [0, T) and
  // blocks that a plane does not use (k > t, or past the ends) are loaded
  // from valid storage and ignored, so no load sits in a branch and the
  // compiler's wait counts stay partial (a conditional load or a store in
  // the loop makes it wait for every load in flight at each barrier).
  // (a thread's 16 entries of a block row are contiguous and 16-byte
  // aligned: block offsets are multiples of 4 elements)
  auto clampt = [&](int t) { return t < 0 ? 0 : (t >= T ? T - 1 : t); };
  auto load_fwd = [&](int t, TV(&d)[5][CW], TV& bt) {
    const int tc = clampt(t);
#pragma unroll
    for (int k = 0; k <= 4; ++k) {
      const uint4* Lk = reinterpret_cast<const uint4*>(Lb + bb_at(base, tc, k, M) + r * M + c0);
#pragma unroll
      for (int v = 0; v < CW * (int)sizeof(TV) / 16; ++v) {
        const uint4 x = Lk[v];
        __builtin_memcpy(&d[k][v * 16 / sizeof(TV)], &x, 16);
      }
    }
    bt = B[(long long)tc * M + r];
  };
  // (one accumulator per block and two for the diagonal product keep the
  // dependent FMA chains short)
  auto fwd = [&](int t, TV(&cur)[5][CW], TV bt, TV(&nxt)[5][CW], TV& nbt) {
    double sk[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 1; k <= 4; ++k)
      if (t - k >= 0) {
        const double* yk = ys + (t - k) * M + c0;
#pragma unroll
        for (int q = 0; q < CW; ++q) sk[k - 1] = fma(-(double)cur[k][q], yk[q], sk[k - 1]);
      }
    load_fwd(t + DEP, nxt, nbt);
    double s = ((h == 0) ? (double)bt : 0.0) + ((sk[0] + sk[1]) + (sk[2] + sk[3]));
    s = quad_sum(s);
    if (h == 0) acc[r] = s;
    __syncthreads();
    double v0 = 0, v1 = 0;
#pragma unroll
    for (int q = 0; q < CW; q += 2) {   // Dinv lower: upper entries are 0
      v0 = fma((double)cur[0][q], acc[c0 + q], v0);
      v1 = fma((double)cur[0][q + 1], acc[c0 + q + 1], v1);
    }
    const double v = quad_sum(v0 + v1);
    if (h == 0) ys[t * M + r] = v;
    __syncthreads();
  };
#pragma unroll
  for (int i = 0; i < DEP; ++i) load_fwd(i, pre[i], bpre[i]);
  // plane t + i uses set i and refills set (i + DEP) mod (DEP + 1); whole
  // groups of DEP + 1 planes, then the remaining planes
  int t = 0;
  for (; t + DEP < T; t += DEP + 1) {
#pragma unroll
    for (int i = 0; i <= DEP; ++i) fwd(t + i, pre[i], bpre[i], pre[(i + DEP) % (DEP + 1)], bpre[(i + DEP) % (DEP + 1)]);
  }
#pragma unroll
  for (int i = 0; i < DEP; ++i)
    if (t + i < T) fwd(t + i, pre[i], bpre[i], pre[(i + DEP) % (DEP + 1)], bpre[(i + DEP) % (DEP + 1)]);
  // backward: x_t = Dinv_t^T (y_t - sum_k L[t+k][k]^T x_{t+k}); thread (r, h)
  // accumulates column r over rows h*16..h*16+15 of each block; x overwrites
  // y in LDS and is written out after the sweep.
  auto load_bwd = [&](int t, TV(&d)[5][CW]) {
#pragma unroll
    for (int k = 0; k <= 4; ++k) {
      const TV* Lk = Lb + bb_at(base, clampt(t + k), k, M);
#pragma unroll
      for (int q = 0; q < CW; ++q) d[k][q] = Lk[(c0 + q) * M + r];
    }
  };
  auto bwd = [&](int t, TV(&cur)[5][CW], TV(&nxt)[5][CW]) {
    double sk[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 1; k <= 4; ++k)
      if (t + k < T) {
        const double* xk = ys + (t + k) * M + c0;
#pragma unroll
        for (int q = 0; q < CW; ++q) sk[k - 1] = fma(-(double)cur[k][q], xk[q], sk[k - 1]);
      }
    load_bwd(t - DEP, nxt);
    double s = ((h == 0) ? ys[t * M + r] : 0.0) + ((sk[0] + sk[1]) + (sk[2] + sk[3]));
    s = quad_sum(s);
    if (h == 0) acc[r] = s;
    __syncthreads();
    double v0 = 0, v1 = 0;
#pragma unroll
    for (int q = 0; q < CW; q += 2) {
      v0 = fma((double)cur[0][q], acc[c0 + q], v0);
      v1 = fma((double)cur[0][q + 1], acc[c0 + q + 1], v1);
    }
    const double v = quad_sum(v0 + v1);
    if (h == 0) ys[t * M + r] = v;
    __syncthreads();
  };
#pragma unroll
  for (int i = 0; i < DEP; ++i) load_bwd(T - 1 - i, pre[i]);
  t = T - 1;
  for (; t - DEP >= 0; t -= DEP + 1) {
#pragma unroll
    for (int i = 0; i <= DEP; ++i) bwd(t - i, pre[i], pre[(i + DEP) % (DEP + 1)]);
  }
#pragma unroll
  for (int i = 0; i < DEP; ++i)
    if (t - i >= 0) bwd(t - i, pre[i], pre[(i + DEP) % (DEP + 1)]);
  for (int e = tid; e < T * M; e += kBlock) X[e] = (TV)ys[e];
}

// Specialisation for planes of at most 16 points: one wavefront per
// instance, lane (r, h) = row r, column class h (columns h, h+4, h+8, h+12).
// The recurrence needs no barrier: row sums are lane shuffles, the
// substituted values of the last four planes stay in registers, and the
// band blocks of the next plane are loaded while the current one is reduced.
constexpr int kBBS = 16;
template <typename TV>
__global__ void __launch_bounds__(64) k_bb_solve16(const int* __restrict__ inst_list, const LInst* __restrict__ li,
                                                   const TV* __restrict__ Lb, const TV* __restrict__ bvec,
                                                   TV* __restrict__ xvec) {
  const LInst& L = li[inst_list[blockIdx.x]];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  const int T = L.n[0], m = L.N / T;
  const long long base = L.doff;
  __shared__ double ys[4096];           // y then x (T * m <= 4096, the coarsest-grid limit)
  const int lane = threadIdx.x, r = lane >> 2, h = lane & 3;
  const bool live = r < m;
  const TV* B = bvec + L.voff;
  TV* X = xvec + L.voff;
  auto rowsum = [](double v) {
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    return v;
  };
  // forward: y_t = Dinv_t (b_t - sum_k L[t][k] y_{t-k}); lane holds row r of
  // L[t][k] at its columns and of Dinv_t
  double yh[4][4] = {};                 // yh[k-1][j] = y_{t-k}[h + 4j]
  double lc[5][4], ln[5][4];
  auto load_fwd = [&](int t, double (&dst)[5][4]) {
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int c = h + 4 * j;
        dst[k][j] = (live && c < m && k <= t && t < T) ? (double)Lb[bb_at(base, t, k, m) + (long long)r * m + c] : 0.0;
      }
  };
  load_fwd(0, lc);
  for (int t = 0; t < T; ++t) {
    load_fwd(t + 1, ln);
    double s = (live && h == 0) ? (double)B[(long long)t * m + r] : 0.0;
#pragma unroll
    for (int k = 1; k <= 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) s -= lc[k][j] * yh[k - 1][j];
    s = rowsum(s);
    double v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int c = h + 4 * j;
      const double sc = __shfl(s, (c < 16 ? c : 15) * 4, 64);
      if (c <= r) v += lc[0][j] * sc;
    }
    const double y = rowsum(v);
    if (live && h == 0) ys[t * m + r] = y;
#pragma unroll
    for (int k = 3; k > 0; --k)
#pragma unroll
      for (int j = 0; j < 4; ++j) yh[k][j] = yh[k - 1][j];
#pragma unroll
    for (int j = 0; j < 4; ++j) yh[0][j] = __shfl(y, (h + 4 * j) * 4, 64);
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) lc[k][j] = ln[k][j];
  }
  __syncthreads();
  // backward: x_t = Dinv_t^T (y_t - sum_k L[t+k][k]^T x_{t+k}); lane holds
  // column r of L[t+k][k] at rows h + 4j, and of Dinv_t
  double xh[4][4] = {};                 // xh[k-1][j] = x_{t+k}[h + 4j]
  auto load_bwd = [&](int t, double (&dst)[5][4]) {
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = h + 4 * j;
        dst[k][j] = (live && q < m && t >= 0 && t + k < T) ? (double)Lb[bb_at(base, t + k, k, m) + (long long)q * m + r]
                                                           : 0.0;
      }
  };
  load_bwd(T - 1, lc);
  for (int t = T - 1; t >= 0; --t) {
    load_bwd(t - 1, ln);
    double s = (live && h == 0) ? ys[t * m + r] : 0.0;
#pragma unroll
    for (int k = 1; k <= 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) s -= lc[k][j] * xh[k - 1][j];
    s = rowsum(s);
    double v = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = h + 4 * j;
      const double sq = __shfl(s, (q < 16 ? q : 15) * 4, 64);
      if (q >= r && q < m) v += lc[0][j] * sq;
    }
    const double x = rowsum(v);
    if (live && h == 0) X[(long long)t * m + r] = (TV)x;
#pragma unroll
    for (int k = 3; k > 0; --k)
#pragma unroll
      for (int j = 0; j < 4; ++j) xh[k][j] = xh[k - 1][j];
#pragma unroll
    for (int j = 0; j < 4; ++j) xh[0][j] = __shfl(x, (h + 4 * j) * 4, 64);
#pragma unroll
    for (int k = 0; k < 5; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) lc[k][j] = ln[k][j];
  }
}

template <typename TV>
void launch_bb_solve16(hipStream_t st, int ninst, const int* inst_list, const LInst* li, const TV* Lb, const TV* b,
                       TV* x) {
  if (ninst <= 0) return;
  hipLaunchKernelGGL((k_bb_solve16<TV>), dim3(ninst), dim3(64), 0, st, inst_list, li, Lb, b, x);
}
template void launch_bb_solve16<float>(hipStream_t, int, const int*, const LInst*, const float*, const float*,
                                       float*);
template void launch_bb_solve16<double>(hipStream_t, int, const int*, const LInst*, const double*, const double*,
                                        double*);

template <typename TV>
void launch_bb_solve(hipStream_t st, int ninst, const int* inst_list, const LInst* li, const TV* Lb, const TV* b,
                     TV* x) {
  if (ninst <= 0) return;
  hipLaunchKernelGGL((k_bb_solve<TV>), dim3(ninst), dim3(kBlock), 0, st, inst_list, li, Lb, b, x);
}

template <typename TV>
void launch_bb_solve64(hipStream_t st, int ninst, const int* inst_list, const LInst* li, const TV* Lb, const TV* b,
                       TV* x) {
  if (ninst <= 0) return;
  hipLaunchKernelGGL((k_bb_solve64<TV>), dim3(ninst), dim3(kBlock), 0, st, inst_list, li, Lb, b, x);
}
template void launch_bb_solve<float>(hipStream_t, int, const int*, const LInst*, const float*, const float*, float*);
template void launch_bb_solve64<float>(hipStream_t, int, const int*, const LInst*, const float*, const float*,
                                       float*);
template void launch_bb_solve64<double>(hipStream_t, int, const int*, const LInst*, const double*, const double*,
                                        double*);
template void launch_bb_solve<double>(hipStream_t, int, const int*, const LInst*, const double*, const double*,
                                      double*);

void launch_band_chol(hipStream_t st, int nmat, double* A, const long long* off, const int* n, const int* bw,
                      int* fail) {
  if (nmat <= 0) return;
  hipLaunchKernelGGL(k_band_chol, dim3(nmat), dim3(kBlock), 0, st, A, off, n, bw, fail);
}

void launch_band_inverse(hipStream_t st, int nblocks, const double* L, double* X, const long long* off,
                         const int* n, const int* bw, const int* mat_of_block, const int* col0_of_block) {
  if (nblocks <= 0) return;
  hipLaunchKernelGGL(k_band_inverse, dim3(nblocks), dim3(kBlock), 0, st, L, X, off, n, bw, mat_of_block,
                     col0_of_block);
}

template <typename TV>
void launch_convert_dense(hipStream_t st, const double* src, TV* dst, long long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_convert_dense<TV>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, src,
                     dst, n);
}

template <typename TV>
void launch_dense_apply(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* Sinv, const TV* r, TV* e) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_dense_apply<TV>), GRID(nb), w, li, Sinv, r, e);
}

template <typename TA, typename TV>
void launch_dot(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* a, const TV* b, double* partial) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_dot<TA, TV>), dim3((unsigned)nb), dim3(kDotLanes), 0, st, w, li, a, b, partial);
}

void launch_finish_sum(hipStream_t st, const double* partial, const int* bstart, int B, double* out) {
  hipLaunchKernelGGL(k_finish_sum, dim3(B), dim3(kBlock), 0, st, partial, bstart, B, out);
}

void launch_finish_scalars(hipStream_t st, const double* partial, const int* bstart, int B, double* out, int op,
                           int first, const double* tol2, double* rz, double* beta, double* alpha,
                           const double* r0n2, int* active, int* iters) {
  hipLaunchKernelGGL(k_finish_scalars, dim3(B), dim3(kBlock), 0, st, partial, bstart, out, op, first, tol2, rz, beta,
                     alpha, r0n2, active, iters);
}

void launch_pcg_scalars(hipStream_t st, int op, int B, int first, const double* tol2, double* rz_new, double* rz,
                        double* beta, double* pq, double* alpha, double* rn2, double* r0n2, int* active,
                        int* iters) {
  hipLaunchKernelGGL(k_pcg_scalars, dim3((B + 255) / 256), dim3(256), 0, st, op, B, first, tol2, rz_new, rz, beta,
                     pq, alpha, rn2, r0n2, active, iters);
}

template <typename TV>
void launch_update_p(hipStream_t st, const Work* w, int nb, const LInst* li, const double* beta, const TV* z,
                     TV* p) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_update_p<TV>), GRID(nb), w, li, beta, z, p);
}
template <typename TV>
void launch_update_pq(hipStream_t st, const Work* w, int nb, const LInst* li, const double* beta, const TV* z,
                      const TV* r, const TV* rv, TV* p, TV* q, double* partial) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_update_pq<TV>), dim3((unsigned)nb), dim3(kDotLanes), 0, st, w, li, beta, z, r, rv, p, q, partial);
}

template <typename TV>
void launch_update_xr(hipStream_t st, const Work* w, int nb, const LInst* li, const double* alpha, const TV* p,
                      const TV* q, TV* x, TV* r, double* partial, const TV* dinv, TV* z0, TV* r0, TV* d0) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_update_xr<TV>), dim3((unsigned)nb), dim3(kDotLanes), 0, st, w, li, alpha, p, q, x, r, partial,
                     dinv, z0, r0, d0);
}

template <typename TS, typename TD>
void launch_copy_scale(hipStream_t st, const Work* w, int nb, const LInst* li, const TS* s, TD* d,
                       const double* scale, int add) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_copy_scale<TS, TD>), GRID(nb), w, li, s, d, scale, add);
}

template <typename TV>
void launch_fill(hipStream_t st, const Work* w, int nb, const LInst* li, TV* d, double v) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_fill<TV>), GRID(nb), w, li, d, v);
}

template <typename TC>
void launch_atd_norm(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                     const TC* f, const TC* bw, double* partial) {
  if (D == 2) hipLaunchKernelGGL((k_atd_norm<2, TC>), GRID(nb), w, li, ci, c, f, bw, partial);
  else hipLaunchKernelGGL((k_atd_norm<3, TC>), GRID(nb), w, li, ci, c, f, bw, partial);
}

template <typename TC, typename TO>
void launch_output(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const double* u,
                   const TC* c, const TC* f, TO* z, const long long* zoff) {
  if (D == 2) hipLaunchKernelGGL((k_output<2, TC, TO>), GRID(nb), w, li, ci, u, c, f, z, zoff);
  else hipLaunchKernelGGL((k_output<3, TC, TO>), GRID(nb), w, li, ci, u, c, f, z, zoff);
}

template <typename TC, typename TG>
void launch_adj_local(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                      const TG* gz, const long long* zoff, double* vloc) {
  if (D == 2) hipLaunchKernelGGL((k_adj_local<2, TC, TG>), GRID(nb), w, li, ci, c, gz, zoff, vloc);
  else hipLaunchKernelGGL((k_adj_local<3, TC, TG>), GRID(nb), w, li, ci, c, gz, zoff, vloc);
}

template <typename TC, typename TG>
void launch_adj_rhs(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                    const TG* gz, const long long* zoff, const double* vloc, double* ghat) {
  if (D == 2) hipLaunchKernelGGL((k_adj_rhs<2, TC, TG>), GRID(nb), w, li, ci, c, gz, zoff, vloc, ghat);
  else hipLaunchKernelGGL((k_adj_rhs<3, TC, TG>), GRID(nb), w, li, ci, c, gz, zoff, vloc, ghat);
}

template <typename TC, typename TG>
void launch_adj_grad(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                     const TC* f, const double* ustar, const double* du, const TG* gz, const long long* zoff,
                     TG* gc, TG* gf, TG* gw) {
  if (D == 2)
    hipLaunchKernelGGL((k_adj_grad<2, TC, TG>), GRID(nb), w, li, ci, c, f, ustar, du, gz, zoff, gc, gf, gw);
  else
    hipLaunchKernelGGL((k_adj_grad<3, TC, TG>), GRID(nb), w, li, ci, c, f, ustar, du, gz, zoff, gc, gf, gw);
}

template <typename T>
void launch_nonfinite(hipStream_t st, const T* a, long long n, int* flag) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_nonfinite<T>), dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, a, n, flag);
}

// ---------------------------------------------------------------- instantiations
#define INST_TV_TC(TA, TV, TC)                                                                                   \
  template void launch_gamma<TA, TV, TC>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const TV*,       \
                                         const TC*, const TC*, int, TV*);                                         \
  template void launch_gather<TA, TV, TC>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const TV*,      \
                                          const TV*, const TC*, const TC*, int, int, TV*, const TV*, TV*, TV*,    \
                                          TV*, const TV*, int, double*);
INST_TV_TC(float, float, float)
INST_TV_TC(double, double, float)
INST_TV_TC(double, double, double)

#define INST_TV(TV)                                                                                              \
  template void launch_cheb_init<TV>(hipStream_t, const Work*, int, const LInst*, const TV*, const TV*, TV*, TV*, \
                                     TV*);                                                                        \
  template void launch_restrict<TV>(int, hipStream_t, const Work*, int, const LInst*, const LInst*, const TV*,    \
                                    TV*, const TV*, TV*, TV*, TV*);                                               \
  template void launch_prolong_add<TV>(int, hipStream_t, const Work*, int, const LInst*, const LInst*, const TV*, \
                                       TV*);                                                                      \
  template void launch_convert_dense<TV>(hipStream_t, const double*, TV*, long long);                             \
  template void launch_dense_apply<TV>(hipStream_t, const Work*, int, const LInst*, const TV*, const TV*, TV*);   \
  template void launch_dot<double, TV>(hipStream_t, const Work*, int, const LInst*, const TV*, const TV*,         \
                                       double*);                                                                  \
  template void launch_update_p<TV>(hipStream_t, const Work*, int, const LInst*, const double*, const TV*, TV*);  \
  template void launch_update_pq<TV>(hipStream_t, const Work*, int, const LInst*, const double*, const TV*,       \
                                     const TV*, const TV*, TV*, TV*, double*);                                    \
  template void launch_update_xr<TV>(hipStream_t, const Work*, int, const LInst*, const double*, const TV*,       \
                                     const TV*, TV*, TV*, double*, const TV*, TV*, TV*, TV*);                     \
  template void launch_fill<TV>(hipStream_t, const Work*, int, const LInst*, TV*, double);
INST_TV(float)
INST_TV(double)

template void launch_diag<float, float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const float*, float*);
template void launch_diag<double, double>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const double*,
                                          double*);
template void launch_diag<double, float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const float*,
                                         double*);
template void launch_coarsen_coef<float>(int, hipStream_t, const Work*, int, const LInst*, const LInst*, int,
                                         const float*, float*);
template void launch_coarsen_coef<double>(int, hipStream_t, const Work*, int, const LInst*, const LInst*, int,
                                          const double*, double*);
template void launch_copy_scale<double, float>(hipStream_t, const Work*, int, const LInst*, const double*, float*,
                                               const double*, int);
template void launch_copy_scale<float, double>(hipStream_t, const Work*, int, const LInst*, const float*, double*,
                                               const double*, int);
template void launch_copy_scale<float, float>(hipStream_t, const Work*, int, const LInst*, const float*, float*,
                                              const double*, int);
template void launch_copy_scale<double, double>(hipStream_t, const Work*, int, const LInst*, const double*,
                                                double*, const double*, int);
template void launch_atd_norm<float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const float*,
                                     const float*, const float*, double*);
template void launch_atd_norm<double>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const double*,
                                      const double*, const double*, double*);
template void launch_output<float, float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const double*,
                                          const float*, const float*, float*, const long long*);
template void launch_output<float, double>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const double*,
                                           const float*, const float*, double*, const long long*);
template void launch_output<double, double>(int, hipStream_t, const Work*, int, const LInst*, CIdx,
                                            const double*, const double*, const double*, double*,
                                            const long long*);
template void launch_adj_local<float, float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const float*,
                                             const float*, const long long*, double*);
template void launch_adj_local<double, double>(int, hipStream_t, const Work*, int, const LInst*, CIdx,
                                               const double*, const double*, const long long*, double*);
template void launch_adj_rhs<float, float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const float*,
                                           const float*, const long long*, const double*, double*);
template void launch_adj_rhs<double, double>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const double*,
                                             const double*, const long long*, const double*, double*);
template void launch_adj_grad<float, float>(int, hipStream_t, const Work*, int, const LInst*, CIdx, const float*,
                                            const float*, const double*, const double*, const float*,
                                            const long long*, float*, float*, float*);
template void launch_adj_grad<double, double>(int, hipStream_t, const Work*, int, const LInst*, CIdx,
                                              const double*, const double*, const double*, const double*,
                                              const double*, const long long*, double*, double*, double*);
template void launch_nonfinite<float>(hipStream_t, const float*, long long, int*);
template void launch_nonfinite<double>(hipStream_t, const double*, long long, int*);

// Power iteration helpers for the Chebyshev interval of D^-1 S.
template <typename TV>
__global__ void __launch_bounds__(kBlock) k_hash_fill(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                      TV* __restrict__ v, unsigned seed) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  if (j >= L.N) return;
  // hashed on the point's index within its instance, so that an instance's
  // start vector (and its Chebyshev interval) does not depend on its place
  // in the batch
  unsigned h = (unsigned)j * 2654435761u ^ (seed * 2246822519u + 0x9e3779b9u);
  h ^= h >> 15; h *= 2246822519u; h ^= h >> 13; h *= 3266489917u; h ^= h >> 16;
  v[L.voff + j] = (TV)((double)(h & 0xffffff) / (double)0x800000 - 1.0);
}

template <typename TV>
__global__ void __launch_bounds__(kBlock) k_mul_dinv(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                     const TV* __restrict__ dinv, const TV* __restrict__ y,
                                                     TV* __restrict__ v, double* __restrict__ partial) {
  // v = D^-1 y, partial = sum v^2 / dinv  (= v^T D v)
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int j = wk.start + threadIdx.x;
  double s = 0;
  if (j < L.N) {
    const long long g = L.voff + j;
    const double di = (double)dinv[g];
    const double vv = di * (double)y[g];
    v[g] = (TV)vv;
    s = vv * vv / di;
  }
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename TV>
void launch_hash_fill(hipStream_t st, const Work* w, int nb, const LInst* li, TV* v, unsigned seed) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_hash_fill<TV>), GRID(nb), w, li, v, seed);
}

template <typename TV>
void launch_mul_dinv(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* dinv, const TV* y, TV* v,
                     double* partial) {
  if (nb <= 0) return;
  hipLaunchKernelGGL((k_mul_dinv<TV>), GRID(nb), w, li, dinv, y, v, partial);
}
template void launch_hash_fill<float>(hipStream_t, const Work*, int, const LInst*, float*, unsigned);
template void launch_hash_fill<double>(hipStream_t, const Work*, int, const LInst*, double*, unsigned);
template void launch_mul_dinv<float>(hipStream_t, const Work*, int, const LInst*, const float*, const float*, float*,
                                     double*);
template void launch_mul_dinv<double>(hipStream_t, const Work*, int, const LInst*, const double*, const double*,
                                      double*, double*);

}  // namespace mpde
