// BF16 MFMA kernels of the learned coarse-grid correction: 3x3x3 "same"
// convolutions over a (t, x, y) grid, 16 input and 16 output channels,
// channels last, zero padding on non-periodic axes and wrap-around on
// periodic ones; FP32 accumulation.  Implicit GEMM on
// v_mfma_f32_16x16x16_bf16: per wave a tile of 16 grid points x 16 output
// channels, K = 16 input channels per tap, 27 taps.
//
// MFMA operand layout (16x16x16, wave64), lane l = 16*g + i:
//   A (16 x 16, rows = points, cols = k): lane holds A[i][4g .. 4g+3]
//   B (16 x 16, rows = k, cols = n):      lane holds B[4g .. 4g+3][i]
//   D (16 x 16, rows = points, cols = n): lane holds D[4g .. 4g+3][i]
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <algorithm>

#include "mpde_conv.hpp"

namespace mpde {

constexpr int kWgradBlocks = 1024;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);   // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Neighbour of point (t, x, y) at tap offset (dt, dx, dy); -1 if padded.
__device__ __forceinline__ int nb3(const Grid3& g, int t, int x, int y, int dt, int dx, int dy) {
  int q[3] = {t + dt, x + dx, y + dy};
  const int n[3] = {g.T, g.X, g.Y};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (q[a] < 0 || q[a] >= n[a]) {
      if (!g.per[a]) return -1;
      q[a] = q[a] < 0 ? q[a] + n[a] : q[a] - n[a];
    }
  }
  return (q[0] * g.X + q[1]) * g.Y + q[2];
}

// Y[p][n] = bias[n] + sum_tap sum_k Wt[tap][n][k] * X[p + sign*off(tap)][k]
// (sign = +1: forward conv; sign = -1 with transposed weights: data gradient).
// Outputs: Yf (FP32, pre-activation) and optionally Yb = bf16(relu(Y)).
__global__ void __launch_bounds__(256) k_conv(const int2* __restrict__ tiles, const Grid3* __restrict__ grids,
                                              const unsigned short* __restrict__ X,
                                              const unsigned short* __restrict__ Wt,
                                              const float* __restrict__ bias, int sign, float* __restrict__ Yf,
                                              unsigned short* __restrict__ Yb, int relu) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int2 tl = tiles[blockIdx.x * 4 + wave];          // (sample, first point of a 16-point tile)
  if (tl.x < 0) return;
  const Grid3 g = grids[tl.x];
  const int N = g.T * g.X * g.Y;
  const int i = lane & 15, grp = lane >> 4;
  const int p = tl.y + i;                                  // A-row point of this lane
  int t = 0, x = 0, y = 0;
  if (p < N) { y = p % g.Y; const int r = p / g.Y; x = r % g.X; t = r / g.X; }
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const unsigned short* Xs = X + g.off * 16;
#pragma unroll 3
  for (int tap = 0; tap < 27; ++tap) {
    const int dt = tap / 9 - 1, dx = (tap / 3) % 3 - 1, dy = tap % 3 - 1;
    const int q = (p < N) ? nb3(g, t, x, y, sign * dt, sign * dx, sign * dy) : -1;
    bf16x4 a = {0, 0, 0, 0};
    if (q >= 0) {
      const uint2 v = *reinterpret_cast<const uint2*>(Xs + (long long)q * 16 + 4 * grp);
      a = __builtin_bit_cast(bf16x4, v);
    }
    const uint2 wv = *reinterpret_cast<const uint2*>(Wt + ((long long)tap * 16 + i) * 16 + 4 * grp);
    const bf16x4 b = __builtin_bit_cast(bf16x4, wv);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  // D rows 4*grp .. 4*grp+3 (points), column i (output channel)
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int pp = tl.y + 4 * grp + j;
    if (pp >= N) continue;
    const float v = acc[j] + (bias ? bias[i] : 0.f);
    const long long o = (g.off + pp) * 16 + i;
    if (Yf) Yf[o] = v;
    if (Yb) Yb[o] = f2bf(relu ? fmaxf(v, 0.f) : v);
  }
}

// Weight gradient partials: per 16-point chunk c and tap,
//   dWp[c][tap][n][k] = sum_{p in chunk} dY[p][n] * X[p + off(tap)][k]
// as an MFMA with rows = n (A = dY^T), K = points, cols = k (B = shifted X).
__global__ void __launch_bounds__(256) k_conv_wgrad(const int2* __restrict__ tiles, const Grid3* __restrict__ grids,
                                                    const unsigned short* __restrict__ X,
                                                    const unsigned short* __restrict__ dY, int ntiles,
                                                    float* __restrict__ partial) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = lane & 15, grp = lane >> 4;
  __shared__ float red[4][27][16][17];
  f32x4 acc[27];
#pragma unroll
  for (int k = 0; k < 27; ++k) acc[k] = (f32x4){0.f, 0.f, 0.f, 0.f};
  // grid-stride over 16-point tiles; fixed tile order per wave
  for (int tidx = blockIdx.x * 4 + wave; tidx < ntiles; tidx += gridDim.x * 4) {
    const int2 tl = tiles[tidx];
    if (tl.x < 0) continue;
    const Grid3 g = grids[tl.x];
    const int N = g.T * g.X * g.Y;
    const unsigned short* Xs = X + g.off * 16;
    const unsigned short* Ds = dY + g.off * 16;
    // A[n = i][k = point 4grp+j]: dY[p][i];  B[k = point 4grp+j][col = i]: X[p+off][i]
    bf16x4 a;
    int pts[4], tt[4], xx[4], yy[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int p = tl.y + 4 * grp + j;
      pts[j] = p;
      a[j] = (p < N) ? (short)Ds[(long long)p * 16 + i] : (short)0;
      if (p < N) { yy[j] = p % g.Y; const int r = p / g.Y; xx[j] = r % g.X; tt[j] = r / g.X; }
      else { yy[j] = xx[j] = tt[j] = 0; }
    }
#pragma unroll
    for (int tap = 0; tap < 27; ++tap) {
      const int dt = tap / 9 - 1, dx = (tap / 3) % 3 - 1, dy = tap % 3 - 1;
      bf16x4 b;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int q = pts[j] < N ? nb3(g, tt[j], xx[j], yy[j], dt, dx, dy) : -1;
        b[j] = q >= 0 ? (short)Xs[(long long)q * 16 + i] : (short)0;
      }
      acc[tap] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[tap], 0, 0, 0);
    }
  }
  // reduce the 4 waves of the block in a fixed order, one partial per block
#pragma unroll
  for (int tap = 0; tap < 27; ++tap)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[wave][tap][4 * grp + j][i] = acc[tap][j];
  __syncthreads();
  for (int e = threadIdx.x; e < 27 * 256; e += 256) {
    const int tap = e / 256, n = (e / 16) % 16, k = e % 16;
    partial[(long long)blockIdx.x * 27 * 256 + e] = red[0][tap][n][k] + red[1][tap][n][k] + red[2][tap][n][k] +
                                                   red[3][tap][n][k];
  }
}

// Fixed-order sum of block partials into dW [27][16][16].
__global__ void k_sum_partials(const float* __restrict__ partial, int nblocks, float* __restrict__ dW) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 27 * 256) return;
  float s = 0.f;
  for (int b = 0; b < nblocks; ++b) s += partial[(long long)b * 27 * 256 + e];
  dW[e] = s;
}

// Bias gradient: db[n] = sum over points of dY[p][n] (FP32 input), fixed order.
__global__ void k_bias_grad(const float* __restrict__ dYf, long long npts, float* __restrict__ db) {
  __shared__ float red[256];
  const int n = blockIdx.x;
  float s = 0.f;
  for (long long p = threadIdx.x; p < npts; p += 256) s += dYf[p * 16 + n];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[n] = red[0];
}

// dpre = dout * (pre > 0) (FP32 in and out) and its bf16 copy.
__global__ void k_relu_bwd(const float* __restrict__ dout, const float* __restrict__ pre, long long n,
                           float* __restrict__ dpre, unsigned short* __restrict__ dpre_b) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float v = pre[e] > 0.f ? dout[e] : 0.f;
  if (dpre) dpre[e] = v;
  if (dpre_b) dpre_b[e] = f2bf(v);
}

__global__ void k_to_bf16(const float* __restrict__ a, long long n, unsigned short* __restrict__ b) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) b[e] = f2bf(a[e]);
}

// Adam on FP32 master weights; writes bf16 weights W[tap][n][k] and their
// transpose Wt[tap][k][n] (for the data gradient) when layout == 1.
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const float gg = g[e];
  const float mm = b1 * m[e] + (1.f - b1) * gg;
  const float vv = b2 * v[e] + (1.f - b2) * gg * gg;
  m[e] = mm;
  v[e] = vv;
  w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void k_pack_weights(const float* __restrict__ w, unsigned short* __restrict__ wb,
                               unsigned short* __restrict__ wtb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 27 * 256) return;
  const int tap = e / 256, n = (e / 16) % 16, k = e % 16;
  const unsigned short v = f2bf(w[e]);
  wb[e] = v;
  wtb[tap * 256 + k * 16 + n] = v;
}

// ---------------------------------------------------------------- launchers
void conv_launch(hipStream_t st, int ntiles, const int2* tiles, const Grid3* grids, const unsigned short* X,
                 const unsigned short* Wt, const float* bias, int sign, float* Yf, unsigned short* Yb, int relu) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_conv, dim3((ntiles + 3) / 4), dim3(256), 0, st, tiles, grids, X, Wt, bias, sign, Yf, Yb,
                     relu);
}

void conv_wgrad_launch(hipStream_t st, int ntiles, const int2* tiles, const Grid3* grids, const unsigned short* X,
                       const unsigned short* dY, float* partial, float* dW) {
  if (ntiles <= 0) return;
  const int nblocks = std::min(kWgradBlocks, (ntiles + 3) / 4);
  hipLaunchKernelGGL(k_conv_wgrad, dim3(nblocks), dim3(256), 0, st, tiles, grids, X, dY, ntiles, partial);
  hipLaunchKernelGGL(k_sum_partials, dim3((27 * 256 + 255) / 256), dim3(256), 0, st, partial, nblocks, dW);
}

void bias_grad_launch(hipStream_t st, const float* dYf, long long npts, float* db) {
  hipLaunchKernelGGL(k_bias_grad, dim3(16), dim3(256), 0, st, dYf, npts, db);
}

void relu_bwd_launch(hipStream_t st, const float* dout, const float* pre, long long n, float* dpre,
                     unsigned short* dpre_b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_relu_bwd, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dout, pre, n, dpre, dpre_b);
}

void to_bf16_launch(hipStream_t st, const float* a, long long n, unsigned short* b) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n, b);
}

void adam_launch(hipStream_t st, float* w, const float* g, float* m, float* v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, w, g, m, v, n, lr, b1, b2, eps,
                     c1, c2);
}

void pack_weights_launch(hipStream_t st, const float* w, unsigned short* wb, unsigned short* wtb) {
  hipLaunchKernelGGL(k_pack_weights, dim3((27 * 256 + 255) / 256), dim3(256), 0, st, w, wb, wtb);
}

}  // namespace mpde

// ------------------------------------------------ solver <-> network glue
#include "mpde_internal.hpp"

namespace mpde {

// Network input at one grid level: channel 0 = r / ||r||, channel 1 = the
// plain V-cycle's coarse correction v in Jacobi units, (v / dinv) / ||r||,
// channels 2..K+1 = the level's coefficient fields, rest 0; bf16.
__global__ void __launch_bounds__(256) k_features(const Work* __restrict__ work, const LInst* __restrict__ li, int K,
                                                  const float* __restrict__ r, const float* __restrict__ v,
                                                  const float* __restrict__ dinv, const double* __restrict__ inv_norm,
                                                  const float* __restrict__ coef, unsigned short* __restrict__ X0) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  if (p >= L.N) return;
  const long long g = L.voff + p;
  unsigned short* o = X0 + g * 16;
  const double in = inv_norm[wk.inst];
  o[0] = f2bf((float)((double)r[g] * in));
  o[1] = f2bf((float)((double)v[g] / (double)dinv[g] * in));
  for (int k = 0; k < 14; ++k) o[2 + k] = k < K ? f2bf(coef[L.coff + (long long)k * L.N + p]) : (unsigned short)0;
}

// Learned correction added to the plain one: e = v + D^-1 n ||r||.
__global__ void __launch_bounds__(256) k_net_out(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                 const float* __restrict__ Y, const float* __restrict__ dinv,
                                                 const double* __restrict__ norm, float* __restrict__ e) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  if (p >= L.N) return;
  const long long g = L.voff + p;
  e[g] = (float)((double)e[g] + (double)Y[g * 16] * (double)dinv[g] * norm[wk.inst]);
}

// Unit-residual prediction o = v / ||r|| + D^-1 n (written to o_out).
__global__ void __launch_bounds__(256) k_predict(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                 const float* __restrict__ Y, const float* __restrict__ v,
                                                 const float* __restrict__ dinv, const double* __restrict__ inv_norm,
                                                 float* __restrict__ o_out) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  if (p >= L.N) return;
  const long long g = L.voff + p;
  o_out[g] = (float)((double)v[g] * inv_norm[wk.inst] + (double)Y[g * 16] * (double)dinv[g]);
}

// Energy loss of o for the unit residual rhat = r/||r||,
// loss_b = o^T S o - 2 o^T rhat, and d loss / d n = D^-1 2 (S o - rhat) / B.
__global__ void __launch_bounds__(256) k_energy_grad(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                     const float* __restrict__ o_in, const float* __restrict__ So,
                                                     const float* __restrict__ r, const double* __restrict__ inv_norm,
                                                     const float* __restrict__ dinv, float scale,
                                                     float* __restrict__ dOut, double* __restrict__ partial) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  double val = 0;
  if (p < L.N) {
    const long long g = L.voff + p;
    const double o = o_in[g];
    const double rh = (double)r[g] * inv_norm[wk.inst];
    val = o * (double)So[g] - 2.0 * o * rh;
    if (dOut) {
      float* d = dOut + g * 16;
      d[0] = (float)(2.0 * ((double)So[g] - rh) * (double)dinv[g]) * scale;
      for (int k = 1; k < 16; ++k) d[k] = 0.f;
    }
  }
  __shared__ double red[256];
  red[threadIdx.x] = val;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// Per-instance norm and inverse norm from squared norms (0 for a zero or
// non-finite norm), on the device so the learned correction needs no host
// round trip.
__global__ void k_norms(int B, const double* __restrict__ n2, double* __restrict__ norm,
                        double* __restrict__ inv) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double n = sqrt(fmax(n2[b], 0.0));
  const bool ok = n > 0 && isfinite(n);
  norm[b] = ok ? n : 0.0;
  inv[b] = ok ? 1.0 / n : 0.0;
}

// Residual of the prolonged correction on the finer level of a coarse-grid
// correction, w = S p - rhat with rhat = r / ||b|| (b the coarse right side).
__global__ void __launch_bounds__(256) k_fine_resid(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                    const float* __restrict__ Sp, const float* __restrict__ r,
                                                    const double* __restrict__ inv_norm, float* __restrict__ w) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  if (p >= L.N) return;
  const long long g = L.voff + p;
  w[g] = (float)((double)Sp[g] - (double)r[g] * inv_norm[wk.inst]);
}

// Output gradient of the network for the finer-level energy of a prolonged
// coarse correction: d loss / d o = 2 P^T w, and restriction is
// P^T / 2^k (k halved axes), so with Rw = R w on the coarse level,
// d loss / d n = D^-1 2 * 2^k Rw * scale.
__global__ void __launch_bounds__(256) k_grad_out(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                  const float* __restrict__ Rw, const float* __restrict__ dinv,
                                                  float scale, float* __restrict__ dOut) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  if (p >= L.N) return;
  const long long g = L.voff + p;
  float* d = dOut + g * 16;
  d[0] = (float)(2.0 * (double)(1 << L.ncoarsened) * (double)Rw[g] * (double)dinv[g]) * scale;
  for (int k = 1; k < 16; ++k) d[k] = 0.f;
}

// o = v / ||r|| (the plain correction alone, for the reference loss).
__global__ void __launch_bounds__(256) k_scale_vec(const Work* __restrict__ work, const LInst* __restrict__ li,
                                                   const float* __restrict__ v, const double* __restrict__ inv_norm,
                                                   float* __restrict__ o) {
  const Work wk = work[blockIdx.x];
  const LInst& L = li[wk.inst];
  const int p = wk.start + threadIdx.x;
  if (p >= L.N) return;
  const long long g = L.voff + p;
  o[g] = (float)((double)v[g] * inv_norm[wk.inst]);
}

void features_launch(hipStream_t st, const Work* w, int nb, const LInst* li, int K, const float* r, const float* v,
                     const float* dinv, const double* inv_norm, const float* coef, unsigned short* X0) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_features, dim3(nb), dim3(256), 0, st, w, li, K, r, v, dinv, inv_norm, coef, X0);
}
void net_out_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Y, const float* dinv,
                    const double* norm, float* e) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_net_out, dim3(nb), dim3(256), 0, st, w, li, Y, dinv, norm, e);
}
void predict_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Y, const float* v,
                    const float* dinv, const double* inv_norm, float* o) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_predict, dim3(nb), dim3(256), 0, st, w, li, Y, v, dinv, inv_norm, o);
}
void energy_grad_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* o, const float* So,
                        const float* r, const double* inv_norm, const float* dinv, float scale, float* dOut,
                        double* partial) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_energy_grad, dim3(nb), dim3(256), 0, st, w, li, o, So, r, inv_norm, dinv, scale, dOut,
                     partial);
}
void norms_launch(hipStream_t st, int B, const double* n2, double* norm, double* inv) {
  if (B <= 0) return;
  hipLaunchKernelGGL(k_norms, dim3((B + 255) / 256), dim3(256), 0, st, B, n2, norm, inv);
}
void fine_resid_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Sp, const float* r,
                       const double* inv_norm, float* out) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_fine_resid, dim3(nb), dim3(256), 0, st, w, li, Sp, r, inv_norm, out);
}
void grad_out_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Rw, const float* dinv,
                     float scale, float* dOut) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_grad_out, dim3(nb), dim3(256), 0, st, w, li, Rw, dinv, scale, dOut);
}
void scale_vec_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* v, const double* inv_norm,
                      float* o) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_scale_vec, dim3(nb), dim3(256), 0, st, w, li, v, inv_norm, o);
}

}  // namespace mpde
