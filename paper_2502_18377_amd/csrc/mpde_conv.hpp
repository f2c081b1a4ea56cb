// Launch wrappers of the BF16 MFMA convolution kernels (mpde_conv.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace mpde {

// One sample grid of a convolution batch (channels last, 16 channels).
struct Grid3 {
  int T, X, Y;        // points per axis
  int per[3];         // periodic axes
  long long off;      // point offset of this sample in the batch arrays
};

void conv_launch(hipStream_t st, int ntiles, const int2* tiles, const Grid3* grids, const unsigned short* X,
                 const unsigned short* Wt, const float* bias, int sign, float* Yf, unsigned short* Yb, int relu);
void conv_wgrad_launch(hipStream_t st, int ntiles, const int2* tiles, const Grid3* grids, const unsigned short* X,
                       const unsigned short* dY, float* partial, float* dW);
void bias_grad_launch(hipStream_t st, const float* dYf, long long npts, float* db);
void relu_bwd_launch(hipStream_t st, const float* dout, const float* pre, long long n, float* dpre,
                     unsigned short* dpre_b);
void to_bf16_launch(hipStream_t st, const float* a, long long n, unsigned short* b);
void adam_launch(hipStream_t st, float* w, const float* g, float* m, float* v, long long n, float lr, float b1,
                 float b2, float eps, float c1, float c2);
void pack_weights_launch(hipStream_t st, const float* w, unsigned short* wb, unsigned short* wtb);

}  // namespace mpde

#include "mpde_internal.hpp"
namespace mpde {
void features_launch(hipStream_t st, const Work* w, int nb, const LInst* li, int K, const float* r, const float* v,
                     const float* dinv, const double* inv_norm, const float* coef, unsigned short* X0);
void net_out_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Y, const float* dinv,
                    const double* norm, float* e);
void predict_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Y, const float* v,
                    const float* dinv, const double* inv_norm, float* o);
void energy_grad_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* o, const float* So,
                        const float* r, const double* inv_norm, const float* dinv, float scale, float* dOut,
                        double* partial);
// norm[b] = sqrt(n2[b]) and inv[b] = 1 / norm[b] (both 0 for a zero or
// non-finite norm), B instances.
void norms_launch(hipStream_t st, int B, const double* n2, double* norm, double* inv);
// w = S p - r / ||b|| on the finer level of a coarse-grid correction.
void fine_resid_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Sp, const float* r,
                       const double* inv_norm, float* out);
// Network output gradient D^-1 2 * 2^k (R w) * scale from the restricted
// finer-level residual R w (k = halved axes of the coarse level).
void grad_out_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* Rw, const float* dinv,
                     float scale, float* dOut);
void scale_vec_launch(hipStream_t st, const Work* w, int nb, const LInst* li, const float* v, const double* inv_norm,
                      float* o);
}  // namespace mpde
