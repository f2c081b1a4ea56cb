// Launch wrappers of the solver kernels (defined in mpde_kernels.hip).
#pragma once
#include "mpde_internal.hpp"

namespace mpde {

hipError_t upload_stencils(const double w1[5][5], const double w2[5][5]);

template <typename TA, typename TV, typename TC>
void launch_gamma(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TV* u,
                  const TC* c, const TC* f, int sigma, TV* gam);
template <typename TA, typename TV, typename TC>
void launch_gather(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TV* u,
                   const TV* gam, const TC* c, const TC* bw, int sigma, int mode, TV* out, const TV* bvec,
                   TV* x, TV* r, TV* d, const TV* dinv, int cheb_step, double* partial);
template <typename TV, typename TC>
void launch_diag(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c, TV* dinv);
template <typename TV>
void launch_cheb_init(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* b, const TV* dinv, TV* x,
                      TV* r, TV* d);
template <typename TV>
void launch_restrict(int D, hipStream_t st, const Work* w, int nb, const LInst* lf, const LInst* lc, const TV* rf,
                     TV* rc, const TV* dinv = nullptr, TV* xc = nullptr, TV* r0 = nullptr, TV* d0 = nullptr);
template <typename TV>
void launch_prolong_add(int D, hipStream_t st, const Work* w, int nb, const LInst* lf, const LInst* lc,
                        const TV* ec, TV* xf);
template <typename TC>
void launch_coarsen_coef(int D, hipStream_t st, const Work* w, int nb, const LInst* lf, const LInst* lc, int K,
                         const TC* cf, TC* cc);
void launch_set_unit(hipStream_t st, const LInst* probe, const int* col, int nprobe, double* U);
void launch_gauss_jordan(hipStream_t st, int nmat, double* A, const long long* off, const int* n, int* fail);
void launch_set_probe(hipStream_t st, const LInst* probe, const int* pc, const int* ps, int nprobe, int ncolor,
                      double* U);
void launch_extract_probe(hipStream_t st, const Work* w, int nb, const LInst* probe, const int* pc, const int* ps,
                          const long long* dout, int ncolor, const double* Y, double* S);
// One probed instance of the coarsest-level probing (see k_probe_lists).
struct ProbeSrc {
  int b;             // instance
  int plane, n;      // points per time plane, points of its coarsest level
  int tpp, toff;     // fused-operator tiles per probe and their origins in torg
  long long yoff;    // first probe vector
  long long boff;    // band storage
  long long pstart, wstart, tstart;   // first probe, work item and tile index
};
struct FTile;
// Probe descriptors, work items and (tiles != null) fused-operator tiles of
// all probes, from nsrc sources and the coarsest-level descriptors lc.
void launch_probe_lists(hipStream_t st, const LInst* lc, const ProbeSrc* src, int nsrc, long long nvq, long long nwk,
                        long long ntile, const int2* torg, LInst* vq, int* pc, int* ps, long long* bo, Work* wk,
                        FTile* tiles);
void launch_extract_band(hipStream_t st, const Work* w, int nb, const LInst* probe, const int* pc, const int* ps,
                         const long long* bout, int ncolor, const double* Y, double* Lb);
void launch_bb_factor(hipStream_t st, int nmat, double* Lb, const long long* boff, const int* T, const int* m,
                      int* fail);
template <typename TV>
void launch_bb_solve(hipStream_t st, int ninst, const int* inst_list, const LInst* li, const TV* Lb, const TV* b,
                     TV* x);
template <typename TV>
void launch_bb_solve16(hipStream_t st, int ninst, const int* inst_list, const LInst* li, const TV* Lb, const TV* b,
                       TV* x);
template <typename TV>
void launch_bb_solve64(hipStream_t st, int ninst, const int* inst_list, const LInst* li, const TV* Lb, const TV* b,
                       TV* x);
void launch_band_chol(hipStream_t st, int nmat, double* A, const long long* off, const int* n, const int* bw,
                      int* fail);
void launch_band_inverse(hipStream_t st, int nblocks, const double* L, double* X, const long long* off,
                         const int* n, const int* bw, const int* mat_of_block, const int* col0_of_block);
template <typename TV>
void launch_convert_dense(hipStream_t st, const double* src, TV* dst, long long n);
template <typename TV>
void launch_dense_apply(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* Sinv, const TV* r, TV* e);
template <typename TA, typename TV>
void launch_dot(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* a, const TV* b, double* partial);
void launch_finish_sum(hipStream_t st, const double* partial, const int* bstart, int B, double* out);
// Per-instance sum of the block partials into out, then the pcg_scalars
// update op (0: beta and rz from r.z, 1: alpha from p.q, 2: convergence
// test of ||r||^2) from that sum, in one launch.
void launch_finish_scalars(hipStream_t st, const double* partial, const int* bstart, int B, double* out, int op,
                           int first, const double* tol2, double* rz, double* beta, double* alpha,
                           const double* r0n2, int* active, int* iters);
// (tol2: per-instance squared relative tolerance of the inner solve, device)
void launch_pcg_scalars(hipStream_t st, int op, int B, int first, const double* tol2, double* rz_new, double* rz,
                        double* beta, double* pq, double* alpha, double* rn2, double* r0n2, int* active,
                        int* iters);
// p = z + beta p, q = (r - rv) + beta q (= S p when rv = r - S z), and the
// per-block partial sums of p.q.
template <typename TV>
void launch_update_pq(hipStream_t st, const Work* w, int nb, const LInst* li, const double* beta, const TV* z,
                      const TV* r, const TV* rv, TV* p, TV* q, double* partial);
template <typename TV>
void launch_update_p(hipStream_t st, const Work* w, int nb, const LInst* li, const double* beta, const TV* z,
                     TV* p);
template <typename TV>
void launch_update_xr(hipStream_t st, const Work* w, int nb, const LInst* li, const double* alpha, const TV* p,
                      const TV* q, TV* x, TV* r, double* partial, const TV* dinv = nullptr, TV* z0 = nullptr,
                      TV* r0 = nullptr, TV* d0 = nullptr);
template <typename TS, typename TD>
void launch_copy_scale(hipStream_t st, const Work* w, int nb, const LInst* li, const TS* s, TD* d,
                       const double* scale, int add);
template <typename TV>
void launch_fill(hipStream_t st, const Work* w, int nb, const LInst* li, TV* d, double v);
template <typename TC>
void launch_atd_norm(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                     const TC* f, const TC* bw, double* partial);
template <typename TC, typename TO>
void launch_output(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const double* u,
                   const TC* c, const TC* f, TO* z, const long long* zoff);
template <typename TC, typename TG>
void launch_adj_local(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                      const TG* gz, const long long* zoff, double* vloc);
template <typename TC, typename TG>
void launch_adj_rhs(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                    const TG* gz, const long long* zoff, const double* vloc, double* ghat);
template <typename TC, typename TG>
void launch_adj_grad(int D, hipStream_t st, const Work* w, int nb, const LInst* li, CIdx ci, const TC* c,
                     const TC* f, const double* ustar, const double* du, const TG* gz, const long long* zoff,
                     TG* gc, TG* gf, TG* gw);
template <typename T>
void launch_nonfinite(hipStream_t st, const T* a, long long n, int* flag);
template <typename TV>
void launch_hash_fill(hipStream_t st, const Work* w, int nb, const LInst* li, TV* v, unsigned seed);
template <typename TV>
void launch_mul_dinv(hipStream_t st, const Work* w, int nb, const LInst* li, const TV* dinv, const TV* y, TV* v,
                     double* partial);

}  // namespace mpde
