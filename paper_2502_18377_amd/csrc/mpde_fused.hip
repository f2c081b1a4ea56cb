// Fused matrix-free operator for levels with three axes (t, x, y), t not
// periodic: y = A_u^T Pi (A_u u - sigma d) with the epilogues of GatherMode,
// in one pass that evaluates every constraint row once.
//
// The two-pass kernels (k_gamma, k_gather) re-evaluate the rows of each
// neighbour in every point that gathers from it (five times per axis) and
// move gamma through HBM.  Here a block owns an (x, y) tile of one instance
// and marches over the time planes.  At plane p it evaluates, for the tile
// and a halo of two points (four next to a non-periodic edge), the rows of
// all three axes (Eqs. 5-7), the coupling scalar gamma and the projected row
// residuals of the reduced operator (the header of mpde_internal.hpp gives
// the formulation).  Then:
//   * the projected x and y rows go to LDS; after a barrier each tile point
//     gathers the rows whose stencils contain it;
//   * the projected time rows are scattered into a per-thread register ring
//     of partial results for the planes p-4 .. p+4 (the thread owns the same
//     (x, y) point on every plane, so no other thread touches that ring);
//   * plane p-2 then has every contribution (rows at most two planes above
//     it reach it, except the one-sided rows of the last five planes, which
//     are finished after the last plane) and its epilogue runs.
// u is staged plane by plane in LDS (double-buffered, the next plane loaded
// into registers while the current one is processed), and the time window
// of every owned point is a register ring, so each value of u, of the
// coefficients and of the mode vectors crosses HBM once per tile.
#include "mpde_fused.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <type_traits>

namespace mpde {

// Compile-time 5-point weights for a window position known at compile time:
// derivatives at 0 of the Lagrange basis polynomials on the nodes m - wp,
// m = 0..4 (the same moment conditions of Eq. 5 that the host table solves;
// here in closed form so that the weights become instruction literals).
__host__ __device__ constexpr double lag_d1(int wp, int k) {
  double den = 1, s = 0;
  for (int m = 0; m < 5; ++m)
    if (m != k) den *= (double)(k - m);
  for (int j = 0; j < 5; ++j) {
    if (j == k) continue;
    double pr = 1;
    for (int m = 0; m < 5; ++m)
      if (m != k && m != j) pr *= -(double)(m - wp);
    s += pr;
  }
  return s / den;
}
__host__ __device__ constexpr double lag_d2(int wp, int k) {
  double den = 1, s = 0;
  for (int m = 0; m < 5; ++m)
    if (m != k) den *= (double)(k - m);
  for (int j = 0; j < 5; ++j) {
    if (j == k) continue;
    for (int l = 0; l < 5; ++l) {
      if (l == k || l == j) continue;
      double pr = 1;
      for (int m = 0; m < 5; ++m)
        if (m != k && m != j && m != l) pr *= -(double)(m - wp);
      s += pr;
    }
  }
  return s / den;
}
template <typename TA, int WP, int K> __device__ __forceinline__ constexpr TA CW1() { return (TA)lag_d1(WP, K); }
template <typename TA, int WP, int K> __device__ __forceinline__ constexpr TA CW2() { return (TA)lag_d2(WP, K); }
static_assert(lag_d1(2, 0) * 12 == 1 && lag_d1(2, 1) * 12 == -8 && lag_d1(2, 3) * 12 == 8, "5-point weights");
static_assert(lag_d2(2, 2) * 12 == -30 && lag_d2(0, 0) * 12 == 35 && lag_d1(0, 0) * 12 == -25, "5-point weights");

constexpr int kFMaxU = 2;   // staged u values per thread and plane

__device__ __forceinline__ int fwrap(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

__device__ __forceinline__ float fm(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fm(double a, double b, double c) { return fma(a, b, c); }
// gamma = num / kappa with kappa >= 1: in FP32 the hardware reciprocal
// (1 ulp) is accurate to rounding; FP64 divides exactly.
__device__ __forceinline__ float fdivk(float n, float k) { return n * __builtin_amdgcn_rcpf(k); }
__device__ __forceinline__ double fdivk(double n, double k) { return n / k; }

// Raw buffer access: the resource (base, size) and the uniform byte offset
// live in scalar registers, the per-thread byte offset in one vector
// register, so a load costs no vector address arithmetic.
using brsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int fu2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ brsrc mkbuf(const void* p, long long bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T bld(brsrc r, unsigned voff, unsigned soff);
template <> __device__ __forceinline__ float bld<float>(brsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0));
}
template <> __device__ __forceinline__ double bld<double>(brsrc r, unsigned voff, unsigned soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0));
}
__device__ __forceinline__ void bst(brsrc r, unsigned voff, unsigned soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)voff, (int)soff, 0);
}
__device__ __forceinline__ void bst(brsrc r, unsigned voff, unsigned soff, double v) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(fu2, v), r, (int)voff, (int)soff, 0);
}
// A per-thread offset past the end of every buffer the kernel uses (their
// sizes are below 2^31 bytes, checked by the host, and offset + plane offset
// stays below 2^32): the buffer range check returns 0 for such a load and
// drops such a store.  Lanes whose result must not be written use it, so
// that every memory instruction of the plane loop is issued unconditionally
// and the compiler's wait counts stay exact across loop iterations.
constexpr unsigned kOOB = 0x80000000u;

// One staged row-value slot (C1, C2, T+, T-) in the arithmetic type.
struct __align__(16) FSlotD {
  double x, y, z, w;
};
template <typename TA> struct FSlot;
template <> struct FSlot<float> {
  using type = float4;
  static __device__ __forceinline__ float4 make(float a, float b, float c, float d) { return make_float4(a, b, c, d); }
};
template <> struct FSlot<double> {
  using type = FSlotD;
  static __device__ __forceinline__ FSlotD make(double a, double b, double c, double d) { return FSlotD{a, b, c, d}; }
};

// Per-axis constant FK_* of the fused operator: the host's FP32 copy, or
// the same quantity formed in FP64 from the FP64 level data.
template <typename TA> __device__ __forceinline__ TA fkc(const LInst& L, int a, int i);
template <> __device__ __forceinline__ float fkc<float>(const LInst& L, int a, int i) { return L.fk[a][i]; }
template <> __device__ __forceinline__ double fkc<double>(const LInst& L, int a, int i) {
  switch (i) {
    case FK_A: return L.wT[a] * L.wT[a];
    case FK_AH: return 0.5 * L.wT[a] * L.wT[a];
    case FK_B1: return L.wC1[a] * L.wC1[a];
    case FK_B2: return L.wC2[a] * L.wC2[a];
    case FK_S1: return L.is1[a];
    case FK_S2: return L.is2[a];
    case FK_G0: return L.gi[a][0][0];
    case FK_G0 + 1: return L.gi[a][0][2];
    case FK_B1D: return L.wC1[a] * L.wC1[a] / 12.0;
    case FK_B2D: return L.wC2[a] * L.wC2[a] / 12.0;
    default: return i < FK_G2 ? L.gi[a][1][i - FK_G1] : L.gi[a][2][i - FK_G2];
  }
}

// Difference sums of the time window w[0..4] of a point at window position WP.
template <typename TA, int WP>
__device__ __forceinline__ void t_sums(const TA* w, TA& s1, TA& s2) {
  s1 = CW1<TA, WP, 0>() * w[0] + CW1<TA, WP, 1>() * w[1] + CW1<TA, WP, 2>() * w[2] + CW1<TA, WP, 3>() * w[3] +
       CW1<TA, WP, 4>() * w[4];
  s2 = CW2<TA, WP, 0>() * w[0] + CW2<TA, WP, 1>() * w[1] + CW2<TA, WP, 2>() * w[2] + CW2<TA, WP, 3>() * w[3] +
       CW2<TA, WP, 4>() * w[4];
}
// Scatter of a time row's projected difference residuals (already weighted
// by wC1^2, wC2^2) into the partial results of the planes of its window:
// one FMA per non-zero weight.
template <typename TA, int WP, int K>
__device__ __forceinline__ void t_push1(TA& a, TA q1, TA q2) {
  constexpr TA w1 = (TA)lag_d1(WP, K), w2 = (TA)lag_d2(WP, K);
  if (w1 != (TA)0) a = fm(-w1, q1, a);
  if (w2 != (TA)0) a = fm(-w2, q2, a);
}
template <typename TA, int WP>
__device__ __forceinline__ void t_push(TA* acc, TA q1, TA q2) {
  t_push1<TA, WP, 0>(acc[4 - WP], q1, q2);
  t_push1<TA, WP, 1>(acc[5 - WP], q1, q2);
  t_push1<TA, WP, 2>(acc[6 - WP], q1, q2);
  t_push1<TA, WP, 3>(acc[7 - WP], q1, q2);
  t_push1<TA, WP, 4>(acc[8 - WP], q1, q2);
}

// Rows of one axis at a point, before weighting: the 5-point difference
// sums s1 = k c1, s2 = k c2 of its window, its Taylor differences
// dp = u_i - u_{i+1}, dm = u_i - u_{i-1} (0 for a missing one-sided row),
// and the right sides of the axis' normal equations for its derivative
// unknowns (x1, x2):
//   b1 = wT^2 (dp - dm) - wC1^2 s1,   b2 = wT^2 (dp + dm) / 2 - wC2^2 s2.
template <typename TA>
struct ARows {
  TA c1, c2, dp, dm, b1, b2;
};
// Window centred on the point (position 2): the weights are
// (1, -8, 0, 8, -1) / 12 and (-1, 16, -30, 16, -1) / 12, so c1 = 12 s1 and
// c2 = 12 s2 are formed from shared sums and differences, and the factor
// 1/12 is folded into B1d = wC1^2 / 12, B2d = wC2^2 / 12.
template <typename TA>
__device__ __forceinline__ ARows<TA> crows(TA wm2, TA wm1, TA ui, TA wp1, TA wp2, TA A, TA Ah, TA B1d, TA B2d) {
  ARows<TA> r;
  const TA d31 = wp1 - wm1, s13 = wm1 + wp1;
  r.c1 = fm((TA)8, d31, wm2 - wp2);
  r.c2 = fm((TA)-30, ui, fm((TA)16, s13, -(wm2 + wp2)));
  r.dp = ui - wp1;
  r.dm = ui - wm1;
  r.b1 = -fm(A, d31, B1d * r.c1);                      // dp - dm = u_{i-1} - u_{i+1}
  r.b2 = fm(Ah, fm((TA)2, ui, -s13), -(B2d * r.c2));   // dp + dm = 2 u_i - u_{i-1} - u_{i+1}
  return r;
}
// Window at position WP on the (non-periodic) time axis: plain sums (k = 1).
template <typename TA, int WP>
__device__ __forceinline__ ARows<TA> wrows(const TA* w, TA A, TA Ah, TA B1, TA B2) {
  ARows<TA> r;
  t_sums<TA, WP>(w, r.c1, r.c2);
  r.dp = WP != 4 ? w[WP] - w[WP != 4 ? WP + 1 : WP] : (TA)0;
  r.dm = WP != 0 ? w[WP] - w[WP != 0 ? WP - 1 : WP] : (TA)0;
  r.b1 = A * (r.dp - r.dm) - B1 * r.c1;
  r.b2 = Ah * (r.dp + r.dm) - B2 * r.c2;
  return r;
}

// Rows of a periodic axis (x or y) from the staged u plane; `w0` is the LDS
// address of the window start (the point itself is at w0 + 2 sd), `sd` the
// LDS stride along the axis.
template <typename TA>
__device__ __forceinline__ ARows<TA> xy_rows(const TA* su, int w0, int sd, TA ui, TA A, TA Ah, TA B1d, TA B2d) {
  return crows<TA>(su[w0], su[w0 + sd], ui, su[w0 + 3 * sd], su[w0 + 4 * sd], A, Ah, B1d, B2d);
}

// Gather of the projected rows of a periodic axis staged in LDS into the
// result at a tile point.  Each slot holds the four projected row residuals
// of one point before weighting, (C1, C2, T+, T-); the gather weights them
// by A = wT^2 (Taylor rows) and wC1^2, wC2^2 (difference rows, passed as
// B1d = wC1^2 / 12, B2d = wC2^2 / 12 against the 12-scaled centred
// weights).  `a` is the point's slot, `sd` the slot stride along the axis.
// Row j + o contains j at window slot 2 - o; T+ of j - 1 and T- of j + 1 end
// at j.
template <typename TA, typename S>
__device__ __forceinline__ TA xy_gather(const S* q, int a, int sd, TA A, TA B1d, TA B2d) {
  const S m2 = q[a - 2 * sd], m1 = q[a - sd], z = q[a], p1 = q[a + sd], p2 = q[a + 2 * sd];
  const TA t = (z.z + z.w) - (m1.z + p1.w);
  const TA c1 = fm((TA)8, m1.x - p1.x, p2.x - m2.x);                          // window slots 4, 3, 1, 0
  const TA c2 = fm((TA)-30, z.y, fm((TA)16, m1.y + p1.y, -(m2.y + p2.y)));
  return fm(A, t, -fm(B1d, c1, B2d * c2));
}

// Block sum (result in thread 0) for blocks of at most NTH threads.
template <int NTH>
__device__ __forceinline__ double fblock_sum(double v) {
  __shared__ double part[NTH / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) part[wid] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NTH / 64; ++w)
      if (w < (int)(blockDim.x >> 6)) s += part[w];
  }
  return s;
}

// SIG: y = A_u^T Pi (A_u u - d) with the right-hand-side terms of the
// source `fsrc` (equation rows) and the boundary values `wsrc` (boundary
// rows), both level-0 point fields.
template <typename TA, typename TV, typename TC, int MODE, int NT, bool SIG>
__global__ void __launch_bounds__(fthreads<TA>()) k_apply3(const FTile* __restrict__ tiles, FGeom g,
                                                      const LInst* __restrict__ li, CIdx ci,
                                                      const TV* __restrict__ u, const TC* __restrict__ c,
                                                      TV* __restrict__ out, const TV* __restrict__ bvec,
                                                      TV* __restrict__ xv, TV* __restrict__ rv,
                                                      TV* __restrict__ dv, const TV* __restrict__ dinv,
                                                      int cheb_step, double* __restrict__ partial,
                                                      const TC* __restrict__ fsrc, const TC* __restrict__ wsrc) {
  static_assert(std::is_same<TC, float>::value && std::is_same<TA, TV>::value, "FP32 coefficients, TA vectors");
  constexpr int NQ = kFMaxQ;
  constexpr int NTH = fthreads<TA>();   // largest block; a launch uses g.nthr <= NTH threads
  const int nthr = g.nthr;
  constexpr unsigned VB = sizeof(TV);   // bytes of a vector element
  using S4 = typename FSlot<TA>::type;
  extern __shared__ __align__(16) unsigned char fsm[];
  TA* su = reinterpret_cast<TA*>(fsm);     // [kFRing][uplane] staged u planes, plane p in slot p % kFRing
  S4* sq = reinterpret_cast<S4*>(su + kFRing * g.uplane);   // [2][2][qplane] projected x, y rows
  const FTile tl = tiles[blockIdx.x];
  const LInst& L = li[tl.inst];
  if (gated_off(L)) return;   // converged instance (Krylov iterations only)
  // NT > 0: every instance of the launch has NT time planes (a compile-time
  // trip count: the plane loop is unrolled completely and no prefetched
  // value is carried around a loop)
  const int nt = NT > 0 ? NT : L.n[0], nx = L.n[1], ny = L.n[2];
  // Time chunks (gridDim.y > 1): block (tile, c) writes the output planes
  // [t0, t1) and evaluates the rows of planes r0 .. (its last output) + 2.
  // Away from the time boundary a row of plane r reaches the outputs
  // r - 2 .. r + 2, and the rows of the first and last two planes reach five
  // planes in, so chunk edges in [5, nt - 5] need two halo row planes on
  // each side and nothing else (the host checks the edges; tc is even, so
  // every chunk starts on an even plane).
  // (the dot-product pass is never chunked: one partial-sum slot per tile)
  const int nch = MODE == G_STORE_DOT ? 1 : (int)gridDim.y, ch = MODE == G_STORE_DOT ? 0 : (int)blockIdx.y;
  const int t0 = ch * g.tc, t1 = ch == nch - 1 ? nt : t0 + g.tc;
  const int r0 = ch == 0 ? 0 : t0 - 2;
  const int tf = t1 < nt - 5 ? t1 : nt - 5;   // outputs below tf are finished in the plane loop
  const FSpan X = fspan(tl.x0, g.TX, nx, 1);
  const FSpan Y = fspan(tl.y0, g.TY, ny, 1);
  const int stt = L.str[0], stx = L.str[1], sty = L.str[2];   // an instance level has < 2^31 points
  const int tid = threadIdx.x;
  const int npts = X.qn * Y.qn;

  // ---- the row points owned by this thread (the same (x, y) on every plane):
  // q-point tid + s * nthr, s < NQ
  bool act[NQ], tile[NQ];
  int ad[NQ], axw[NQ], ayw[NQ], qsl[NQ], qdx[NQ], qdy[NQ];
  unsigned go[NQ];   // byte offset of the point's coefficient within a plane (0 if none)
  unsigned gt[NQ];   // byte offset of its vector element for tile points, kOOB for halo points
#pragma unroll
  for (int s = 0; s < NQ; ++s) {
    const int qi = tid + s * nthr;
    act[s] = qi < npts;
    const int lx = act[s] ? qi / Y.qn : 0, ly = act[s] ? qi - lx * Y.qn : 0;
    const int gx = fwrap(X.qlo + lx, nx), gy = fwrap(Y.qlo + ly, ny);
    go[s] = act[s] ? 4u * (unsigned)(gx * stx + gy * sty) : 0u;
    // staged u: the point sits at (lx + 2, ly + 2); its windows start 2 before
    ad[s] = (lx + 2) * Y.un + (ly + 2);
    axw[s] = lx * Y.un + (ly + 2);
    ayw[s] = (lx + 2) * Y.un + ly;
    const int sx = lx + X.qoff, sy = ly + Y.qoff;
    qsl[s] = sx * Y.qs + sy;
    qdx[s] = qdy[s] = -1;   // wrapped copies of a whole-axis tile
    if (X.fw) {
      if (lx < 2) qdx[s] = (sx + nx) * Y.qs + sy;
      else if (lx >= nx - 2) qdx[s] = (sx - nx) * Y.qs + sy;
    }
    if (Y.fw) {
      if (ly < 2) qdy[s] = qsl[s] + ny;
      else if (ly >= ny - 2) qdy[s] = qsl[s] - ny;
    }
    tile[s] = act[s] && (unsigned)(lx - X.ilo) < (unsigned)X.icnt && (unsigned)(ly - Y.ilo) < (unsigned)Y.icnt;
    gt[s] = tile[s] ? go[s] * (VB / 4) : kOOB;
  }

  // Loads are raw buffer loads: a per-thread byte offset fixed over the
  // planes and a uniform plane offset.  Slots without a row point load point
  // 0 and planes past the end load the last plane; both are ignored.
  const unsigned pbytes = 4u * (unsigned)stt;                 // one coefficient plane
  const unsigned vpbytes = VB * (unsigned)stt;                // one plane of a vector
  const brsrc rU = mkbuf(u + L.voff, (long long)VB * L.N);
  const brsrc rC = mkbuf(c + L.coff, 4LL * L.N * ci.K);
  const brsrc rF = mkbuf(SIG ? fsrc + L.voff : nullptr, SIG ? 4LL * L.N : 0);
  const brsrc rW = mkbuf(SIG ? wsrc + L.voff : nullptr, SIG ? 4LL * L.N : 0);
  constexpr int NC = SIG ? 8 : 7;   // per-plane point loads: the coefficient planes (and the source)
  auto psoff = [&](int pl) { return (unsigned)(pl < nt ? pl : nt - 1) * pbytes; };
  auto pvoff = [&](int pl) { return (unsigned)(pl < nt ? pl : nt - 1) * vpbytes; };
  // coefficient plane offsets (bytes) of c_phi and of the first / second
  // derivative of each axis; a missing field loads plane 0 and is zeroed by
  // its scale factor below
  unsigned cko[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) cko[k] = ci.k[k] >= 0 ? 4u * (unsigned)ci.k[k] * (unsigned)L.N : 0u;

  // ---- partial results over the time axis: a register ring of length 10,
  // shifted by two planes after every odd plane; on an even plane p,
  // acc[s][k] holds plane p - 4 + k of point s, on an odd plane the same
  // entries sit one slot higher.  The time windows of u are read from the
  // staged planes (the ring keeps planes p - 4 .. p + 5).
  TA acc[NQ][10];
#pragma unroll
  for (int s = 0; s < NQ; ++s)
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[s][k] = 0;
  auto slot = [&](int pl) { return (pl % kFRing) * g.uplane; };
  // staged-u slot -> byte offset within a plane (fixed over the planes)
  const int nus = X.un * Y.un;
  // (slots past the region load point 0 and are written to the spare slot
  // at the end of the staged plane, which nothing reads)
  unsigned uof[kFMaxU];
  int uslot[kFMaxU];
#pragma unroll
  for (int k = 0; k < kFMaxU; ++k) {
    const int i = tid + k * nthr;
    uof[k] = 0;
    uslot[k] = g.uplane - 1;
    if (i < nus) {
      const int ux = i / Y.un, uy = i - ux * Y.un;
      uof[k] = VB * (unsigned)(fwrap(X.ulo + ux, nx) * stx + fwrap(Y.ulo + uy, ny) * sty);
      uslot[k] = i;
    }
  }

  // Loads run two planes ahead of their use, into register sets indexed by
  // plane parity; the plane loop is unrolled by two so that every set has a
  // fixed register name (a register copy would wait for the load):
  //   cs[q]  coefficients of the next plane of parity q to be processed,
  //   us[q]  u of the next plane of parity q to be staged in LDS.
  TC cs[2][NQ][NC];
  TV us[2][kFMaxU];
  auto ld_coef = [&](int pl, TC(&d)[NQ][NC]) {
    const unsigned po = psoff(pl);
#pragma unroll
    for (int s = 0; s < NQ; ++s) {
#pragma unroll
      for (int k = 0; k < 7; ++k) d[s][k] = bld<TC>(rC, go[s], cko[k] + po);
      if (SIG) d[s][NC - 1] = bld<TC>(rF, go[s], po);
    }
  };
  auto ld_u = [&](int pl, TV(&d)[kFMaxU]) {
    const unsigned po = pvoff(pl);
#pragma unroll
    for (int k = 0; k < kFMaxU; ++k) d[k] = bld<TV>(rU, uof[k], po);
  };
  // planes r0 - 2 .. r0 + 4 staged before the loop; plane p + 5 is staged at
  // plane p
  for (int pl = r0 > 0 ? r0 - 2 : 0; pl < r0 + 5; ++pl) {
    const unsigned po = pvoff(pl);
#pragma unroll
    for (int k = 0; k < kFMaxU; ++k) su[slot(pl) + uslot[k]] = bld<TV>(rU, uof[k], po);
  }
  ld_coef(r0, cs[0]);
  ld_coef(r0 + 1, cs[1]);
  ld_u(r0 + 5, us[0]);
  ld_u(r0 + 6, us[1]);
  __syncthreads();

  // Per-axis constants (uniform; FP32 copies made by the host): squared row
  // weights, coefficient scales (0 for a field the equation lacks) and the
  // diagonal Gram inverses of two-sided rows (x and y are periodic, so all of
  // their rows are two-sided).
  auto kt = [&](int i) { return fkc<TA>(L, 0, i); };
  auto kx = [&](int i) { return fkc<TA>(L, 1, i); };
  auto ky = [&](int i) { return fkc<TA>(L, 2, i); };
  const TA At = kt(FK_A), Aht = kt(FK_AH), B1t = kt(FK_B1), B2t = kt(FK_B2), B1dt = kt(FK_B1D), B2dt = kt(FK_B2D);
  const TA Ax = kx(FK_A), Ahx = kx(FK_AH), B1dx = kx(FK_B1D), B2dx = kx(FK_B2D);
  const TA Ay = ky(FK_A), Ahy = ky(FK_AH), B1dy = ky(FK_B1D), B2dy = ky(FK_B2D);
  auto has = [&](int k) { return ci.k[k] >= 0 ? (TA)1 : (TA)0; };
  const TA m0 = has(0);
  const TA s1t = kt(FK_S1) * has(1), s2t = kt(FK_S2) * has(2), s1x = kx(FK_S1) * has(3);
  const TA s2x = kx(FK_S2) * has(4), s1y = ky(FK_S1) * has(5), s2y = ky(FK_S2) * has(6);
  const TA gx1 = kx(FK_G0), gx2 = kx(FK_G0 + 1), gy1 = ky(FK_G0), gy2 = ky(FK_G0 + 1);

  // Chebyshev coefficients of this step (uniform)
  TA chA = 0, chB = 0;
  if (MODE == G_CHEB) {
    const double th = L.cheb_theta, de = L.cheb_delta, s1 = th / de;
    double rp = 1.0 / s1, rn = 0;
    for (int s = 0; s <= cheb_step; ++s) { rn = 1.0 / (2.0 * s1 - rp); if (s < cheb_step) rp = rn; }
    chA = (TA)(rn * rp);
    chB = (TA)(2.0 * rn / de);
  }
  const TA ith = (TA)(1.0 / L.cheb_theta);
  TA dot = 0;   // per-thread u.y over at most a few dozen planes; the block sum is FP64

  // Epilogue inputs of plane j (x, r, dinv for a Chebyshev step; b, dinv for
  // a residual), loaded one plane before the epilogue runs.
  const long long vb = (long long)VB * L.N;
  const brsrc rOut = mkbuf(out ? out + L.voff : nullptr, out ? vb : 0);
  const brsrc rB = mkbuf(bvec ? bvec + L.voff : nullptr, bvec ? vb : 0);
  const brsrc rX = mkbuf(xv ? xv + L.voff : nullptr, xv ? vb : 0);
  const brsrc rR = mkbuf(rv ? rv + L.voff : nullptr, rv ? vb : 0);
  const brsrc rD = mkbuf(dv ? dv + L.voff : nullptr, dv ? vb : 0);
  const brsrc rDi = mkbuf(dinv ? dinv + L.voff : nullptr, dinv ? vb : 0);
  auto ld_epi = [&](int j, unsigned o, TV(&e)[3]) {
    const unsigned pj = (unsigned)j * vpbytes;
    e[0] = e[1] = e[2] = 0;
    if (MODE == G_RESID) {
      if (bvec) e[0] = bld<TV>(rB, o, pj);
      if (dv) e[2] = bld<TV>(rDi, o, pj);
    } else if (MODE == G_CHEB) {
      e[0] = bld<TV>(rX, o, pj);
      e[1] = bld<TV>(rR, o, pj);
      e[2] = bld<TV>(rDi, o, pj);
    }
  };
  auto finalize = [&](int j, unsigned o, TA y, TA uj, const TV(&e)[3]) {
    const unsigned pj = (unsigned)j * vpbytes;
    if (MODE == G_STORE) {
      bst(rOut, o, pj, y);
    } else if (MODE == G_STORE_DOT) {
      bst(rOut, o, pj, y);
      if (o != kOOB) dot += uj * y;
    } else if (MODE == G_RESID) {
      const TA r = e[0] - y;
      bst(rOut, o, pj, r);
      if (dv) bst(rD, o, pj, e[2] * r * ith);
    } else {   // G_CHEB
      bst(rX, o, pj, e[0] + uj);
      const TA r = e[1] - y;
      bst(rR, o, pj, r);
      bst(rD, o, pj, chA * uj + chB * e[2] * r);
    }
  };
  TV es[2][NQ][3];                   // epilogue inputs by plane parity
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int s = 0; s < NQ; ++s) es[q][s][0] = es[q][s][1] = es[q][s][2] = 0;

  // One plane.  Phase A evaluates the rows at plane p (staged u slot p & 1)
  // and stores the projected x and y rows in row buffer p & 1, then stages
  // plane p + 1; after the single barrier, phase B gathers plane p.  Buffers
  // alternate, so the next phase A (which writes the other buffers) needs no
  // second barrier: everything it overwrites was last read before this one.
  // WP is the window position of plane p on the time axis (0, 1 on the
  // first two planes, 3, 4 on the last two, 2 elsewhere), a template
  // constant so that every ring index is fixed at compile time.
  auto step = [&](int p, auto par, auto wpc) __attribute__((always_inline)) {
    constexpr int Q = decltype(par)::value;   // p & 1, also the ring offset
    constexpr int WP = decltype(wpc)::value;
    constexpr int tpt = WP != 4, tmt = WP != 0;
    constexpr int clt = tmt ? (tpt ? 0 : 2) : 1;
    const TA* cu = su + slot(p);
    TA* nu = su + slot(p + 5);
    const int tw0 = slot(p - WP), tw1 = slot(p - WP + 1), tw2 = slot(p - WP + 2), tw3 = slot(p - WP + 3),
              tw4 = slot(p - WP + 4);
    S4* qx = sq + Q * 2 * g.qplane;
    S4* qy = qx + g.qplane;
    // Gram inverse of this plane's time rows (one-sided on the first and
    // last plane)
    TA gt11, gt12 = 0, gt22;
    if (clt == 0) {
      gt11 = kt(FK_G0);
      gt22 = kt(FK_G0 + 1);
    } else {
      constexpr int gk = clt == 1 ? FK_G1 : FK_G2;
      gt11 = kt(gk);
      gt12 = kt(gk + 1);
      gt22 = kt(gk + 2);
    }
    const bool onB = (L.dlo[0] && p == 0) || (L.dhi[0] && p == nt - 1);

#pragma unroll
    for (int s = 0; s < NQ; ++s) {
      if (!act[s]) continue;
      TA* const ra = acc[s] + Q;
      const TC* cc = cs[Q][s];
      // time window of the point (planes p - WP .. p - WP + 4)
      const TA w[5] = {su[tw0 + ad[s]], su[tw1 + ad[s]], su[tw2 + ad[s]], su[tw3 + ad[s]], su[tw4 + ad[s]]};
      const TA ui = w[WP];
      // rows of the three axes (Eqs. 5-7) before weighting
      const ARows<TA> rt = WP == 2 ? crows<TA>(w[0], w[1], ui, w[3], w[4], At, Aht, B1dt, B2dt)
                                   : wrows<TA, WP>(w, At, Aht, B1t, B2t);
      const ARows<TA> rx = xy_rows<TA>(cu, axw[s], Y.un, ui, Ax, Ahx, B1dx, B2dx);
      const ARows<TA> ry = xy_rows<TA>(cu, ayw[s], 1, ui, Ay, Ahy, B1dy, B2dy);
      constexpr TA kt_ = WP == 2 ? (TA)1 / (TA)12 : (TA)1;   // s = k c on the time axis
      constexpr TA kc_ = (TA)1 / (TA)12;                      // x and y windows are centred
      // scaled coefficients of the derivative unknowns in the equation row
      const TA c0 = (TA)cc[0] * m0;
      const TA cat = (TA)cc[1] * s1t, catt = (TA)cc[2] * s2t;
      const TA cax = (TA)cc[3] * s1x, caxx = (TA)cc[4] * s2x;
      const TA cay = (TA)cc[5] * s1y, cayy = (TA)cc[6] * s2y;
      const TA b1t = rt.b1, b2t = rt.b2, b1x = rx.b1, b2x = rx.b2, b1y = ry.b1, b2y = ry.b2;
      // G^-1 b and G^-1 (c_a, c_aa) of each axis
      TA g1t, g2t, h1t, h2t;
      if (clt == 0) {
        g1t = gt11 * b1t;
        g2t = gt22 * b2t;
        h1t = gt11 * cat;
        h2t = gt22 * catt;
      } else {
        g1t = gt11 * b1t + gt12 * b2t;
        g2t = gt12 * b1t + gt22 * b2t;
        h1t = gt11 * cat + gt12 * catt;
        h2t = gt12 * cat + gt22 * catt;
      }
      const TA g1x = gx1 * b1x, g2x = gx2 * b2x, h1x = gx1 * cax, h2x = gx2 * caxx;
      const TA g1y = gy1 * b1y, g2y = gy2 * b2y, h1y = gy1 * cay, h2y = gy2 * cayy;
      // Sherman-Morrison scalar gamma (kappa >= 1)
      const TA kap = (TA)1 + cat * h1t + catt * h2t + cax * h1x + caxx * h2x + cay * h1y + cayy * h2y;
      const TA rhoE = SIG ? c0 * ui - (TA)cc[NC - 1] : c0 * ui;   // equation-row residual
      const TA num = rhoE - (cat * g1t + catt * g2t + cax * g1x + caxx * g2x + cay * g1y + cayy * g2y);
      const TA gam = fdivk(num, kap);
      // eliminated derivative unknowns x = -(G^-1 b + gamma G^-1 c), then the
      // projected rows before weighting: C1 = x1 - s1, C2 = x2 - s2,
      // T+ = dp + x1 + x2 / 2, T- = dm - x1 + x2 / 2
      {
        const TA x1 = -fm(h1x, gam, g1x), x2 = -fm(h2x, gam, g2x);
        const S4 v = FSlot<TA>::make(fm(-kc_, rx.c1, x1), fm(-kc_, rx.c2, x2), fm((TA)0.5, x2, rx.dp) + x1,
                                     fm((TA)0.5, x2, rx.dm) - x1);
        qx[qsl[s]] = v;
        if (qdx[s] >= 0) qx[qdx[s]] = v;
      }
      {
        const TA x1 = -fm(h1y, gam, g1y), x2 = -fm(h2y, gam, g2y);
        const S4 v = FSlot<TA>::make(fm(-kc_, ry.c1, x1), fm(-kc_, ry.c2, x2), fm((TA)0.5, x2, ry.dp) + x1,
                                     fm((TA)0.5, x2, ry.dm) - x1);
        qy[qsl[s]] = v;
        if (qdy[s] >= 0) qy[qdy[s]] = v;
      }
      if (tile[s]) {
        const TA x1 = -fm(h1t, gam, g1t), x2 = -fm(h2t, gam, g2t);
        const TA Q1 = B1t * fm(-kt_, rt.c1, x1), Q2 = B2t * fm(-kt_, rt.c2, x2);
        const TA Tp = tpt ? At * (fm((TA)0.5, x2, rt.dp) + x1) : (TA)0;
        const TA Tm = tmt ? At * (fm((TA)0.5, x2, rt.dm) - x1) : (TA)0;
        TA e = fm(c0, gam, Tp + Tm);                 // equation row (q_E = gamma), own Taylor rows
        if (onB) e += SIG ? ui - (TA)bld<TC>(rW, go[s], psoff(p)) : ui;   // boundary row
        ra[4] += e;
        ra[5] -= Tp;                                   // T+ of plane p ends at p + 1
        ra[3] -= Tm;                                   // T- of plane p ends at p - 1
        t_push<TA, WP>(ra, Q1, Q2);
      }
    }
    // Keep the refills of the parity sets after the last use of their old
    // contents: if the scheduler hoists them, the old and new values overlap,
    // the sets cannot keep one register each across the loop, and the copies
    // inserted at the loop latch wait for every load in flight.
    __builtin_amdgcn_sched_barrier(0);
    ld_coef(p + 2, cs[Q]);
    // stage plane p + 5 (the slot of plane p - 5, which no reader needs any
    // more; planes past the end stage a copy of the last plane, never read)
#pragma unroll
    for (int k = 0; k < kFMaxU; ++k) nu[uslot[k]] = us[Q][k];
    ld_u(p + 7, us[Q]);
    if (WP != 0) {
#pragma unroll
      for (int s = 0; s < NQ; ++s) ld_epi(p - 1 < nt ? p - 1 : nt - 1, gt[s], es[1 - Q][s]);
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NQ; ++s) {
      TA* const ra = acc[s] + Q;
      if (tile[s])
        ra[4] += xy_gather<TA>(qx, qsl[s], Y.qs, Ax, B1dx, B2dx) + xy_gather<TA>(qy, qsl[s], 1, Ay, B1dy, B2dy);
      // plane p - 2 is complete unless it is one of the last five planes
      // (those are written after the last plane)
      if (WP >= 2)
        finalize(p - 2, (p - 2 >= t0 && p - 2 < tf) ? gt[s] : kOOB, ra[2], su[slot(p - 2) + ad[s]], es[Q][s]);
      if (WP == 4) {   // p = nt - 1
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          const int j = p - 4 + k;
          if (j >= 0 && j >= nt - 5 && j >= t0) {
            TV e[3];
            ld_epi(j, gt[s], e);
            finalize(j, gt[s], ra[k], su[slot(j) + ad[s]], e);
          }
        }
      }
    }
    if (Q == 1) {   // shift both rings by two planes
#pragma unroll
      for (int s = 0; s < NQ; ++s) {
#pragma unroll
        for (int k = 0; k < 8; ++k) acc[s][k] = acc[s][k + 2];
        acc[s][8] = acc[s][9] = 0;
      }
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  using I3 = std::integral_constant<int, 3>;
  using I4 = std::integral_constant<int, 4>;
  auto tail = [&](int p) __attribute__((always_inline)) {   // the last two planes, p = nt - 2
    if (p & 1) {
      step(p, I1(), I3());
      step(p + 1, I0(), I4());
    } else {
      step(p, I0(), I3());
      step(p + 1, I1(), I4());
    }
  };
  if (nch == 1) {   // whole time axis (trip count fixed at compile time when NT > 0)
    step(0, I0(), I0());
    step(1, I1(), I1());
    int p = 2;
#pragma unroll
    for (; p + 1 <= nt - 3; p += 2) {
      step(p, I0(), I2());
      step(p + 1, I1(), I2());
    }
    if (p <= nt - 3) step(p++, I0(), I2());
    tail(p);
  } else {          // one chunk: interior planes in a loop unrolled by two
    int p = r0;
    if (ch == 0) {
      step(0, I0(), I0());
      step(1, I1(), I1());
      p = 2;
    }
    const int pe = ch == nch - 1 ? nt - 3 : t1 + 1;
    for (; p + 1 <= pe; p += 2) {
      step(p, I0(), I2());
      step(p + 1, I1(), I2());
    }
    if (p <= pe) step(p++, I0(), I2());
    if (ch == nch - 1) tail(p);
  }
  if (MODE == G_STORE_DOT) {
    const double sdot = fblock_sum<NTH>((double)dot);
    if (threadIdx.x == 0) partial[tl.pad] = sdot;
  }
}

template <typename TA, typename TV, typename TC, int M, int T, bool SIG>
static void apply3_one(hipStream_t st, const FTile* tiles, int nb, FGeom g, const LInst* li, CIdx ci, const TV* u,
                       const TC* c, TV* out, const TV* bvec, TV* x, TV* r, TV* d, const TV* dinv, int cheb_step,
                       double* partial, size_t lds, hipEvent_t e0, hipEvent_t e1, const TC* f, const TC* w) {
  // Raise the dynamic-LDS limit of this instantiation on the current device
  // to the largest size requested so far (a host call, kept out of the
  // per-launch path).
  static size_t granted[64] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  dev = dev < 0 || dev >= 64 ? 0 : dev;
  if (lds > granted[dev]) {
    const size_t want = std::max<size_t>(lds, 96 * 1024);
    (void)hipFuncSetAttribute((const void*)k_apply3<TA, TV, TC, M, T, SIG>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)want);
    granted[dev] = want;
  }
  // time chunks along y (not for the dot product: its per-tile partial sum
  // has one slot per tile)
  const dim3 grid((unsigned)nb, M == G_STORE_DOT || g.nch < 1 ? 1u : (unsigned)g.nch);
  if (e0 && e1)   // timed: the events take the dispatch's own start and end times
    hipExtLaunchKernelGGL((k_apply3<TA, TV, TC, M, T, SIG>), grid, dim3((unsigned)g.nthr), lds, st, e0, e1, 0,
                          tiles, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step, partial, f, w);
  else
    hipLaunchKernelGGL((k_apply3<TA, TV, TC, M, T, SIG>), grid, dim3((unsigned)g.nthr), lds, st, tiles, g, li, ci,
                       u, c, out, bvec, x, r, d, dinv, cheb_step, partial, f, w);
}

template <typename TA, typename TV, typename TC, int M>
static void apply3_mode(hipStream_t st, const FTile* tiles, int nb, FGeom g, const LInst* li, CIdx ci, const TV* u,
                        const TC* c, TV* out, const TV* bvec, TV* x, TV* r, TV* d, const TV* dinv, int cheb_step,
                        double* partial, size_t lds, hipEvent_t e0, hipEvent_t e1, const TC* f, const TC* w) {
  // (the FP64 dot-product pass has no unrolled variant: it would not fit the
  // register file; right-hand-side terms exist for the FP64 residual only)
  constexpr bool unroll = !(sizeof(TA) == 8 && M == G_STORE_DOT);
  constexpr bool rhs = sizeof(TA) == 8 && M == G_RESID;
  if constexpr (rhs) {
    if (f && w) {
      if (g.nt == 32)
        apply3_one<TA, TV, TC, M, 32, true>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step,
                                            partial, lds, e0, e1, f, w);
      else
        apply3_one<TA, TV, TC, M, 0, true>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step,
                                           partial, lds, e0, e1, f, w);
      return;
    }
  }
  if (f || w) throw std::string("fused operator: right-hand-side terms only in the FP64 residual");
  if (unroll && g.nt == 32)
    apply3_one<TA, TV, TC, M, unroll ? 32 : 0, false>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv,
                                                       cheb_step, partial, lds, e0, e1, nullptr, nullptr);
  else
    apply3_one<TA, TV, TC, M, 0, false>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step, partial,
                                        lds, e0, e1, nullptr, nullptr);
}

template <typename TA, typename TV, typename TC>
void launch_apply3(hipStream_t st, const FTile* tiles, int nb, FGeom g, const LInst* li, CIdx ci, const TV* u,
                   const TC* c, int mode, TV* out, const TV* bvec, TV* x, TV* r, TV* d, const TV* dinv,
                   int cheb_step, double* partial, hipEvent_t e0, hipEvent_t e1, const TC* f, const TC* w) {
  if (nb <= 0) return;
  const size_t lds = sizeof(TA) * (kFRing * (size_t)g.uplane + 16 * (size_t)g.qplane);   // qplane: 4-value slots x 4
  switch (mode) {
    case G_STORE:
      apply3_mode<TA, TV, TC, G_STORE>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step, partial,
                                       lds, e0, e1, f, w);
      break;
    case G_RESID:
      apply3_mode<TA, TV, TC, G_RESID>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step, partial,
                                       lds, e0, e1, f, w);
      break;
    case G_CHEB:
      apply3_mode<TA, TV, TC, G_CHEB>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step, partial,
                                      lds, e0, e1, f, w);
      break;
    default:
      apply3_mode<TA, TV, TC, G_STORE_DOT>(st, tiles, nb, g, li, ci, u, c, out, bvec, x, r, d, dinv, cheb_step,
                                           partial, lds, e0, e1, f, w);
      break;
  }
}

template void launch_apply3<float, float, float>(hipStream_t, const FTile*, int, FGeom, const LInst*, CIdx,
                                                 const float*, const float*, int, float*, const float*, float*,
                                                 float*, float*, const float*, int, double*, hipEvent_t, hipEvent_t,
                                                 const float*, const float*);
template void launch_apply3<double, double, float>(hipStream_t, const FTile*, int, FGeom, const LInst*, CIdx,
                                                   const double*, const float*, int, double*, const double*, double*,
                                                   double*, double*, const double*, int, double*, hipEvent_t,
                                                   hipEvent_t, const float*, const float*);

}  // namespace mpde
