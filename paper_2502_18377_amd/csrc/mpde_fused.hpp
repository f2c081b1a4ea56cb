// Fused operator for three-axis levels (t, x, y): tile geometry shared by the
// host (tile tables, LDS sizing) and the kernel, and the launch wrapper.
#pragma once
#include "mpde_internal.hpp"

namespace mpde {

constexpr int kFThreads = 768;   // threads per block, FP32 arithmetic
constexpr int kFThreads64 = 512; // threads per block, FP64 arithmetic (twice the registers per value)
template <typename TA>
constexpr int fthreads() {
  return sizeof(TA) == 8 ? kFThreads64 : kFThreads;
}
constexpr int kFMaxQ = 1;        // row points per thread and plane
constexpr int kFRing = 10;       // staged u planes kept in LDS

// One block: an instance and the origin of its (x, y) tile; the block marches
// over every time plane.
struct FTile {
  int inst, x0, y0, pad;
};

// Per-launch constants: tile extents and LDS strides (maxima over the tiles).
struct FGeom {
  int TX, TY;        // tile extent in x and y
  int uplane;        // elements of one staged u plane
  int qplane;        // float4 slots of one staged row-value plane
  int nt;            // time planes of every instance of the launch, 0 if they differ
  int nthr;          // threads per block: the tiles' row points rounded up to whole
                     // wavefronts (at most fthreads<TA>(); staged u slots <= 2 nthr)
  int nch;           // time chunks per tile (1: the whole time axis per block)
  int tc;            // output planes per time chunk (even; chunk edges in [5, nt - 5])
};

// Ranges of one axis for a tile [x0, x0 + T) of an axis with n points:
//   rows  [qlo, qlo + qn): points whose rows reach the tile (windows and
//                          Taylor neighbours);
//   u     [ulo, ulo + un): points those rows read;
//   slots: staged row values are stored at (row - qlo) + qoff, with qoff = 2
//          and wrapped copies at both ends when the tile spans a whole
//          periodic axis (fw), so that every read is a plain offset;
//   tile  [ilo, ilo + icnt) in row-local coordinates.
struct FSpan {
  int qlo, qn, ulo, un, fw, qoff, qs, ilo, icnt;
};

__host__ __device__ inline int fclampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

__host__ __device__ inline FSpan fspan(int x0, int T, int n, int per) {
  FSpan s;
  const int x1 = (x0 + T < n) ? x0 + T : n;
  s.icnt = x1 - x0;
  if (per) {
    s.fw = (x0 == 0 && x1 == n) ? 1 : 0;
    s.qlo = s.fw ? 0 : x0 - 2;
    s.qn = s.fw ? n : s.icnt + 4;
    s.ulo = s.qlo - 2;
    s.un = s.qn + 4;
    s.qoff = s.fw ? 2 : 0;
    s.qs = s.qn + (s.fw ? 4 : 0);
    s.ilo = x0 - s.qlo;
    return s;
  }
  // Rows 0..2 (window 0..4) reach points up to 4, rows n-3..n-1 reach down to
  // n-5; other rows reach +-2.
  const int qlo = x0 <= 4 ? 0 : x0 - 2;
  const int qhi = x1 >= n - 4 ? n : x1 + 2;
  const int ulo = fclampi(qlo - 2, 0, n - 5), uhi = fclampi(qhi - 3, 0, n - 5) + 5;
  s.fw = 0;
  s.qlo = qlo;
  s.qn = qhi - qlo;
  s.ulo = ulo;
  s.un = uhi - ulo;
  s.qoff = 0;
  s.qs = s.qn;
  s.ilo = x0 - qlo;
  return s;
}

// y = S u with the epilogue of `mode` (GatherMode); with f and w (level-0
// source and boundary values; FP64 residual only) y = A_u^T Pi (A_u u - d),
// the right-hand-side terms included.  Every instance of the tile table must
// have periodic x and y axes and a non-periodic time axis of at least five
// points, and the table must be cut for at most fthreads<TA>() threads
// (g.nthr per block).  Instantiated for FP32 (all modes) and FP64 (vectors
// and arithmetic in FP64, coefficients FP32).  With events e0, e1 the launch
// records the dispatch's start and end time in them.
template <typename TA, typename TV, typename TC>
void launch_apply3(hipStream_t st, const FTile* tiles, int nb, FGeom g, const LInst* li, CIdx ci, const TV* u,
                   const TC* c, int mode, TV* out, const TV* bvec, TV* x, TV* r, TV* d, const TV* dinv,
                   int cheb_step, double* partial, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                   const TC* f = nullptr, const TC* w = nullptr);

}  // namespace mpde
