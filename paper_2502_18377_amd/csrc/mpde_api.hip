// Host runtime of the MI355X NeuRLP-PDE solver: the C ABI of include/mpde.h.
//
// Solve structure (paper: Sec. "An Iterative Sparse Multigrid Solver" and
// the V-cycle algorithm of the appendix):
//   * outer loop: FP64 iterate u and FP64 residual g - S u formed row by row
//     as A_u^T Pi (d - A u) (never as A^T d - A^T A u), stop at the requested
//     normal-equation relative residual;
//   * inner solve: conjugate gradients in the problem's precision (FP32 or
//     FP64) on S e = r, preconditioned by one multigrid V-cycle;
//   * V-cycle: Chebyshev/point-Jacobi smoothing (a parallel replacement of
//     the paper's Gauss-Seidel relaxation), residual, restriction by the
//     transpose of linear interpolation, recursion, prolongation by linear
//     interpolation, correction, smoothing; the coarsest grid is solved
//     exactly with a dense inverse built once per problem;
//   * grids: every spatial axis is halved with its step doubled while it
//     stays at or above the minimum size (time is never coarsened, because the
//     reduced operator couples space far more strongly than time); coarse
//     operators are re-discretised from coefficient fields coarsened by
//     normalised full weighting, with Taylor and first-difference rows
//     weighted 2^-k and second-difference rows 4^-k (k = halvings of that
//     axis), which keeps each derivative unknown's stiffness level-invariant.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <new>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <functional>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/mpde.h"
#include "mpde_internal.hpp"
#include "mpde_kernels.hpp"
#include "mpde_fused.hpp"
#include "mpde_conv.hpp"

using namespace mpde;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct HipError {
  hipError_t e;
  const char* what;
};

#define HIPCHK(x)                                                   \
  do {                                                              \
    hipError_t _e = (x);                                            \
    if (_e != hipSuccess) throw HipError{_e, #x};                   \
  } while (0)

constexpr int kMaxDense = 4096;   // coarsest points per instance (block solves keep T*m doubles in LDS)

// ---------------------------------------------------------------- stencils
// 5-point weights from the moment conditions sum_k w_k o_k^p / p! = [p == q]
// (Gaussian elimination with partial pivoting in double precision).
void fd_table(int q, double out[5][5]) {
  for (int pos = 0; pos < 5; ++pos) {
    double M[5][6];
    for (int p = 0; p < 5; ++p) {
      double fact = 1;
      for (int t = 2; t <= p; ++t) fact *= t;
      for (int k = 0; k < 5; ++k) M[p][k] = std::pow((double)(k - pos), p) / fact;
      M[p][5] = (p == q) ? 1.0 : 0.0;
    }
    for (int c = 0; c < 5; ++c) {
      int piv = c;
      for (int r = c + 1; r < 5; ++r)
        if (std::fabs(M[r][c]) > std::fabs(M[piv][c])) piv = r;
      for (int k = 0; k < 6; ++k) std::swap(M[c][k], M[piv][k]);
      for (int r = 0; r < 5; ++r) {
        if (r == c) continue;
        const double f = M[r][c] / M[c][c];
        for (int k = c; k < 6; ++k) M[r][k] -= f * M[c][k];
      }
    }
    for (int k = 0; k < 5; ++k) out[pos][k] = M[k][5] / M[k][k];
  }
}

// Device-memory cache.  Buffers a problem releases are kept per (device,
// size) and handed to later builds, so that one-problem-per-batch use (build,
// solve, free, repeated) pays hipMalloc/hipFree (about 0.1 ms per buffer,
// ~160 buffers per problem) only once.  At most kCacheCap bytes per device
// stay cached; a release beyond that, and every cached block when hipMalloc
// runs out of memory, goes back to the runtime.  The cache lives until the
// process ends.
constexpr size_t kCacheCap = size_t(16) << 30;
struct DevCache {
  std::mutex mu;
  std::map<std::pair<int, size_t>, std::vector<void*>> blocks;
  std::map<int, size_t> bytes;
  std::map<int, std::vector<hipStream_t>> streams;
};
DevCache& dcache() {
  static DevCache* c = new DevCache();   // never destroyed: used until exit
  return *c;
}
int cur_device() {
  int d = 0;
  (void)hipGetDevice(&d);
  return d;
}
size_t cache_round(size_t b) { return (std::max<size_t>(b, 1) + 255) & ~size_t(255); }

void* dev_get(size_t bytes) {
  bytes = cache_round(bytes);
  const int dev = cur_device();
  DevCache& c = dcache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto it = c.blocks.find({dev, bytes});
    if (it != c.blocks.end() && !it->second.empty()) {
      void* p = it->second.back();
      it->second.pop_back();
      c.bytes[dev] -= bytes;
      return p;
    }
  }
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e == hipErrorOutOfMemory) {   // give the cached blocks of this device back and retry
    (void)hipGetLastError();
    std::lock_guard<std::mutex> g(c.mu);
    for (auto& kv : c.blocks)
      if (kv.first.first == dev) {
        for (void* q : kv.second) (void)hipFree(q);
        kv.second.clear();
      }
    c.bytes[dev] = 0;
    e = hipMalloc(&p, bytes);
  }
  if (e != hipSuccess) throw HipError{e, "hipMalloc"};
  return p;
}

void dev_put(void* p, size_t bytes, int dev) {
  if (!p) return;
  bytes = cache_round(bytes);
  DevCache& c = dcache();
  std::lock_guard<std::mutex> g(c.mu);
  if (c.bytes[dev] + bytes > kCacheCap) {
    int keep = cur_device();
    (void)hipSetDevice(dev);
    (void)hipFree(p);
    (void)hipSetDevice(keep);
    return;
  }
  c.blocks[{dev, bytes}].push_back(p);
  c.bytes[dev] += bytes;
}

// Streams for captured graphs, kept per device like the buffers.
hipStream_t stream_get() {
  const int dev = cur_device();
  DevCache& c = dcache();
  {
    std::lock_guard<std::mutex> g(c.mu);
    auto& v = c.streams[dev];
    if (!v.empty()) {
      hipStream_t s = v.back();
      v.pop_back();
      return s;
    }
  }
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e != hipSuccess) throw HipError{e, "hipStreamCreateWithFlags"};
  return s;
}
void stream_put(hipStream_t s, int dev) {
  if (!s) return;
  DevCache& c = dcache();
  std::lock_guard<std::mutex> g(c.mu);
  c.streams[dev].push_back(s);
}

// A device buffer owned by a problem: returned to the cache on release.
struct Block {
  void* p;
  size_t bytes;
  int dev;
};

template <typename T>
T* dalloc(size_t n) {
  return (T*)dev_get((n == 0 ? 1 : n) * sizeof(T));
}

// A host work table and its device copy, with per-instance block ranges.
struct Table {
  std::vector<Work> h;
  std::vector<int> bstart;     // [B+1]
  long long npts = 0;          // points covered
  Work* d = nullptr;
  int* d_bstart = nullptr;
  int nb() const { return (int)h.size(); }
};

// Tiles of the fused three-axis operator over the selected instances, with
// per-instance ranges of block-partial slots (FTile.pad).
struct FTab {
  std::vector<FTile> h;
  std::vector<int> bstart;     // [B+1] over partial slots
  FGeom g{};
  bool ok = false;             // every selected instance fits the fused kernel
  FTile* d = nullptr;
  int* d_bstart = nullptr;
  int nb() const { return (int)h.size(); }
};

struct Level {
  std::vector<LInst> h;        // [B]; N = 0 for instances without this level
  LInst* d = nullptr;
  std::vector<LInst> hg;       // h with the Krylov gate (act) set, and its device copy
  LInst* dg = nullptr;
  long long npts = 0;          // total points of this level
  Table all, smooth, dense;    // all instances / non-coarsest / coarsest (rows)
  FTab fall, fsmooth;          // fused-operator tiles for `all` and `smooth`
  FTab fall64;                 // level 0, FP64 arithmetic (outer residual)
  std::vector<int> cinst64, cinst16, cinstg;   // coarsest here: 64-point / <= 16-point / other planes
  int *d_cinst64 = nullptr, *d_cinst16 = nullptr, *d_cinstg = nullptr;
  void* coef = nullptr;        // TC [K planes per instance]
  void *x = nullptr, *r = nullptr, *dd = nullptr, *dd2 = nullptr, *b = nullptr, *gam = nullptr, *dinv = nullptr;
};

}  // namespace

// Learned coarse correction: FP32 master parameters, Adam state and bf16
// weight copies (layout [tap][out][in] and transposed [tap][in][out]).
struct mpde_net {
  int cin = 1;
  long long t = 0;                   // Adam step
  float *w = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
  unsigned short *wb = nullptr, *wtb = nullptr;   // 3 layers x 27*256
  float* partial = nullptr;          // weight-gradient block partials
  std::vector<void*> owned;
  ~mpde_net() {
    for (void* p : owned) (void)hipFree(p);
  }
};

namespace {
constexpr int kLayerW = 27 * 256;
constexpr int kLayerP = kLayerW + 16;
}  // namespace

// Per-problem buffers of the network at its grid level.
struct NetScratch {
  int level = -1;
  long long npts = 0;
  int ntiles = 0;
  mpde::Grid3* grids = nullptr;
  int2* tiles = nullptr;
  unsigned short *X0 = nullptr, *A1 = nullptr, *A2 = nullptr, *Db = nullptr;
  float *P1 = nullptr, *P2 = nullptr, *Y3 = nullptr, *dA = nullptr, *dB = nullptr;
  double *norm = nullptr, *inv = nullptr;
};

struct mpde_problem {
  int dtype = 0, D = 0, B = 0, K = 0, V = 0;
  uint32_t mset = 0;
  CIdx ci{};
  mpde_options opt{};
  hipStream_t st = nullptr;
  int bc_lo[3] = {0, 0, 0}, bc_hi[3] = {0, 0, 0};
  std::vector<std::vector<std::array<int, 3>>> lshape;   // [b][level]
  std::vector<int> nlev;
  std::vector<Level> lv;
  std::vector<long long> zoff_h;
  long long* zoff = nullptr;
  void *f = nullptr, *w = nullptr;                          // TC, level-0 layout
  double *u64 = nullptr, *r64 = nullptr, *g64 = nullptr, *ghat = nullptr, *vloc = nullptr, *du64 = nullptr;
  double* rhs64 = nullptr;   // forward right side A_u^T Pi d on level 0 (the residual at u = 0)
  void *e = nullptr, *rk = nullptr, *zk = nullptr, *pk = nullptr, *qk = nullptr;   // TV, level 0
  double* partial = nullptr;
  double *rz_new = nullptr, *rz = nullptr, *beta = nullptr, *pq = nullptr, *alpha = nullptr, *rn2 = nullptr,
         *r0n2 = nullptr, *atd2 = nullptr, *scale = nullptr, *iscale = nullptr,
         *itol2 = nullptr;   // per-instance squared relative tolerance of the inner solve
  int *active = nullptr, *iters = nullptr, *flag = nullptr;
  void* Sinv = nullptr;                                    // TV dense inverses
  bool has_solution = false;
  const mpde_net* net = nullptr;                           // learned coarse correction
  int net_level = 0;
  NetScratch ns;
  void* zp = nullptr;                                      // previous z (flexible CG)
  double* rzp = nullptr;
  long long fallbacks = 0;                                 // learned -> plain V-cycle switches
  // captured Krylov chunks (first chunk of a solve / later chunks)
  hipStream_t gst = nullptr;
  hipGraphExec_t gexec[2] = {nullptr, nullptr};
  int gkey[2] = {0, 0};                                    // (nu, chunk) the graphs were captured with
  hipEvent_t gev[2] = {nullptr, nullptr};
  void drop_graphs() {
    for (auto& g : gexec)
      if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
  }
  // profiling (options.profile): event pairs around finest-grid kernels
  struct Rec { int kind; hipEvent_t a, b; double bytes; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  mpde_kstat kst[3]{};
  hipEvent_t ev() {
    if (pool_used == pool.size()) {
      hipEvent_t e;
      // no system-scope release on record: the timed kernels only touch device memory
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[pool_used++];
  }
  std::vector<Block> owned;
  int home = 0;                                            // device of the buffers and streams
  ~mpde_problem() {
    drop_graphs();
    for (hipEvent_t e : gev) if (e) (void)hipEventDestroy(e);
    if (gst) {
      (void)hipStreamSynchronize(gst);
      stream_put(gst, home);
    }
    if (st) (void)hipStreamSynchronize(st);               // nothing in flight may still use a released buffer
    for (const Block& b : owned) dev_put(b.p, b.bytes, b.dev);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
  template <typename T>
  T* alloc(size_t n) {
    T* p = dalloc<T>(n);
    owned.push_back({p, (n == 0 ? 1 : n) * sizeof(T), cur_device()});
    return p;
  }
};

namespace {

// Host tables bound for one device arena: each add() reserves a 256-byte
// aligned slot in a host image and remembers which device pointer to set;
// commit() allocates the arena, copies the image in one transfer and sets
// the pointers (one copy instead of a synchronous copy per table).
struct Uploads {
  std::vector<char> img;
  std::vector<std::pair<void**, size_t>> slots;
  template <typename T>
  void add(T*& dst, const void* src, size_t bytes) {
    const size_t off = (img.size() + 255) & ~size_t(255);
    img.resize(off + std::max<size_t>(bytes, 1));
    if (bytes) std::memcpy(img.data() + off, src, bytes);
    slots.push_back({reinterpret_cast<void**>(&dst), off});
  }
  void commit(mpde_problem* P) {
    char* a = P->alloc<char>(std::max<size_t>(img.size(), 1));
    if (!img.empty()) HIPCHK(hipMemcpy(a, img.data(), img.size(), hipMemcpyHostToDevice));
    for (auto& s : slots) *s.first = a + s.second;
    img.clear();
    slots.clear();
  }
};

// The gated copy of a level's descriptors: act points at the instance's
// active flag, so that the kernels of a Krylov iteration skip converged
// instances.
void gate_copy(mpde_problem* P, Level& L) {
  L.hg = L.h;
  for (size_t b = 0; b < L.hg.size(); ++b) L.hg[b].act = P->active + b;
}

void upload_table(Uploads& U, Table& t) {
  U.add(t.d, t.h.data(), t.h.size() * sizeof(Work));
  U.add(t.d_bstart, t.bstart.data(), t.bstart.size() * sizeof(int));
}

// Work items over the points of the selected instances (instance-major).
void make_table(Table& t, const std::vector<LInst>& h, int B, const std::vector<int>& sel) {
  t.h.clear();
  t.npts = 0;
  t.bstart.assign(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    t.bstart[b] = (int)t.h.size();
    if (!sel[b]) continue;
    for (int s = 0; s < h[b].N; s += kBlock) t.h.push_back(Work{b, s});
    t.npts += h[b].N;
  }
  t.bstart[B] = (int)t.h.size();
}

// Tiles of the fused operator: each selected instance is cut into (TX, TY)
// tiles of its (x, y) plane; TX and TY are divisors of the largest extents,
// common to the level, such that the rows of a tile plus halo fit one block
// of `nth` threads (one row point each) and its staged u plane fits two
// values per thread.  The tile shape and the number of time chunks (at most
// `chunks`, 0 = up to 4) are those of least estimated time (below); halo
// rows are evaluated by every tile that needs them and halo planes by every
// chunk, so the estimate weighs that redundant work against the parallelism
// it buys.  `esize` is the byte size of the
// arithmetic type (LDS budget); `mult` (optional) counts each instance that
// many times in the choice (instances that stand for several identical
// ones).  Consecutive groups of 8 instances are
// interleaved tile by tile, so that with round-robin block dispatch all
// tiles of one instance (which share halos) run on the same XCD and its L2.
void make_ftab(FTab& f, const std::vector<LInst>& h, int B, const std::vector<int>& sel, int D, int nth,
               size_t esize, const std::vector<long long>* mult = nullptr, int chunks = 1) {
  f.h.clear();
  f.bstart.assign(B + 1, 0);
  f.ok = false;
  if (D != 3) return;
  int nsel = 0, mnx = 0, mny = 0;
  for (int b = 0; b < B; ++b) {
    if (!sel[b] || h[b].N == 0) continue;
    const LInst& q = h[b];
    if (q.per[0] || !q.per[1] || !q.per[2] || q.n[0] < 5 || q.n[1] < 4 || q.n[2] < 4) return;
    if (4LL * q.N * 7 >= (1LL << 31) || (long long)esize * q.N >= (1LL << 31)) return;   // 31-bit buffer offsets
    ++nsel;
    mnx = std::max(mnx, q.n[1]);
    mny = std::max(mny, q.n[2]);
  }
  if (nsel == 0) return;
  // tiles of shape (TX, TY): count, total wavefronts, LDS extents; false if
  // some tile does not fit a block
  struct Cut {
    long long tiles = 0, waves = 0;
    int uplane = 0, qplane = 0, nthr = 0;
  };
  // instances grouped by plane shape: a candidate is evaluated once per shape
  std::map<std::pair<int, int>, long long> shapes;
  for (int b = 0; b < B; ++b)
    if (sel[b] && h[b].N > 0) shapes[{h[b].n[1], h[b].n[2]}] += mult ? (*mult)[b] : 1;
  auto cut = [&](int TX, int TY, Cut& c) {
    c = Cut{};
    for (const auto& sh : shapes) {
      const int nx = sh.first.first, ny = sh.first.second;
      const long long cnt = sh.second;
      for (int x0 = 0; x0 < nx; x0 += TX)
        for (int y0 = 0; y0 < ny; y0 += TY) {
          const FSpan X = fspan(x0, TX, nx, 1), Y = fspan(y0, TY, ny, 1);
          if (X.qn * Y.qn > nth || X.un * Y.un > 2 * nth) return false;
          c.tiles += cnt;
          c.waves += cnt * ((X.qn * Y.qn + 63) / 64);
          c.uplane = std::max(c.uplane, X.un * Y.un);
          c.qplane = std::max(c.qplane, X.qs * Y.qs);
          // block size: every row point, and every staged u slot within two per thread
          c.nthr = std::max(c.nthr, std::max(X.qn * Y.qn, (X.un * Y.un + 1) / 2));
        }
    }
    c.uplane = (c.uplane + 1 + 3) & ~3;   // spare slot for idle threads' staging writes; 16-byte rows
    c.nthr = (c.nthr + 63) / 64 * 64;
    return esize * (kFRing * (size_t)c.uplane + 16 * (size_t)c.qplane) <= 160000;   // LDS per block
  };
  std::vector<std::pair<int, int>> cand;   // larger tiles first (preferred on ties)
  for (int ty = mny; ty >= std::min(4, mny); --ty)
    if (mny % ty == 0)
      for (int tx = mnx; tx >= std::min(4, mnx); --tx)
        if (mnx % tx == 0) cand.push_back({tx, ty});
  std::vector<std::pair<std::pair<int, int>, Cut>> ok;
  for (auto& tt : cand) {
    Cut c;
    if (!cut(tt.first, tt.second, c)) continue;
    ok.push_back({tt, c});
  }
  if (ok.empty()) return;
  // time planes: common to every selected instance (nt > 0) or not (0)
  int nt = -1, mnt = 0;
  for (int b = 0; b < B; ++b)
    if (sel[b] && h[b].N > 0) {
      nt = (nt == -1 || nt == h[b].n[0]) ? h[b].n[0] : 0;
      mnt = std::max(mnt, h[b].n[0]);
    }
  // time chunkings (count, planes per chunk): an even chunk length, so every
  // chunk starts on an even plane, and chunk edges in [5, nt - 5]
  std::vector<std::pair<int, int>> chk{{1, 0}};
  if (nt > 0 && chunks != 1)
    for (int want = 2; want <= (chunks == 0 ? 4 : chunks); want *= 2) {
      const int tc = ((nt + want - 1) / want + 1) & ~1;
      const int nc = (nt + tc - 1) / tc;
      if (tc >= 5 && (nc - 1) * tc <= nt - 5 && nc > chk.back().first) chk.push_back({nc, tc});
    }
  if (chunks > 1) chk.erase(chk.begin(), chk.end() - 1);   // forced: the most chunks allowed
  // Estimated launch time (us) of the FP32 one-pass kernel, a model fitted
  // to its measured launches: a block's plane step takes at least 0.93 us
  // (one wavefront per SIMD: the dependent chain of a step), and beyond that
  // the 1024 SIMDs retire one wavefront plane step per 0.55 us each (issue
  // bound).  The fewest wavefronts is not always the fastest choice: on
  // small levels the latency term rules, and time chunks shorten it.
  auto est = [&](const Cut& c, int nc, int tc) {
    const int T = nt > 0 ? nt : mnt;
    const double longest = nc == 1 ? T : nc == 2 ? std::max(tc + 2, T - tc + 2) : tc + 4;
    const double total = (double)c.waves * (T + 4.0 * (nc - 1));
    return std::max(0.93 * longest, 0.55 * total / 1024.0);
  };
  int bi = -1, bc = 0;
  double best = 0;
  for (int i = 0; i < (int)ok.size(); ++i)
    for (int k = 0; k < (int)chk.size(); ++k) {
      const double e = est(ok[i].second, chk[k].first, chk[k].second);
      const long long w = ok[i].second.waves * chk[k].first;
      if (bi < 0 || e < best - 1e-9 || (e <= best + 1e-9 && w < ok[bi].second.waves * chk[bc].first)) {
        bi = i;
        bc = k;
        best = e;
      }
    }
  const int TX = ok[bi].first.first, TY = ok[bi].first.second;
  f.g.TX = TX;
  f.g.TY = TY;
  f.g.uplane = ok[bi].second.uplane;
  f.g.qplane = ok[bi].second.qplane;
  f.g.nthr = ok[bi].second.nthr;
  f.g.nch = chk[bc].first;
  f.g.tc = chk[bc].second;
  f.g.nt = -1;
  std::vector<std::vector<FTile>> per(B);
  int slot = 0;
  for (int b = 0; b < B; ++b) {
    f.bstart[b] = slot;
    if (!sel[b] || h[b].N == 0) continue;
    const LInst& q = h[b];
    for (int x0 = 0; x0 < q.n[1]; x0 += TX)
      for (int y0 = 0; y0 < q.n[2]; y0 += TY) {
        per[b].push_back(FTile{b, x0, y0, slot++});
        f.g.nt = (f.g.nt == -1 || f.g.nt == q.n[0]) ? q.n[0] : 0;
      }
  }
  f.bstart[B] = slot;
  for (int g0 = 0; g0 < B; g0 += 8) {
    size_t mt = 0;
    for (int b = g0; b < std::min(B, g0 + 8); ++b) mt = std::max(mt, per[b].size());
    for (size_t t = 0; t < mt; ++t)
      for (int b = g0; b < std::min(B, g0 + 8); ++b)
        if (t < per[b].size()) f.h.push_back(per[b][t]);
  }
  f.ok = true;
}

void upload_ftab(Uploads& U, FTab& f) {
  if (!f.ok) return;
  U.add(f.d, f.h.data(), f.h.size() * sizeof(FTile));
  U.add(f.d_bstart, f.bstart.data(), f.bstart.size() * sizeof(int));
}

template <typename TV>
struct Ptr {
  static TV* v(void* p) { return (TV*)p; }
};

// ----------------------------------------------------------------- solver
template <typename TV, typename TC>
struct Solver {
  mpde_problem* P;
  hipStream_t st;
  int D;
  bool use_net = true;
  explicit Solver(mpde_problem* p) : P(p), st(p->st), D(p->D) {}

  // ---------------------------------------------------------- network
  // Scratch and conv tables for the network at level l (all instances that
  // have level l).
  void net_setup(int l) {
    NetScratch& S = P->ns;
    if (S.level == l) return;
    Level& L = P->lv[l];
    std::vector<mpde::Grid3> g(P->B);
    std::vector<int2> tiles;
    for (int b = 0; b < P->B; ++b) {
      const LInst& q = L.h[b];
      g[b] = mpde::Grid3{q.n[0], q.n[1], D == 3 ? q.n[2] : 1, {q.per[0], q.per[1], D == 3 ? q.per[2] : 0}, q.voff};
      for (int s0 = 0; s0 < q.N; s0 += 16) tiles.push_back(make_int2(b, s0));
    }
    while (tiles.size() % 4) tiles.push_back(make_int2(-1, 0));
    S.level = l;
    S.npts = L.npts;
    S.ntiles = (int)tiles.size();
    S.grids = P->alloc<mpde::Grid3>(P->B);
    S.tiles = P->alloc<int2>(tiles.size());
    HIPCHK(hipMemcpy(S.grids, g.data(), P->B * sizeof(mpde::Grid3), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.tiles, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice));
    const size_t n16 = (size_t)L.npts * 16;
    S.X0 = P->alloc<unsigned short>(n16);
    S.A1 = P->alloc<unsigned short>(n16);
    S.A2 = P->alloc<unsigned short>(n16);
    S.Db = P->alloc<unsigned short>(n16);
    S.P1 = P->alloc<float>(n16);
    S.P2 = P->alloc<float>(n16);
    S.Y3 = P->alloc<float>(n16);
    S.dA = P->alloc<float>(n16);
    S.dB = P->alloc<float>(n16);
    S.norm = P->alloc<double>(P->B);
    S.inv = P->alloc<double>(P->B);
  }

  // Per-instance ||r|| and 1/||r|| of a level vector into ns.norm / ns.inv.
  void level_norms(int l, const TV* r) {
    Level& L = P->lv[l];
    launch_dot<double, TV>(st, L.all.d, L.all.nb(), L.d, r, r, P->partial);
    finish(L.all, P->rzp);
    norms_launch(st, P->B, P->rzp, P->ns.norm, P->ns.inv);
  }

  void net_forward(const mpde_net* net) {
    NetScratch& S = P->ns;
    const unsigned short* W = net->wb;
    const float* bias = net->w;
    conv_launch(st, S.ntiles, S.tiles, S.grids, S.X0, W, bias + kLayerW, 1, S.P1, S.A1, 1);
    conv_launch(st, S.ntiles, S.tiles, S.grids, S.A1, W + kLayerW, bias + kLayerP + kLayerW, 1, S.P2, S.A2, 1);
    conv_launch(st, S.ntiles, S.tiles, S.grids, S.A2, W + 2 * kLayerW, bias + 2 * kLayerP + kLayerW, 1, S.Y3,
                nullptr, 0);
  }

  // Learned coarse correction on level l: the plain V-cycle's correction
  // v = V_l(b) plus the network's refinement, x = v + D^-1 N(b, v, c) ||b||.
  void learned(int l, TV* b, TV* x) {
    Level& L = P->lv[l];
    const bool keep = use_net;
    use_net = false;
    vcycle(l, b, x);
    use_net = keep;
    level_norms(l, b);
    features_launch(st, L.all.d, L.all.nb(), L.d, P->K, (const float*)b, (const float*)x, (const float*)L.dinv,
                    P->ns.inv, (const float*)L.coef, P->ns.X0);
    net_forward(P->net);
    net_out_launch(st, L.all.d, L.all.nb(), L.d, P->ns.Y3, (const float*)L.dinv, P->ns.norm, (float*)x);
  }

  // Training residuals at level l: a hashed right-hand side per instance on
  // the finest grid, Chebyshev-smoothed and restricted level by level as in
  // the down leg of a V-cycle; the result is left in lv[l].b.
  void sample_residuals(int l, unsigned seed) {
    for (int k = 0; k < l; ++k) {
      Level& L = P->lv[k];
      const Table& t = L.smooth;
      if (k == 0) launch_hash_fill<TV>(st, t.d, t.nb(), L.d, V(L.b), seed);
      launch_cheb_init<TV>(st, t.d, t.nb(), L.d, V(L.b), V(L.dinv), V(L.x), V(L.r), V(L.dd));
      chebyshev(k, V(L.x), P->opt.nu);
      Level& Cc = P->lv[k + 1];
      launch_restrict<TV>(D, st, Cc.all.d, Cc.all.nb(), L.d, Cc.d, V(L.r), V(Cc.b));
    }
  }

  // One training step of net on problem level l >= 1; returns the mean loss
  // of the learned correction and (loss_plain) of the plain V-cycle's.  The
  // loss is the energy on the next finer level f = l - 1 of the prolonged
  // coarse correction, E(o) = (P o)^T S_f (P o) - 2 (P o)^T r_f for the
  // pre-smoothed residual r_f (both scaled by 1 / ||R r_f||): its minimiser
  // is the Galerkin coarse correction, so the network learns what the
  // rediscretised coarse operator and the recursive V-cycle miss for the
  // finer level's smooth error.
  double train_step(mpde_net* net, int l, unsigned seed, double lr, double* loss_plain) {
    net_setup(l);
    NetScratch& S = P->ns;
    Level& L = P->lv[l];
    Level& F = P->lv[l - 1];
    const Table& tf = F.smooth;             // finer-level points of the instances that reach level l
    sample_residuals(l, seed);              // F.r = pre-smoothed finer residual, L.b = R F.r
    // plain coarse correction v = V_l(b) into a scratch level vector
    TV* v = (TV*)S.dB;                      // FP32 scratch, >= L.npts entries
    const bool keep = use_net;
    use_net = false;
    vcycle(l, V(L.b), v);
    use_net = keep;
    level_norms(l, V(L.b));
    int nb_inst = 0;
    for (int b = 0; b < P->B; ++b) nb_inst += L.h[b].N > 0;
    // finer-level energy of the unit-scaled coarse correction o (level l
    // vector); with dOut, also the network's output gradient
    auto fine_energy = [&](TV* o, double* loss, float* dOut) {
      launch_fill<TV>(st, tf.d, tf.nb(), F.d, V(F.dd), (TV)0);
      launch_prolong_add<TV>(D, st, tf.d, tf.nb(), F.d, L.d, o, V(F.dd));       // p = P o
      apply(l - 1, tf, V(F.dd), V(F.x), G_STORE, nullptr);                       // S_f p
      energy_grad_launch(st, tf.d, tf.nb(), F.d, (const float*)F.dd, (const float*)F.x, (const float*)F.r, S.inv,
                         (const float*)F.dinv, 1.0f, nullptr, P->partial);
      finish(tf, loss);
      if (dOut) {
        fine_resid_launch(st, tf.d, tf.nb(), F.d, (const float*)F.x, (const float*)F.r, S.inv, (float*)F.dd);
        launch_restrict<TV>(D, st, L.all.d, L.all.nb(), F.d, L.d, V(F.dd), V(L.r));   // R (S_f p - rhat)
        grad_out_launch(st, L.all.d, L.all.nb(), L.d, (const float*)L.r, (const float*)L.dinv, 1.0f / nb_inst,
                        dOut);
      }
    };
    // reference: the plain correction
    scale_vec_launch(st, L.all.d, L.all.nb(), L.d, (const float*)v, S.inv, (float*)L.dd);
    fine_energy(V(L.dd), P->rzp, nullptr);
    // learned correction
    features_launch(st, L.all.d, L.all.nb(), L.d, P->K, (const float*)L.b, (const float*)v, (const float*)L.dinv,
                    S.inv, (const float*)L.coef, S.X0);
    net_forward(net);
    predict_launch(st, L.all.d, L.all.nb(), L.d, S.Y3, (const float*)v, (const float*)L.dinv, S.inv, (float*)L.dd);
    fine_energy(V(L.dd), P->rz, S.dA);
    std::vector<double> lossb(P->B), lossp(P->B);
    HIPCHK(hipMemcpyAsync(lossb.data(), P->rz, P->B * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(lossp.data(), P->rzp, P->B * sizeof(double), hipMemcpyDeviceToHost, st));
    // backward through the three layers
    const long long n16 = S.npts * 16;
    float* gw = net->g;
    const unsigned short* Wt = net->wtb;
    to_bf16_launch(st, S.dA, n16, S.Db);                                              // dY3
    conv_wgrad_launch(st, S.ntiles, S.tiles, S.grids, S.A2, S.Db, net->partial, gw + 2 * kLayerP);
    bias_grad_launch(st, S.dA, S.npts, gw + 2 * kLayerP + kLayerW);
    conv_launch(st, S.ntiles, S.tiles, S.grids, S.Db, Wt + 2 * kLayerW, nullptr, -1, S.dB, nullptr, 0);
    relu_bwd_launch(st, S.dB, S.P2, n16, S.dA, S.Db);                                 // dpre2
    conv_wgrad_launch(st, S.ntiles, S.tiles, S.grids, S.A1, S.Db, net->partial, gw + kLayerP);
    bias_grad_launch(st, S.dA, S.npts, gw + kLayerP + kLayerW);
    conv_launch(st, S.ntiles, S.tiles, S.grids, S.Db, Wt + kLayerW, nullptr, -1, S.dB, nullptr, 0);
    relu_bwd_launch(st, S.dB, S.P1, n16, S.dA, S.Db);                                 // dpre1
    conv_wgrad_launch(st, S.ntiles, S.tiles, S.grids, S.X0, S.Db, net->partial, gw);
    bias_grad_launch(st, S.dA, S.npts, gw + kLayerW);
    net->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    adam_launch(st, net->w, gw, net->m, net->v, 3 * kLayerP, (float)lr, b1, b2, 1e-8f,
                1.f - std::pow(b1, (float)net->t), 1.f - std::pow(b2, (float)net->t));
    for (int k = 0; k < 3; ++k)
      pack_weights_launch(st, net->w + k * kLayerP, net->wb + k * kLayerW, net->wtb + k * kLayerW);
    HIPCHK(hipStreamSynchronize(st));
    double tot = 0, totp = 0;
    for (int b = 0; b < P->B; ++b)
      if (L.h[b].N > 0) { tot += lossb[b]; totp += lossp[b]; }
    if (loss_plain) *loss_plain = totp / std::max(1, nb_inst);
    return tot / std::max(1, nb_inst);
  }

  TV* V(void* p) { return (TV*)p; }
  TC* C(void* p) { return (TC*)p; }

  void finish(const Table& t, double* out) { launch_finish_sum(st, P->partial, t.d_bstart, P->B, out); }
  // finish(t, out), then the PCG scalar update `op` from that sum (one launch)
  void finish_scalars(const Table& t, double* out, int op, bool first) {
    launch_finish_scalars(st, P->partial, t.d_bstart, P->B, out, op, first ? 1 : 0, P->itol2, P->rz, P->beta, P->alpha,
                          P->r0n2, P->active, P->iters);
  }
  // Descriptors to launch with: the gated copy inside the Krylov iterations.
  bool gate = false;
  const LInst* LD(const Level& L) const { return gate ? L.dg : L.d; }

  // Profiling of finest-grid kernels: kind 0 = gamma, 1 = gather, 2 = fused
  // three-axis operator.  Bytes are
  // algorithmic: every input element read once, every output written once.
  hipEvent_t pa = nullptr;
  bool prof(int l) const { return P->opt.profile && l == 0; }
  void pbeg(int l) {
    if (!prof(l)) return;
    pa = P->ev();
    if (pa) (void)hipEventRecord(pa, st);
  }
  void pend(int l, int kind, const Table& t, int mode) {
    if (!prof(l) || !pa) return;
    hipEvent_t pb = P->ev();
    if (!pb) return;
    (void)hipEventRecord(pb, st);
    precord(kind, pa, pb, t, mode);
    pa = nullptr;
  }
  void precord(int kind, hipEvent_t a, hipEvent_t b, const Table& t, int mode) {
    const double p = sizeof(TV), K = P->K;
    double per;
    if (kind == 2) {                                        // fused: no gamma round trip
      if (mode == G_CHEB) per = (7 + K) * p;                // d, c, x, r, dinv in; x, r, d' out
      else if (mode == G_RESID) per = (5 + K) * p;          // u, c, b, dinv in; r, d out
      else per = (2 + K) * p;                               // u, c in; y out
    } else if (kind == 0) per = (2 + K) * p;                // u, c in; gamma out
    else if (mode == G_CHEB) per = (8 + K) * p;             // d, gamma, c, x, r, dinv in; x, r, d' out
    else if (mode == G_RESID) per = (6 + K) * p;            // u, gamma, c, b, dinv in; r, d out
    else per = (3 + K) * p;                                 // u, gamma, c in; y out
    P->recs.push_back({kind, a, b, per * (double)t.npts});
  }
  void collect() {
    if (!P->opt.profile) return;
    HIPCHK(hipStreamSynchronize(st));
    std::snprintf(P->kst[0].name, 32, "gamma");
    std::snprintf(P->kst[1].name, 32, "gather");
    std::snprintf(P->kst[2].name, 32, "apply3");
    for (auto& k : P->kst) { k.launches = 0; k.ms = 0; k.bytes = 0; }
    for (auto& r : P->recs) {
      float ms = 0;
      if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) continue;
      P->kst[r.kind].launches += 1;
      P->kst[r.kind].ms += ms;
      P->kst[r.kind].bytes += r.bytes;
    }
    P->recs.clear();
    P->pool_used = 0;
  }

  // Fused three-axis operator for table t of level l, or null when the
  // two-pass kernels must be used (other shapes, FP64, option off).
  const FTab* fused(int l, const Table& t) {
    if constexpr (!(std::is_same<TV, float>::value && std::is_same<TC, float>::value)) {
      return nullptr;
    } else {
      if (!P->opt.fused) return nullptr;
      Level& L = P->lv[l];
      const FTab* f = (&t == &L.all) ? &L.fall : (&t == &L.smooth) ? &L.fsmooth : nullptr;
      return (f && f->ok) ? f : nullptr;
    }
  }

  // One operator pass y = S u over table t with the epilogue of `mode`
  // (GatherMode; vectors as for launch_gather).
  void op(int l, const Table& t, TV* u, int mode, TV* out, const TV* b, TV* x, TV* r, TV* d, int cheb_step,
          double* partial) {
    Level& L = P->lv[l];
    if (const FTab* f = fused(l, t)) {
      if constexpr (std::is_same<TV, float>::value && std::is_same<TC, float>::value) {
        // timed launches carry their events in the dispatch itself
        hipEvent_t e0 = prof(l) ? P->ev() : nullptr, e1 = prof(l) ? P->ev() : nullptr;
        launch_apply3<float, float, float>(st, f->d, f->nb(), f->g, LD(L), P->ci, u, C(L.coef), mode, out, b, x, r, d,
                                           V(L.dinv), cheb_step, partial, e0, e1);
        if (e0 && e1) precord(2, e0, e1, t, mode);
      }
      return;
    }
    pbeg(l);
    launch_gamma<TV, TV, TC>(D, st, t.d, t.nb(), LD(L), P->ci, u, C(L.coef), C(P->f), 0, V(L.gam));
    pend(l, 0, t, 0);
    pbeg(l);
    launch_gather<TV, TV, TC>(D, st, t.d, t.nb(), LD(L), P->ci, u, V(L.gam), C(L.coef), C(P->w), 0, mode, out, b, x,
                              r, d, V(L.dinv), cheb_step, partial);
    pend(l, 1, t, mode);
  }

  // `reps` back-to-back operator passes on level 0 in `mode`, between two
  // events; mean microseconds per pass and algorithmic bytes per pass.
  void time_operator(int mode, int reps, double& us, double& bytes) {
    Level& L = P->lv[0];
    const Table& t = L.all;
    hipEvent_t a, b;
    HIPCHK(hipEventCreate(&a));
    HIPCHK(hipEventCreate(&b));
    launch_hash_fill<TV>(st, t.d, t.nb(), L.d, V(L.dd), 777u);
    launch_hash_fill<TV>(st, t.d, t.nb(), L.d, V(L.dd2), 778u);
    launch_hash_fill<TV>(st, t.d, t.nb(), L.d, V(L.x), 779u);
    launch_hash_fill<TV>(st, t.d, t.nb(), L.d, V(L.r), 780u);
    // mode 4: the FP64 residual pass of the outer refinement
    const FTab& f64 = L.fall64;
    if (mode == 4) {
      if (!std::is_same<TC, float>::value || !P->opt.fused || !f64.ok)
        throw std::string("time_operator: this problem has no fused FP64 residual pass");
      launch_hash_fill<double>(st, t.d, t.nb(), L.d, P->u64, 781u);
      launch_hash_fill<double>(st, t.d, t.nb(), L.d, P->rhs64, 782u);
    }
    auto one = [&](int k) {
      TV* cur = V((k & 1) ? L.dd2 : L.dd);
      TV* nxt = V((k & 1) ? L.dd : L.dd2);
      if (mode == 4) {
        if constexpr (std::is_same<TC, float>::value)
          launch_apply3<double, double, float>(st, f64.d, f64.nb(), f64.g, L.d, P->ci, P->u64, C(L.coef), G_RESID,
                                               P->r64, P->rhs64, nullptr, nullptr, nullptr, nullptr, 0, nullptr);
      } else if (mode == G_CHEB) op(0, t, cur, G_CHEB, nullptr, nullptr, V(L.x), V(L.r), nxt, k & 1, nullptr);
      else if (mode == G_RESID) op(0, t, cur, G_RESID, nxt, V(L.x), nullptr, nullptr, V(L.r), 0, nullptr);
      else op(0, t, cur, mode, nxt, nullptr, nullptr, nullptr, nullptr, 0, P->partial);
    };
    one(0);   // warm
    HIPCHK(hipEventRecord(a, st));
    for (int k = 0; k < reps; ++k) one(k);
    HIPCHK(hipEventRecord(b, st));
    HIPCHK(hipEventSynchronize(b));
    float ms = 0;
    HIPCHK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    us = 1e3 * ms / reps;
    const double p = sizeof(TV), K = P->K;
    const bool f = fused(0, t) != nullptr;
    // fused: as in precord(); two-pass: the gamma pass (2 + K) plus the gather
    // mode 4: u, rhs, r in FP64 and the FP32 coefficients
    const double per = mode == 4 ? 24 + 4 * K
                       : mode == G_CHEB ? (f ? 7 + K : 10 + 2 * K) * p
                       : mode == G_RESID ? (f ? 5 + K : 8 + 2 * K) * p
                                         : (f ? 2 + K : 5 + 2 * K) * p;
    bytes = per * (double)t.npts;
  }

  // y = S u on level l for the instances of table t.
  void apply(int l, const Table& t, TV* u, TV* out, int mode, double* partial) {
    op(l, t, u, mode, out, nullptr, nullptr, nullptr, nullptr, 0, partial);
  }

  // out = S u and the per-instance dot products u.out into dots[B].
  void apply_dot(int l, const Table& t, TV* u, TV* out, double* dots) {
    op(l, t, u, G_STORE_DOT, out, nullptr, nullptr, nullptr, nullptr, 0, P->partial);
    const FTab* f = fused(l, t);
    launch_finish_sum(st, P->partial, f ? f->d_bstart : t.d_bstart, P->B, dots);
  }

  // nu Chebyshev steps; the search direction is double-buffered (dd / dd2):
  // each step reads d at stencil neighbours, so the new direction must go to
  // the other buffer.  The start direction is in dd.
  void chebyshev(int l, TV* x, int nu) {
    Level& L = P->lv[l];
    for (int s = 0; s < nu; ++s) {
      TV* cur = V((s & 1) ? L.dd2 : L.dd);
      TV* nxt = V((s & 1) ? L.dd : L.dd2);
      op(l, L.smooth, cur, G_CHEB, nullptr, nullptr, x, V(L.r), nxt, s, nullptr);
    }
  }

  // x = V-cycle(b) on level l (x and b are level-l vectors).  `started`:
  // the Chebyshev start vectors of level l (x = 0, r = b, d) were written by
  // the restriction that produced b.
  void vcycle(int l, TV* b, TV* x, bool started = false) {
    Level& L = P->lv[l];
    const int nu = P->opt.nu;
    if (!L.cinst64.empty())
      launch_bb_solve64<TV>(st, (int)L.cinst64.size(), L.d_cinst64, LD(L), V(P->Sinv), b, x);
    if (!L.cinst16.empty())
      launch_bb_solve16<TV>(st, (int)L.cinst16.size(), L.d_cinst16, LD(L), V(P->Sinv), b, x);
    if (!L.cinstg.empty()) launch_bb_solve<TV>(st, (int)L.cinstg.size(), L.d_cinstg, LD(L), V(P->Sinv), b, x);
    if (L.smooth.nb() == 0) return;
    const Table& t = L.smooth;
    if (!started) launch_cheb_init<TV>(st, t.d, t.nb(), LD(L), b, V(L.dinv), x, V(L.r), V(L.dd));
    chebyshev(l, x, nu);
    Level& Cc = P->lv[l + 1];
    launch_restrict<TV>(D, st, Cc.all.d, Cc.all.nb(), LD(L), LD(Cc), V(L.r), V(Cc.b), V(Cc.dinv), V(Cc.x), V(Cc.r),
                        V(Cc.dd));
    if (use_net && P->net && l + 1 == P->net_level) learned(l + 1, V(Cc.b), V(Cc.x));
    else vcycle(l + 1, V(Cc.b), V(Cc.x), true);
    launch_prolong_add<TV>(D, st, t.d, t.nb(), LD(L), LD(Cc), V(Cc.x), x);
    op(l, t, x, G_RESID, V(L.r), b, nullptr, nullptr, V(L.dd), 0, nullptr);
    chebyshev(l, x, nu);
  }

  // After z = V(r): p = z + beta p and q = S p, per-instance p.q into pq.
  // S z is r - r_V with r_V = r - S z the V-cycle's final level-0 residual
  // (its Chebyshev steps keep it); instances solved exactly on level 0 have
  // S z = r, so their r_V is zero.  This replaces an operator pass per
  // iteration by a recurrence q = S z + beta q (algebraically S p).
  void update_pq() {
    Level& L0 = P->lv[0];
    const Table& t = L0.all;
    if (L0.dense.nb() > 0) launch_fill<TV>(st, L0.dense.d, L0.dense.nb(), L0.d, V(L0.r), (TV)0);
    launch_update_pq<TV>(st, t.d, t.nb(), LD(L0), P->beta, V(P->zk), V(P->rk), V(L0.r), V(P->pk), V(P->qk),
                         P->partial);
    finish_scalars(t, P->pq, 1, false);   // alpha = rz / pq
  }

  // One PCG iteration (plain V-cycle preconditioner, no host interaction).
  void pcg_iter(bool first) {
    Level& L0 = P->lv[0];
    const Table& t = L0.all;
    vcycle(0, V(P->rk), V(P->zk), !first);   // after the first iteration update_xr wrote the start
    launch_dot<double, TV>(st, t.d, t.nb(), LD(L0), V(P->rk), V(P->zk), P->partial);
    finish_scalars(t, P->rz_new, 0, first);
    update_pq();
    launch_update_xr<TV>(st, t.d, t.nb(), LD(L0), P->alpha, V(P->pk), V(P->qk), V(P->e), V(P->rk), P->partial,
                         V(L0.dinv), V(P->zk), V(L0.r), V(L0.dd));
    finish_scalars(t, P->rn2, 2, false);
  }

  // Run `chunk` iterations through a captured graph (captured on first use
  // for this (nu, chunk) and replayed afterwards; the tolerances are read
  // from the device).
  void pcg_chunk_graph(int which, int chunk) {
    const int key = (P->opt.nu * 1000 + chunk) * 2 + which;
    if (!P->gst) {
      P->gst = stream_get();
      HIPCHK(hipEventCreateWithFlags(&P->gev[0], hipEventDisableTiming));
      HIPCHK(hipEventCreateWithFlags(&P->gev[1], hipEventDisableTiming));
    }
    if (P->gexec[which] && P->gkey[which] != key) {
      (void)hipGraphExecDestroy(P->gexec[which]);
      P->gexec[which] = nullptr;
    }
    HIPCHK(hipEventRecord(P->gev[0], st));
    HIPCHK(hipStreamWaitEvent(P->gst, P->gev[0], 0));
    if (!P->gexec[which]) {
      hipStream_t keep = st;
      st = P->gst;
      HIPCHK(hipStreamBeginCapture(P->gst, hipStreamCaptureModeThreadLocal));
      for (int k = 0; k < chunk; ++k) pcg_iter(which == 0 && k == 0);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(P->gst, &g);
      st = keep;
      if (e != hipSuccess) throw HipError{e, "hipStreamEndCapture"};
      e = hipGraphInstantiate(&P->gexec[which], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) throw HipError{e, "hipGraphInstantiate"};
      P->gkey[which] = key;
    }
    HIPCHK(hipGraphLaunch(P->gexec[which], P->gst));
    HIPCHK(hipEventRecord(P->gev[1], P->gst));
    HIPCHK(hipStreamWaitEvent(st, P->gev[1], 0));
  }

  // PCG on S e = rk (level 0), e = 0 start; instances with active=0 stay frozen.
  // Inner Krylov solve: instance b stops once its residual fell by the
  // factor whose square P->itol2[b] holds.
  void pcg(int max_it) {
    Level& L0 = P->lv[0];
    const Table& t = L0.all;
    const int B = P->B;
    launch_fill<TV>(st, t.d, t.nb(), L0.d, V(P->e), 0.0);
    launch_fill<TV>(st, t.d, t.nb(), L0.d, V(P->pk), 0.0);
    launch_fill<TV>(st, t.d, t.nb(), L0.d, V(P->qk), 0.0);
    if (P->net) launch_fill<TV>(st, t.d, t.nb(), L0.d, V(P->zp), 0.0);
    launch_dot<double, TV>(st, t.d, t.nb(), L0.d, V(P->rk), V(P->rk), P->partial);
    finish(t, P->r0n2);
    // the iterations (and the graphs captured from them) launch with the
    // gated descriptors: instances that have converged are skipped
    struct GateOn {
      bool& g;
      explicit GateOn(bool& x) : g(x) { g = true; }
      ~GateOn() { g = false; }
    } gate_on(gate);
    const double* tol2 = P->itol2;
    std::vector<int> act(B);
    const int chunk = std::max(1, P->opt.check_every);
    if (P->opt.graph && !P->opt.profile && !P->net) {
      for (int it = 0; it < max_it; it += chunk) {
        pcg_chunk_graph(it == 0 ? 0 : 1, chunk);
        HIPCHK(hipMemcpyAsync(act.data(), P->active, B * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool any = false;
        for (int b = 0; b < B; ++b) any |= act[b] != 0;
        if (!any) break;
      }
      return;
    }
    const bool flex = P->net != nullptr;
    bool use_net_solve = flex;
    std::vector<double> rzh(B), rn_prev(B, 0.0);
    HIPCHK(hipMemcpyAsync(rn_prev.data(), P->r0n2, B * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int it = 0; it < max_it; ++it) {
      use_net = use_net_solve;
      vcycle(0, V(P->rk), V(P->zk), it > 0);   // after the first iteration update_xr wrote the start
      launch_dot<double, TV>(st, t.d, t.nb(), LD(L0), V(P->rk), V(P->zk), P->partial);
      if (flex) finish(t, P->rz_new);
      else finish_scalars(t, P->rz_new, 0, it == 0);
      if (flex) {
        // Guard: a learned correction that is not a descent direction for
        // some active instance is replaced by the plain V-cycle.
        HIPCHK(hipMemcpyAsync(rzh.data(), P->rz_new, B * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(act.data(), P->active, B * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool bad = false;
        for (int b = 0; b < B; ++b) bad |= act[b] && !(rzh[b] > 0);
        if (bad) {
          P->fallbacks += 1;
          use_net = false;
          vcycle(0, V(P->rk), V(P->zk));
          launch_dot<double, TV>(st, t.d, t.nb(), L0.d, V(P->rk), V(P->zk), P->partial);
          finish(t, P->rz_new);
        }
        use_net = use_net_solve;
        // Polak-Ribiere (flexible) beta: (r.z - r.z_prev) / r_prev.z_prev
        launch_dot<double, TV>(st, t.d, t.nb(), L0.d, V(P->rk), V(P->zp), P->partial);
        finish(t, P->rzp);
        launch_pcg_scalars(st, 3, B, it == 0, tol2, P->rz_new, P->rz, P->beta, P->rzp, P->alpha, P->rn2, P->r0n2,
                           P->active, P->iters);
        launch_copy_scale<TV, TV>(st, t.d, t.nb(), L0.d, V(P->zk), V(P->zp), nullptr, 0);
      }
      update_pq();
      launch_update_xr<TV>(st, t.d, t.nb(), LD(L0), P->alpha, V(P->pk), V(P->qk), V(P->e), V(P->rk), P->partial,
                         V(L0.dinv), V(P->zk), V(L0.r), V(L0.dd));
      finish_scalars(t, P->rn2, 2, false);
      if (flex && use_net_solve && (it + 1) % 5 == 0) {
        // Stagnation guard: if the learned correction reduced the residual
        // more slowly than 0.8 per iteration over the last 5 iterations for
        // any active instance, finish this solve with the plain V-cycle.
        std::vector<double> rn(B);
        HIPCHK(hipMemcpyAsync(rn.data(), P->rn2, B * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPCHK(hipMemcpyAsync(act.data(), P->active, B * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool slow = false;
        for (int b = 0; b < B; ++b)
          if (act[b] && rn_prev[b] > 0 && rn[b] > 0.8 * 0.8 * 0.8 * 0.8 * 0.8 * 0.8 * 0.8 * 0.8 * 0.8 * 0.8 * rn_prev[b])
            slow = true;
        rn_prev = rn;
        if (slow) { use_net_solve = false; P->fallbacks += 1; }
      }
      if ((it + 1) % std::max(1, P->opt.check_every) == 0 || it + 1 == max_it) {
        HIPCHK(hipMemcpyAsync(act.data(), P->active, B * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        bool any = false;
        for (int b = 0; b < B; ++b) any |= act[b] != 0;
        if (!any) break;
      }
    }
  }

  // FP64 residual r64 = rhs - S u64 on level 0, and ||r64||^2 per instance
  // into rn2 (adjoint: rhs = ghat, sigma = 0; forward: sigma = 1, rhs = g).
  // The forward right side A_u^T Pi d is the residual at u = 0: the first
  // residual of a solve (zero_u) is the operator pass with the right-side
  // terms and is kept in rhs64; later ones, and every adjoint one, are the
  // pass r = rhs - S u.  One fused FP64 pass where the level has a fused
  // tile table, else the two-pass kernels.
  void residual64(bool adjoint, double* u64, bool zero_u) {
    Level& L0 = P->lv[0];
    const Table& t = L0.all;
    const FTab& f = L0.fall64;
    const bool first = !adjoint && zero_u;
    bool done = false;
    if constexpr (std::is_same<TC, float>::value) {
      if (P->opt.fused && f.ok) {
        launch_apply3<double, double, float>(st, f.d, f.nb(), f.g, L0.d, P->ci, u64, C(L0.coef), G_RESID, P->r64,
                                             adjoint ? P->ghat : (first ? nullptr : P->rhs64), nullptr, nullptr,
                                             nullptr, nullptr, 0, nullptr, nullptr, nullptr,
                                             first ? C(P->f) : nullptr, first ? C(P->w) : nullptr);
        done = true;
      }
    }
    if (!done) {
      launch_gamma<double, double, TC>(D, st, t.d, t.nb(), L0.d, P->ci, u64, C(L0.coef), C(P->f), adjoint ? 0 : 1,
                                       P->g64);
      launch_gather<double, double, TC>(D, st, t.d, t.nb(), L0.d, P->ci, u64, P->g64, C(L0.coef), C(P->w),
                                        adjoint ? 0 : 1, G_RESID, P->r64, adjoint ? P->ghat : nullptr, nullptr,
                                        nullptr, nullptr, nullptr, 0, nullptr);
    }
    if (first)
      HIPCHK(hipMemcpyAsync(P->rhs64, P->r64, (size_t)L0.npts * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_dot<double, double>(st, t.d, t.nb(), L0.d, P->r64, P->r64, P->partial);
    finish(t, P->rn2);
  }

  // Outer refinement; returns the code; fills info arrays.
  int refine(bool adjoint, double* u64, const double* norm2, mpde_info* info) {
    Level& L0 = P->lv[0];
    const Table& t = L0.all;
    const int B = P->B;
    std::vector<double> rn(B), nb(B);
    std::vector<int> outer(B, 0), status(B, MPDE_STATUS_NOT_CONVERGED), itv(B, 0);
    HIPCHK(hipMemcpyAsync(nb.data(), norm2, B * sizeof(double), hipMemcpyDeviceToHost, st));
    launch_fill<double>(st, t.d, t.nb(), L0.d, u64, 0.0);
    HIPCHK(hipMemsetAsync(P->iters, 0, B * sizeof(int), st));
    // Relative reduction asked of each inner solve: inner_tol if the caller
    // set it; otherwise what instance b still needs, 0.3 tol / relres_b (a
    // factor 3 of margin), at most 0.1 and at least a floor: in FP32 the
    // larger of 1e-4 (what the FP32 recurrence resolves reliably) and
    // sqrt(0.3 tol), so that two outer steps share the reduction instead
    // of the first one overshooting it; in FP64 1e-10.
    const double rho_min = P->dtype == MPDE_F32 ? std::max(1e-4, std::sqrt(0.3 * P->opt.tol)) : 1e-10;
    std::vector<double> relres(B, 1.0), sc(B), isc(B), it2(B);
    std::vector<int> act(B);
    int code = MPDE_WARN_NOT_CONVERGED;
    for (int k = 0; k <= P->opt.max_outer; ++k) {
      residual64(adjoint, u64, k == 0);
      HIPCHK(hipMemcpyAsync(rn.data(), P->rn2, B * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool all = true;
      for (int b = 0; b < B; ++b) {
        const double den = nb[b] > 0 ? std::sqrt(nb[b]) : 1.0;
        relres[b] = std::sqrt(rn[b]) / den;
        if (!std::isfinite(relres[b])) status[b] = MPDE_STATUS_NONFINITE;
        else if (relres[b] <= P->opt.tol || rn[b] == 0.0) status[b] = MPDE_STATUS_CONVERGED;
        else status[b] = MPDE_STATUS_NOT_CONVERGED;
        act[b] = status[b] == MPDE_STATUS_NOT_CONVERGED;
        all &= !act[b];
        sc[b] = (rn[b] > 0 && std::isfinite(rn[b])) ? 1.0 / std::sqrt(rn[b]) : 0.0;
        isc[b] = (rn[b] > 0 && std::isfinite(rn[b])) ? std::sqrt(rn[b]) : 0.0;
        double rho = P->opt.inner_tol;
        if (!(rho > 0)) {
          rho = relres[b] > 0 && std::isfinite(relres[b]) ? 0.3 * P->opt.tol / relres[b] : 0.1;
          rho = std::min(0.1, std::max(rho_min, rho));
        }
        it2[b] = rho * rho;
      }
      if (all || k == P->opt.max_outer) { code = all ? MPDE_OK : MPDE_WARN_NOT_CONVERGED; break; }
      for (int b = 0; b < B; ++b) if (act[b]) outer[b] += 1;
      HIPCHK(hipMemcpyAsync(P->scale, sc.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(P->iscale, isc.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(P->itol2, it2.data(), B * sizeof(double), hipMemcpyHostToDevice, st));
      HIPCHK(hipMemcpyAsync(P->active, act.data(), B * sizeof(int), hipMemcpyHostToDevice, st));
      launch_copy_scale<double, TV>(st, t.d, t.nb(), L0.d, P->r64, V(P->rk), P->scale, 0);
      pcg(P->opt.max_inner);
      launch_copy_scale<TV, double>(st, t.d, t.nb(), L0.d, V(P->e), u64, P->iscale, 1);
    }
    HIPCHK(hipMemcpyAsync(itv.data(), P->iters, B * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool nonfinite = false;
    for (int b = 0; b < B; ++b) nonfinite |= status[b] == MPDE_STATUS_NONFINITE;
    if (info) {
      for (int b = 0; b < B; ++b) {
        if (info->iters) info->iters[b] = itv[b];
        if (info->outer) info->outer[b] = outer[b];
        if (info->relres) info->relres[b] = relres[b];
        if (info->status) info->status[b] = status[b];
      }
    }
    if (nonfinite && code == MPDE_OK) code = MPDE_WARN_NOT_CONVERGED;
    return code;
  }

  // ---------------------------------------------------------- build parts
  void setup_level_operators() {
    const int nlevels = (int)P->lv.size();
    for (int l = 0; l < nlevels; ++l) {
      Level& L = P->lv[l];
      launch_diag<TV, TC>(D, st, L.all.d, L.all.nb(), L.d, P->ci, C(L.coef), V(L.dinv));
    }
    // Chebyshev interval: power iteration x <- D^-1 S x (12 steps) and the
    // Rayleigh quotient x^T S x / x^T D x; hi = 1.1 * estimate, lo = hi / 60
    // (the error multigrid leaves is smooth: a low lower end lets the
    // smoother damp part of it too; measured PCG iterations at 64x128x128:
    // 86.8 with hi / 10, 81.8 with hi / 25, 77.5 with hi / 60).
    for (int l = 0; l < nlevels; ++l) {
      Level& L = P->lv[l];
      if (L.smooth.nb() == 0) continue;
      const Table& t = L.smooth;
      launch_hash_fill<TV>(st, t.d, t.nb(), L.d, V(L.x), 12345u + l);
      for (int it = 0; it < 12; ++it) {
        apply(l, t, V(L.x), V(L.r), G_STORE, nullptr);
        launch_mul_dinv<TV>(st, t.d, t.nb(), L.d, V(L.dinv), V(L.r), V(L.x), P->partial);  // partial: x^T D x
      }
      finish(t, P->pq);
      apply_dot(l, t, V(L.x), V(L.r), P->rz);                                               // x^T S x
      std::vector<double> vsv(P->B), vdv(P->B);
      HIPCHK(hipMemcpyAsync(vsv.data(), P->rz, P->B * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(vdv.data(), P->pq, P->B * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      for (int b = 0; b < P->B; ++b) {
        if (L.h[b].N == 0 || L.h[b].coarsest) continue;
        double lam = vdv[b] > 0 ? vsv[b] / vdv[b] : 0.0;
        if (!(lam > 0) || !std::isfinite(lam)) lam = 4.0;
        const double hi = 1.1 * lam, lo = hi / 60.0;
        L.h[b].cheb_theta = 0.5 * (hi + lo);
        L.h[b].cheb_delta = 0.5 * (hi - lo);
      }
      HIPCHK(hipMemcpyAsync(L.d, L.h.data(), L.h.size() * sizeof(LInst), hipMemcpyHostToDevice, st));
      gate_copy(P, L);
      HIPCHK(hipMemcpyAsync(L.dg, L.hg.data(), L.hg.size() * sizeof(LInst), hipMemcpyHostToDevice, st));
    }
  }

  // Coarsest-grid factors.  The re-discretised operator of each instance's
  // coarsest level is block banded in time (plane blocks, |t - t'| <= 4).
  // Its lower band blocks are probed with time-coloured vectors (9 colours
  // per plane point), factored by a block Cholesky in FP64 (diagonal blocks
  // kept as inverses) and stored in the working precision for the block
  // forward/backward substitution of every V-cycle.
  // `overlap` runs on the problem's stream while the factorisation (one
  // block per instance) runs on a side stream; both join before the factor
  // is checked.
  void build_dense(const std::function<void()>& overlap) {
    const int B = P->B;
    constexpr int NCOL = 9;
    std::vector<long long> boff(B, 0), yoff(B, 0);
    long long totb = 0, toty = 0;
    std::vector<int> Tn(B), mn(B);
    for (int b = 0; b < B; ++b) {
      const LInst& q = P->lv[P->nlev[b] - 1].h[b];
      Tn[b] = q.n[0];
      mn[b] = q.N / q.n[0];
      boff[b] = totb; totb += (long long)Tn[b] * 5 * mn[b] * mn[b];
      totb = (totb + 3) & ~3LL;   // 16-byte aligned rows for the vector loads of the solve
      yoff[b] = toty; toty += (long long)std::min(q.n[0], NCOL) * mn[b] * q.N;
    }
    double* LB = dalloc<double>(totb);
    double* U = dalloc<double>(toty);
    double* GM = dalloc<double>(toty);
    double* Y = dalloc<double>(toty);
    int* dfail = dalloc<int>(B);
    // temporaries go back to the cache after the probing (the stream is
    // synchronised below before this scope ends)
    const int dev = cur_device();
    struct Free {
      hipStream_t s;
      std::vector<Block> v;
      ~Free() {
        (void)hipStreamSynchronize(s);
        for (const Block& b : v) dev_put(b.p, b.bytes, b.dev);
      }
    } fr{st, {{LB, totb * sizeof(double), dev}, {U, toty * sizeof(double), dev}, {GM, toty * sizeof(double), dev},
              {Y, toty * sizeof(double), dev}, {dfail, B * sizeof(int), dev}}};
    HIPCHK(hipMemsetAsync(LB, 0, totb * sizeof(double), st));
    HIPCHK(hipMemsetAsync(U, 0, toty * sizeof(double), st));
    HIPCHK(hipMemsetAsync(dfail, 0, B * sizeof(int), st));
    auto upload = [&](const void* h, size_t bytes) {
      void* d = dalloc<char>(bytes);
      fr.v.push_back({d, bytes, dev});
      HIPCHK(hipMemcpyAsync(d, h, bytes, hipMemcpyHostToDevice, st));
      return d;
    };
    auto scratch = [&](size_t bytes) {
      void* d = dalloc<char>(std::max<size_t>(bytes, 1));
      fr.v.push_back({d, std::max<size_t>(bytes, 1), dev});
      return d;
    };
    for (int l = 0; l < (int)P->lv.size(); ++l) {
      Level& L = P->lv[l];
      // probed instances (their coarsest level is l); the probe descriptors,
      // work items and tiles are expanded on the device from these
      std::vector<ProbeSrc> src;
      std::vector<LInst> reps;
      std::vector<long long> mult;
      int ncolor = -1;
      long long nvq = 0, nwk = 0;
      for (int b = 0; b < B; ++b) {
        if (L.h[b].N == 0 || !L.h[b].coarsest) continue;
        const int n = L.h[b].N, plane = mn[b], nc = std::min(L.h[b].n[0], NCOL);
        if (ncolor >= 0 && nc != ncolor)
          throw std::string("mixed time-axis lengths below 9 on one coarsest level are not supported");
        ncolor = nc;
        ProbeSrc sr{};
        sr.b = b;
        sr.plane = plane;
        sr.n = n;
        sr.yoff = yoff[b];
        sr.boff = boff[b];
        sr.pstart = nvq;
        sr.wstart = nwk;
        const long long np = (long long)nc * plane;
        nvq += np;
        nwk += np * ((n + kBlock - 1) / kBlock);
        src.push_back(sr);
        reps.push_back(L.h[b]);
        mult.push_back(np);
      }
      if (src.empty()) continue;
      if (nvq >= (1LL << 31) || nwk >= (1LL << 31)) throw std::string("too many coarsest-grid probes");
      // responses Y = S U of the probe vectors: one fused FP64 pass over the
      // probe instances where the level's shape allows (the tile geometry of
      // each probed instance, repeated for its probes), else the two-pass
      // kernels
      FTab ft;
      std::vector<int2> torg;
      long long ntile = 0;
      bool fusedp = false;
      if constexpr (std::is_same<TC, float>::value) {
        if (P->opt.fused) {
          make_ftab(ft, reps, (int)reps.size(), std::vector<int>(reps.size(), 1), D, kFThreads64, sizeof(double),
                    &mult);
          if (ft.ok) {
            std::vector<std::vector<int2>> org(reps.size());
            for (const FTile& t : ft.h) org[t.inst].push_back(make_int2(t.x0, t.y0));
            for (size_t k = 0; k < src.size(); ++k) {
              src[k].tpp = (int)org[k].size();
              src[k].toff = (int)torg.size();
              src[k].tstart = ntile;
              torg.insert(torg.end(), org[k].begin(), org[k].end());
              ntile += mult[k] * src[k].tpp;
            }
            fusedp = ntile < (1LL << 31);
          }
        }
      }
      auto* dsrc = (ProbeSrc*)upload(src.data(), src.size() * sizeof(ProbeSrc));
      auto* dorg = fusedp ? (int2*)upload(torg.data(), torg.size() * sizeof(int2)) : nullptr;
      auto* dvq = (LInst*)scratch(nvq * sizeof(LInst));
      auto* dpc = (int*)scratch(nvq * sizeof(int));
      auto* dps = (int*)scratch(nvq * sizeof(int));
      auto* dbo = (long long*)scratch(nvq * sizeof(long long));
      auto* dwk = (Work*)scratch(nwk * sizeof(Work));
      auto* dt = fusedp ? (FTile*)scratch(ntile * sizeof(FTile)) : nullptr;
      launch_probe_lists(st, L.d, dsrc, (int)src.size(), nvq, nwk, ntile, dorg, dvq, dpc, dps, dbo, dwk, dt);
      launch_set_probe(st, dvq, dpc, dps, (int)nvq, ncolor, U);
      if (fusedp) {
        if constexpr (std::is_same<TC, float>::value)
          launch_apply3<double, double, float>(st, dt, (int)ntile, ft.g, dvq, P->ci, U, C(L.coef), G_STORE, Y,
                                               nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr);
      } else {
        launch_gamma<double, double, TC>(D, st, dwk, (int)nwk, dvq, P->ci, U, C(L.coef), C(P->f), 0, GM);
        launch_gather<double, double, TC>(D, st, dwk, (int)nwk, dvq, P->ci, U, GM, C(L.coef), C(P->w), 0, G_STORE, Y,
                                          nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr);
      }
      launch_extract_band(st, dwk, (int)nwk, dvq, dpc, dps, dbo, ncolor, Y, LB);
    }
    auto* dboff = (long long*)upload(boff.data(), B * sizeof(long long));
    auto* dT = (int*)upload(Tn.data(), B * sizeof(int));
    auto* dm = (int*)upload(mn.data(), B * sizeof(int));
    P->Sinv = P->alloc<TV>(totb);
    {
      hipStream_t side = stream_get();
      hipEvent_t ev[2];
      for (auto& e : ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      HIPCHK(hipEventRecord(ev[0], st));
      HIPCHK(hipStreamWaitEvent(side, ev[0], 0));
      launch_bb_factor(side, B, LB, dboff, dT, dm, dfail);
      launch_convert_dense<TV>(side, LB, V(P->Sinv), totb);
      HIPCHK(hipEventRecord(ev[1], side));
      overlap();
      HIPCHK(hipStreamWaitEvent(st, ev[1], 0));
      for (auto& e : ev) (void)hipEventDestroy(e);
      stream_put(side, dev);
    }
    std::vector<int> hf(B);
    HIPCHK(hipMemcpyAsync(hf.data(), dfail, B * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int b = 0; b < B; ++b)
      if (hf[b]) throw std::string("coarsest-grid operator of instance " + std::to_string(b) +
                                   " is not positive definite (rank-deficient problem?)");
    for (int l = 0; l < (int)P->lv.size(); ++l) {
      Level& L = P->lv[l];
      L.cinst64.clear();
      L.cinst16.clear();
      L.cinstg.clear();
      for (int b = 0; b < B; ++b)
        if (L.h[b].N && L.h[b].coarsest) {
          L.h[b].doff = boff[b];
          (mn[b] == 64 ? L.cinst64 : mn[b] <= 16 ? L.cinst16 : L.cinstg).push_back(b);
        }
      if (!L.cinst64.empty() || !L.cinst16.empty() || !L.cinstg.empty()) {
        HIPCHK(hipMemcpyAsync(L.d, L.h.data(), L.h.size() * sizeof(LInst), hipMemcpyHostToDevice, st));
        gate_copy(P, L);
        HIPCHK(hipMemcpyAsync(L.dg, L.hg.data(), L.hg.size() * sizeof(LInst), hipMemcpyHostToDevice, st));
      }
      if (!L.cinst16.empty()) {
        L.d_cinst16 = P->alloc<int>(L.cinst16.size());
        HIPCHK(hipMemcpyAsync(L.d_cinst16, L.cinst16.data(), L.cinst16.size() * sizeof(int), hipMemcpyHostToDevice, st));
      }
      if (!L.cinst64.empty()) {
        L.d_cinst64 = P->alloc<int>(L.cinst64.size());
        HIPCHK(hipMemcpyAsync(L.d_cinst64, L.cinst64.data(), L.cinst64.size() * sizeof(int), hipMemcpyHostToDevice, st));
      }
      if (!L.cinstg.empty()) {
        L.d_cinstg = P->alloc<int>(L.cinstg.size());
        HIPCHK(hipMemcpyAsync(L.d_cinstg, L.cinstg.data(), L.cinstg.size() * sizeof(int), hipMemcpyHostToDevice, st));
      }
    }
    HIPCHK(hipStreamSynchronize(st));
  }

  void atd_norm() {
    Level& L0 = P->lv[0];
    launch_atd_norm<TC>(D, st, L0.all.d, L0.all.nb(), L0.d, P->ci, C(L0.coef), C(P->f), C(P->w), P->partial);
    finish(L0.all, P->atd2);
  }

  void alloc_vectors() {
    for (auto& L : P->lv) {
      L.coef = P->alloc<TC>((size_t)P->K * L.npts);
      L.x = P->alloc<TV>(L.npts);
      L.r = P->alloc<TV>(L.npts);
      L.dd = P->alloc<TV>(L.npts);
      L.dd2 = P->alloc<TV>(L.npts);
      L.b = P->alloc<TV>(L.npts);
      L.gam = P->alloc<TV>(L.npts);
      L.dinv = P->alloc<TV>(L.npts);
    }
    const long long n0 = P->lv[0].npts;
    P->f = P->alloc<TC>(n0);
    P->w = P->alloc<TC>(n0);
    P->e = P->alloc<TV>(n0);
    P->rk = P->alloc<TV>(n0);
    P->zk = P->alloc<TV>(n0);
    P->pk = P->alloc<TV>(n0);
    P->qk = P->alloc<TV>(n0);
    P->zp = P->alloc<TV>(n0);
  }

  void coarsen_all() {
    for (int l = 0; l + 1 < (int)P->lv.size(); ++l) {
      Level& L = P->lv[l];
      Level& Cc = P->lv[l + 1];
      launch_coarsen_coef<TC>(D, st, Cc.all.d, Cc.all.nb(), L.d, Cc.d, P->K, C(L.coef), C(Cc.coef));
    }
  }

  template <typename TO>
  void output(TO* z) {
    Level& L0 = P->lv[0];
    launch_output<TC, TO>(D, st, L0.all.d, L0.all.nb(), L0.d, P->ci, P->u64, C(L0.coef), C(P->f), z, P->zoff);
  }

  template <typename TG>
  int adjoint(const TG* gz, TG* gc, TG* gf, TG* gw, mpde_info* info) {
    Level& L0 = P->lv[0];
    const Table& t = L0.all;
    launch_adj_local<TC, TG>(D, st, t.d, t.nb(), L0.d, P->ci, C(L0.coef), gz, P->zoff, P->vloc);
    launch_adj_rhs<TC, TG>(D, st, t.d, t.nb(), L0.d, P->ci, C(L0.coef), gz, P->zoff, P->vloc, P->ghat);
    launch_dot<double, double>(st, t.d, t.nb(), L0.d, P->ghat, P->ghat, P->partial);
    finish(t, P->pq);
    // The adjoint tolerance is relative to ||g^||; keep pq as the norm.
    HIPCHK(hipMemcpyAsync(P->scale, P->pq, P->B * sizeof(double), hipMemcpyDeviceToDevice, st));
    int code = refine(true, P->du64, P->scale, info);
    launch_adj_grad<TC, TG>(D, st, t.d, t.nb(), L0.d, P->ci, C(L0.coef), C(P->f), P->u64, P->du64, gz, P->zoff, gc,
                            gf, gw);
    HIPCHK(hipStreamSynchronize(st));
    return code;
  }
};

}  // namespace

// ================================================================== build
namespace {

int validate(const mpde_desc* d, mpde_options& opt) {
  if (!d) return fail(MPDE_ERR_INVALID_ARG, "descriptor is NULL");
  if (d->dtype != MPDE_F32 && d->dtype != MPDE_F64) return fail(MPDE_ERR_INVALID_ARG, "dtype must be MPDE_F32 or MPDE_F64");
  if (d->ndim != 2 && d->ndim != 3) return fail(MPDE_ERR_UNSUPPORTED, "ndim must be 2 or 3");
  if (d->batch < 1) return fail(MPDE_ERR_INVALID_ARG, "batch must be >= 1");
  if (!d->shape || !d->step) return fail(MPDE_ERR_INVALID_ARG, "shape and step must be non-NULL host arrays");
  if (!d->coeff || !d->rhs || !d->bc_values) return fail(MPDE_ERR_INVALID_ARG, "coeff, rhs and bc_values must be non-NULL");
  const int D = d->ndim, V = 1 + 2 * D;
  if (d->mset == 0 || (d->mset >> V) != 0) return fail(MPDE_ERR_INVALID_ARG, "mset must be nonzero with bits < V = 1+2D");
  for (int a = 0; a < D; ++a) {
    for (int v : {d->bc_lo[a], d->bc_hi[a]})
      if (v < MPDE_BC_NONE || v > MPDE_BC_PERIODIC) return fail(MPDE_ERR_INVALID_ARG, "boundary code out of range");
    if ((d->bc_lo[a] == MPDE_BC_PERIODIC) != (d->bc_hi[a] == MPDE_BC_PERIODIC))
      return fail(MPDE_ERR_INVALID_ARG, "periodic must be set on both faces of an axis");
  }
  for (int b = 0; b < d->batch; ++b) {
    long long N = 1;
    for (int a = 0; a < D; ++a) {
      const int n = d->shape[b * D + a];
      const double s = d->step[b * D + a];
      if (n < 5) return fail(MPDE_ERR_INVALID_ARG, "every axis needs at least 5 points");
      if (!(s > 0) || !std::isfinite(s)) return fail(MPDE_ERR_INVALID_ARG, "steps must be finite and > 0");
      N *= n;
    }
    if (N > (1LL << 30)) return fail(MPDE_ERR_UNSUPPORTED, "instance too large (> 2^30 points)");
  }
  if (d->opts) opt = *d->opts; else mpde_default_options(&opt);
  if (!(opt.tol > 0) || opt.max_outer < 0 || opt.max_inner < 1 || opt.nu < 1 || opt.nu > 16 || opt.coarse_min < 4 ||
      opt.max_levels < 1 || opt.inner_tol < 0 || opt.inner_tol >= 1 || (opt.time_chunks != 0 && opt.time_chunks != 1 && opt.time_chunks != 2 && opt.time_chunks != 4))
    return fail(MPDE_ERR_INVALID_ARG, "invalid options");
  return MPDE_OK;
}

// Level plan of one instance: halve spatial axes (a >= 1) while even and at
// or above the minimum (periodic: coarse_min, else 5); time stays.
void plan(const int* n0, const double* s0, int D, const int* per, const mpde_options& opt,
          std::vector<std::array<int, 3>>& shapes, std::vector<std::array<double, 3>>& steps,
          std::vector<std::array<int, 3>>& halv) {
  std::array<int, 3> n{1, 1, 1}, k{0, 0, 0};
  std::array<double, 3> s{1, 1, 1};
  for (int a = 0; a < D; ++a) { n[a] = n0[a]; s[a] = s0[a]; }
  shapes = {n}; steps = {s}; halv = {k};
  while ((int)shapes.size() < opt.max_levels) {
    long long N = 1;
    for (int a = 0; a < D; ++a) N *= n[a];
    bool any = false;
    for (int a = 1; a < D; ++a) {
      // periodic axes stop at coarse_min, or continue to 4 while the grid is
      // still too large for the dense coarsest solve; others stop at >= 5
      const int lim = per[a] ? (N > kMaxDense ? std::min(4, opt.coarse_min) : opt.coarse_min) : 5;
      if (n[a] % 2 == 0 && n[a] / 2 >= lim) { n[a] /= 2; s[a] *= 2; k[a] += 1; any = true; }
    }
    if (!any) break;
    shapes.push_back(n); steps.push_back(s); halv.push_back(k);
  }
}

template <typename TV, typename TC>
void build_impl(mpde_problem* P, const mpde_desc* d) {
  Solver<TV, TC> S(P);
  hipStream_t st = P->st;
  const int B = P->B, D = P->D;
  int per[3] = {0, 0, 0};
  for (int a = 0; a < D; ++a) per[a] = d->bc_lo[a] == MPDE_BC_PERIODIC;
  // plan
  std::vector<std::vector<std::array<double, 3>>> lsteps(B);
  std::vector<std::vector<std::array<int, 3>>> lhalv(B);
  P->lshape.resize(B);
  P->nlev.resize(B);
  int maxl = 0;
  for (int b = 0; b < B; ++b) {
    plan(d->shape + b * D, d->step + b * D, D, per, P->opt, P->lshape[b], lsteps[b], lhalv[b]);
    P->nlev[b] = (int)P->lshape[b].size();
    maxl = std::max(maxl, P->nlev[b]);
    long long Nc = 1;
    for (int a = 0; a < D; ++a) Nc *= P->lshape[b].back()[a];
    if (Nc / P->lshape[b].back()[0] > 64)
      throw std::string("coarsest spatial plane of instance " + std::to_string(b) + " exceeds 64 points");
    if (Nc > kMaxDense)
      throw std::string("coarsest grid of instance " + std::to_string(b) + " has " + std::to_string(Nc) +
                        " points; the dense coarsest solve supports at most " + std::to_string(kMaxDense) +
                        " (time axis too long or spatial axes not halvable)");
  }
  P->lv.resize(maxl);
  for (int l = 0; l < maxl; ++l) {
    Level& L = P->lv[l];
    L.h.assign(B, LInst{});
    long long off = 0;
    std::vector<int> sel_all(B, 0), sel_smooth(B, 0), sel_dense(B, 0);
    for (int b = 0; b < B; ++b) {
      LInst& q = L.h[b];
      std::memset(&q, 0, sizeof(q));
      for (int a = 0; a < 3; ++a) { q.n[a] = 1; q.wT[a] = q.wC1[a] = q.wC2[a] = 1.0; q.s[a] = 1; q.is1[a] = q.is2[a] = 1; }
      if (l >= P->nlev[b]) continue;
      long long N = 1;
      for (int a = 0; a < D; ++a) {
        q.n[a] = P->lshape[b][l][a];
        q.s[a] = lsteps[b][l][a];
        q.is1[a] = 1.0 / q.s[a];
        q.is2[a] = 1.0 / (q.s[a] * q.s[a]);
        q.per[a] = per[a];
        q.dlo[a] = d->bc_lo[a] == MPDE_BC_DIRICHLET;
        q.dhi[a] = d->bc_hi[a] == MPDE_BC_DIRICHLET;
        const int k = lhalv[b][l][a];
        q.wT[a] = std::ldexp(1.0, -k);
        q.wC1[a] = std::ldexp(1.0, -k);
        q.wC2[a] = std::ldexp(1.0, -2 * k);
        N *= q.n[a];
      }
      int st_ = 1;
      for (int a = D - 1; a >= 0; --a) { q.str[a] = st_; st_ *= q.n[a]; }
      for (int a = 0; a < 3; ++a) {
        // Gram block of the axis rows (T+, T-, C1, C2) for each row class.
        for (int cls = 0; cls < 3; ++cls) {
          const int tp = cls != 2, tm = cls != 1;
          const double wT2 = q.wT[a] * q.wT[a];
          const double g11 = wT2 * (tp + tm) + q.wC1[a] * q.wC1[a];
          const double g12 = wT2 * (tp - tm) * 0.5;
          const double g22 = wT2 * (tp + tm) * 0.25 + q.wC2[a] * q.wC2[a];
          const double det = g11 * g22 - g12 * g12;
          q.gi[a][cls][0] = g22 / det;
          q.gi[a][cls][1] = -g12 / det;
          q.gi[a][cls][2] = g11 / det;
        }
        float* fk = q.fk[a];
        fk[FK_A] = (float)(q.wT[a] * q.wT[a]);
        fk[FK_AH] = (float)(0.5 * q.wT[a] * q.wT[a]);
        fk[FK_B1] = (float)(q.wC1[a] * q.wC1[a]);
        fk[FK_B2] = (float)(q.wC2[a] * q.wC2[a]);
        fk[FK_B1D] = (float)(q.wC1[a] * q.wC1[a] / 12.0);
        fk[FK_B2D] = (float)(q.wC2[a] * q.wC2[a] / 12.0);
        fk[FK_S1] = (float)q.is1[a];
        fk[FK_S2] = (float)q.is2[a];
        fk[FK_G0] = (float)q.gi[a][0][0];
        fk[FK_G0 + 1] = (float)q.gi[a][0][2];
        for (int k = 0; k < 3; ++k) {
          fk[FK_G1 + k] = (float)q.gi[a][1][k];
          fk[FK_G2 + k] = (float)q.gi[a][2][k];
        }
      }
      q.N = (int)N;
      q.coarsest = (l == P->nlev[b] - 1);
      q.ncoarsened = 0;
      if (l > 0)
        for (int a = 0; a < D; ++a) q.ncoarsened += (P->lshape[b][l][a] != P->lshape[b][l - 1][a]);
      q.cheb_theta = 2.2; q.cheb_delta = 1.8;
      q.voff = off;
      q.coff = off * P->K;
      off += N;
      sel_all[b] = 1;
      sel_smooth[b] = !q.coarsest;
      sel_dense[b] = q.coarsest;
    }
    L.npts = off;
    make_table(L.all, L.h, B, sel_all);
    make_table(L.smooth, L.h, B, sel_smooth);
    make_table(L.dense, L.h, B, sel_dense);
    make_ftab(L.fall, L.h, B, sel_all, D, kFThreads, sizeof(float), nullptr, P->opt.time_chunks);
    make_ftab(L.fsmooth, L.h, B, sel_smooth, D, kFThreads, sizeof(float), nullptr, P->opt.time_chunks);
    if (l == 0) make_ftab(L.fall64, L.h, B, sel_all, D, kFThreads64, sizeof(double));
  }
  // device structures (one arena, one copy)
  size_t maxnb = 1;
  Uploads up;
  P->active = P->alloc<int>(B);
  for (auto& L : P->lv) {
    up.add(L.d, L.h.data(), B * sizeof(LInst));
    gate_copy(P, L);
    up.add(L.dg, L.hg.data(), B * sizeof(LInst));
    upload_table(up, L.all); upload_table(up, L.smooth); upload_table(up, L.dense);
    upload_ftab(up, L.fall); upload_ftab(up, L.fsmooth); upload_ftab(up, L.fall64);
    maxnb = std::max(maxnb, L.all.h.size());
    maxnb = std::max(maxnb, (size_t)L.fall.bstart.back());
    if (!L.fall64.bstart.empty()) maxnb = std::max(maxnb, (size_t)L.fall64.bstart.back());   // level 0 only
  }
  S.alloc_vectors();
  const long long n0 = P->lv[0].npts;
  P->partial = P->alloc<double>(maxnb);
  for (double** a : {&P->rz_new, &P->rz, &P->beta, &P->pq, &P->alpha, &P->rn2, &P->r0n2, &P->atd2, &P->scale,
                     &P->iscale, &P->rzp, &P->itol2})
    *a = P->alloc<double>(B);
  P->iters = P->alloc<int>(B);
  P->flag = P->alloc<int>(1);
  P->u64 = P->alloc<double>(n0);
  P->du64 = P->alloc<double>(n0);
  P->r64 = P->alloc<double>(n0);
  P->rhs64 = P->alloc<double>(n0);
  P->g64 = P->alloc<double>(n0);
  P->ghat = P->alloc<double>(n0);
  P->vloc = P->alloc<double>((size_t)2 * D * n0);
  P->zoff_h.resize(B);
  for (int b = 0; b < B; ++b) P->zoff_h[b] = (long long)P->V * P->lv[0].h[b].voff;
  up.add(P->zoff, P->zoff_h.data(), B * sizeof(long long));
  up.commit(P);
  // inputs (caller's device memory, same concatenated layout as level 0)
  HIPCHK(hipMemcpyAsync(P->lv[0].coef, d->coeff, (size_t)P->K * n0 * sizeof(TC), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(P->f, d->rhs, n0 * sizeof(TC), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(P->w, d->bc_values, n0 * sizeof(TC), hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemsetAsync(P->flag, 0, sizeof(int), st));
  launch_nonfinite<TC>(st, (const TC*)P->lv[0].coef, (long long)P->K * n0, P->flag);
  launch_nonfinite<TC>(st, (const TC*)P->f, n0, P->flag);
  launch_nonfinite<TC>(st, (const TC*)P->w, n0, P->flag);
  int hflag = 0;
  HIPCHK(hipMemcpyAsync(&hflag, P->flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hflag) throw 1;   // non-finite input
  S.coarsen_all();
  S.build_dense([&] { S.setup_level_operators(); });
  S.atd_norm();
  HIPCHK(hipStreamSynchronize(st));
}

template <typename TV, typename TC>
int solve_impl(mpde_problem* P, void* z_out, mpde_info* info) {
  Solver<TV, TC> S(P);
  P->recs.clear();
  P->pool_used = 0;
  const int code = S.refine(false, P->u64, P->atd2, info);
  S.collect();
  if (P->opt.out_f64) S.template output<double>((double*)z_out);
  else S.template output<TC>((TC*)z_out);
  HIPCHK(hipStreamSynchronize(P->st));
  P->has_solution = true;
  return code;
}

template <typename TV, typename TC>
int adjoint_impl(mpde_problem* P, const void* gz, void* gc, void* gf, void* gw, mpde_info* info) {
  Solver<TV, TC> S(P);
  return S.template adjoint<TC>((const TC*)gz, (TC*)gc, (TC*)gf, (TC*)gw, info);
}

int hip_fail(const HipError& h) {
  const int code = (h.e == hipErrorOutOfMemory || h.e == hipErrorMemoryAllocation) ? MPDE_ERR_OUT_OF_MEMORY : MPDE_ERR_HIP;
  return fail(code, std::string("HIP error in ") + h.what + ": " + hipGetErrorString(h.e));
}

bool g_stencils_ready = false;

int ensure_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(MPDE_ERR_NO_DEVICE, "no HIP device available");
  if (!g_stencils_ready) {
    double w1[5][5], w2[5][5];
    fd_table(1, w1);
    fd_table(2, w2);
    if (upload_stencils(w1, w2) != hipSuccess) return fail(MPDE_ERR_HIP, "failed to upload stencil weights");
    g_stencils_ready = true;
  }
  return MPDE_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

int mpde_default_options(mpde_options* o) {
  if (!o) return fail(MPDE_ERR_INVALID_ARG, "options pointer is NULL");
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->inner_tol = 0.0;
  o->max_outer = 30;
  o->max_inner = 200;
  o->nu = 2;
  o->coarse_min = 8;
  o->check_every = 2;
  o->max_levels = 16;
  o->graph = 1;
  o->fused = 1;
  return MPDE_OK;
}

const char* mpde_last_error(void) { return g_err.c_str(); }

int mpde_build(const mpde_desc* d, mpde_problem** out) {
  g_err.clear();
  if (!out) return fail(MPDE_ERR_INVALID_ARG, "out pointer is NULL");
  *out = nullptr;
  mpde_options opt;
  int rc = validate(d, opt);
  if (rc) return rc;
  rc = ensure_device();
  if (rc) return rc;
  mpde_problem* P = new (std::nothrow) mpde_problem();
  if (!P) return fail(MPDE_ERR_OUT_OF_MEMORY, "host allocation failed");
  P->dtype = d->dtype; P->D = d->ndim; P->B = d->batch; P->V = 1 + 2 * d->ndim;
  P->mset = d->mset; P->opt = opt; P->st = (hipStream_t)d->stream;
  P->home = cur_device();
  for (int a = 0; a < 3; ++a) { P->bc_lo[a] = d->bc_lo[a]; P->bc_hi[a] = d->bc_hi[a]; }
  int K = 0;
  for (int v = 0; v < 1 + 2 * kMaxD; ++v) P->ci.k[v] = -1;
  for (int v = 0; v < P->V; ++v)
    if (d->mset >> v & 1u) P->ci.k[v] = K++;
  P->ci.K = K; P->K = K;
  try {
    if (P->dtype == MPDE_F32) build_impl<float, float>(P, d);
    else build_impl<double, double>(P, d);
  } catch (const HipError& h) {
    delete P;
    return hip_fail(h);
  } catch (const std::string& m) {
    delete P;
    return fail(MPDE_ERR_UNSUPPORTED, m);
  } catch (int) {
    delete P;
    return fail(MPDE_ERR_NONFINITE, "non-finite value in coeff, rhs or bc_values");
  } catch (const std::bad_alloc&) {
    delete P;
    return fail(MPDE_ERR_OUT_OF_MEMORY, "host allocation failed");
  }
  *out = P;
  return MPDE_OK;
}

int mpde_solve(mpde_problem* p, void* z_out, mpde_info* info) {
  g_err.clear();
  if (!p) return fail(MPDE_ERR_INVALID_ARG, "problem handle is NULL");
  if (!z_out) return fail(MPDE_ERR_INVALID_ARG, "z_out is NULL");
  auto t0 = std::chrono::steady_clock::now();
  int rc;
  try {
    rc = p->dtype == MPDE_F32 ? solve_impl<float, float>(p, z_out, info) : solve_impl<double, double>(p, z_out, info);
  } catch (const HipError& h) {
    return hip_fail(h);
  }
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rc == MPDE_WARN_NOT_CONVERGED) g_err = "at least one instance did not reach the tolerance";
  return rc;
}

int mpde_solve_adjoint(mpde_problem* p, const void* g_z, void* grad_coeff, void* grad_rhs, void* grad_bc,
                       mpde_info* info) {
  g_err.clear();
  if (!p) return fail(MPDE_ERR_INVALID_ARG, "problem handle is NULL");
  if (!g_z) return fail(MPDE_ERR_INVALID_ARG, "g_z is NULL");
  if (!p->has_solution) return fail(MPDE_ERR_BAD_STATE, "mpde_solve must succeed before mpde_solve_adjoint");
  auto t0 = std::chrono::steady_clock::now();
  int rc;
  try {
    rc = p->dtype == MPDE_F32 ? adjoint_impl<float, float>(p, g_z, grad_coeff, grad_rhs, grad_bc, info)
                              : adjoint_impl<double, double>(p, g_z, grad_coeff, grad_rhs, grad_bc, info);
  } catch (const HipError& h) {
    return hip_fail(h);
  }
  if (info) info->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rc == MPDE_WARN_NOT_CONVERGED) g_err = "at least one instance did not reach the tolerance";
  return rc;
}


void mpde_free(mpde_problem* p) { delete p; }

int mpde_net_create(int32_t in_channels, uint64_t seed, mpde_net** out) {
  g_err.clear();
  if (!out) return fail(MPDE_ERR_INVALID_ARG, "out pointer is NULL");
  *out = nullptr;
  if (in_channels < 1 || in_channels > 16) return fail(MPDE_ERR_INVALID_ARG, "in_channels must be 1..16");
  int rc = ensure_device();
  if (rc) return rc;
  mpde_net* n = new (std::nothrow) mpde_net();
  if (!n) return fail(MPDE_ERR_OUT_OF_MEMORY, "host allocation failed");
  n->cin = in_channels;
  try {
    auto al = [&](size_t cnt, size_t sz) {
      void* p = nullptr;
      HIPCHK(hipMalloc(&p, cnt * sz));
      n->owned.push_back(p);
      return p;
    };
    const size_t np = 3 * kLayerP;
    n->w = (float*)al(np, 4); n->g = (float*)al(np, 4); n->m = (float*)al(np, 4); n->v = (float*)al(np, 4);
    n->wb = (unsigned short*)al(3 * kLayerW, 2);
    n->wtb = (unsigned short*)al(3 * kLayerW, 2);
    n->partial = (float*)al((size_t)1024 * kLayerW, 4);
    // He-scaled seeded initialisation (host), biases zero; weights on input
    // channels >= in_channels of the first layer are zero.
    std::vector<float> h(np, 0.f);
    uint64_t st = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto rnd = [&]() {
      st = st * 6364136223846793005ULL + 1442695040888963407ULL;
      uint64_t z = st;
      z ^= z >> 33; z *= 0xff51afd7ed558ccdULL; z ^= z >> 33;
      return ((double)(z >> 11) / 9007199254740992.0) * 2.0 - 1.0;   // U(-1, 1)
    };
    for (int l = 0; l < 3; ++l) {
      const int fan_in = 27 * (l == 0 ? in_channels : 16);
      // the last layer starts at zero, so an untrained network is exactly
      // the plain V-cycle
      const double sc = l == 2 ? 0.0 : std::sqrt(6.0 / fan_in);
      for (int tap = 0; tap < 27; ++tap)
        for (int o = 0; o < 16; ++o)
          for (int i = 0; i < 16; ++i) {
            const bool live = (l > 0 || i < in_channels) && (l < 2 || o == 0);
            h[l * kLayerP + (tap * 16 + o) * 16 + i] = live ? (float)(sc * rnd()) : 0.f;
          }
    }
    HIPCHK(hipMemcpy(n->w, h.data(), np * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(n->m, 0, np * 4));
    HIPCHK(hipMemset(n->v, 0, np * 4));
    for (int k = 0; k < 3; ++k) pack_weights_launch(nullptr, n->w + k * kLayerP, n->wb + k * kLayerW, n->wtb + k * kLayerW);
    HIPCHK(hipDeviceSynchronize());
  } catch (const HipError& h) {
    delete n;
    return hip_fail(h);
  }
  *out = n;
  return MPDE_OK;
}

void mpde_net_free(mpde_net* n) { delete n; }

int mpde_net_get(const mpde_net* n, float* host, int64_t cnt) {
  if (!n || !host || cnt < MPDE_NET_PARAMS) return fail(MPDE_ERR_INVALID_ARG, "bad net/host/size");
  if (hipMemcpy(host, n->w, (size_t)MPDE_NET_PARAMS * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(MPDE_ERR_HIP, "copy failed");
  return MPDE_OK;
}

int mpde_net_set(mpde_net* n, const float* host, int64_t cnt) {
  if (!n || !host || cnt < MPDE_NET_PARAMS) return fail(MPDE_ERR_INVALID_ARG, "bad net/host/size");
  if (hipMemcpy(n->w, host, (size_t)MPDE_NET_PARAMS * 4, hipMemcpyHostToDevice) != hipSuccess)
    return fail(MPDE_ERR_HIP, "copy failed");
  for (int k = 0; k < 3; ++k) pack_weights_launch(nullptr, n->w + k * kLayerP, n->wb + k * kLayerW, n->wtb + k * kLayerW);
  if (hipDeviceSynchronize() != hipSuccess) return fail(MPDE_ERR_HIP, "pack failed");
  return MPDE_OK;
}

int mpde_net_train_step(mpde_net* n, mpde_problem* p, int32_t level, uint64_t seed, double lr, double* loss,
                        double* loss_plain) {
  g_err.clear();
  if (!n || !p) return fail(MPDE_ERR_INVALID_ARG, "net or problem is NULL");
  if (p->dtype != MPDE_F32) return fail(MPDE_ERR_UNSUPPORTED, "the learned correction runs on FP32 problems");
  if (level < 1 || level >= (int)p->lv.size()) return fail(MPDE_ERR_INVALID_ARG, "level must be 1..levels-1");
  if (2 + p->K > 16 || n->cin != 2 + p->K)
    return fail(MPDE_ERR_INVALID_ARG, "network in_channels must equal 2 + number of coefficient fields");
  if (!(lr > 0)) return fail(MPDE_ERR_INVALID_ARG, "lr must be > 0");
  try {
    Solver<float, float> S(p);
    const double l = S.train_step(n, level, (unsigned)(seed * 2654435761u + 17u), lr, loss_plain);
    if (loss) *loss = l;
  } catch (const HipError& h) {
    return hip_fail(h);
  }
  return MPDE_OK;
}

int mpde_net_attach(mpde_problem* p, const mpde_net* n, int32_t level) {
  g_err.clear();
  if (!p) return fail(MPDE_ERR_INVALID_ARG, "problem is NULL");
  if (!n) { p->net = nullptr; return MPDE_OK; }
  if (p->dtype != MPDE_F32) return fail(MPDE_ERR_UNSUPPORTED, "the learned correction runs on FP32 problems");
  if (level < 1 || level >= (int)p->lv.size()) return fail(MPDE_ERR_INVALID_ARG, "level must be 1..levels-1");
  if (n->cin != 2 + p->K) return fail(MPDE_ERR_INVALID_ARG, "network in_channels must equal 2 + K");
  for (int b = 0; b < p->B; ++b)
    if (p->nlev[b] <= level) return fail(MPDE_ERR_UNSUPPORTED, "every instance must have the network's level");
  try {
    Solver<float, float> S(p);
    S.net_setup(level);
  } catch (const HipError& h) {
    return hip_fail(h);
  }
  p->net = n;
  p->net_level = level;
  return MPDE_OK;
}

int mpde_conv3d(const void* x, const void* w, const float* bias, float* y, void* yb, int32_t relu, int32_t sign,
                int32_t batch, int32_t T, int32_t X, int32_t Y, const int32_t* periodic, void* stream) {
  g_err.clear();
  if (!x || !w || (!y && !yb) || !periodic || batch < 1 || T < 1 || X < 1 || Y < 1 || (sign != 1 && sign != -1))
    return fail(MPDE_ERR_INVALID_ARG, "bad conv3d arguments");
  int rc = ensure_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const long long N = (long long)T * X * Y;
  std::vector<mpde::Grid3> g(batch);
  std::vector<int2> tiles;
  for (int b = 0; b < batch; ++b) {
    g[b] = mpde::Grid3{T, X, Y, {periodic[0], periodic[1], periodic[2]}, b * N};
    for (long long s0 = 0; s0 < N; s0 += 16) tiles.push_back(make_int2(b, (int)s0));
  }
  while (tiles.size() % 4) tiles.push_back(make_int2(-1, 0));
  void *dg = nullptr, *dt = nullptr;
  if (hipMalloc(&dg, batch * sizeof(mpde::Grid3)) != hipSuccess || hipMalloc(&dt, tiles.size() * sizeof(int2)) != hipSuccess) {
    (void)hipFree(dg);
    return fail(MPDE_ERR_OUT_OF_MEMORY, "conv3d tables");
  }
  (void)hipMemcpyAsync(dg, g.data(), batch * sizeof(mpde::Grid3), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, st);
  conv_launch(st, (int)tiles.size(), (const int2*)dt, (const mpde::Grid3*)dg, (const unsigned short*)x,
              (const unsigned short*)w, bias, sign, y, (unsigned short*)yb, relu);
  hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(dg);
  (void)hipFree(dt);
  return e == hipSuccess ? MPDE_OK : fail(MPDE_ERR_HIP, hipGetErrorString(e));
}

int mpde_conv3d_wgrad(const void* x, const void* dy, float* dw, int32_t batch, int32_t T, int32_t X, int32_t Y,
                      const int32_t* periodic, void* stream) {
  g_err.clear();
  if (!x || !dy || !dw || !periodic || batch < 1 || T < 1 || X < 1 || Y < 1)
    return fail(MPDE_ERR_INVALID_ARG, "bad conv3d_wgrad arguments");
  int rc = ensure_device();
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  const long long N = (long long)T * X * Y;
  std::vector<mpde::Grid3> g(batch);
  std::vector<int2> tiles;
  for (int b = 0; b < batch; ++b) {
    g[b] = mpde::Grid3{T, X, Y, {periodic[0], periodic[1], periodic[2]}, b * N};
    for (long long s0 = 0; s0 < N; s0 += 16) tiles.push_back(make_int2(b, (int)s0));
  }
  void *dg = nullptr, *dt = nullptr, *part = nullptr;
  if (hipMalloc(&dg, batch * sizeof(mpde::Grid3)) != hipSuccess || hipMalloc(&dt, tiles.size() * sizeof(int2)) != hipSuccess ||
      hipMalloc(&part, (size_t)1024 * kLayerW * 4) != hipSuccess) {
    (void)hipFree(dg);
    (void)hipFree(dt);
    return fail(MPDE_ERR_OUT_OF_MEMORY, "conv3d_wgrad tables");
  }
  (void)hipMemcpyAsync(dg, g.data(), batch * sizeof(mpde::Grid3), hipMemcpyHostToDevice, st);
  (void)hipMemcpyAsync(dt, tiles.data(), tiles.size() * sizeof(int2), hipMemcpyHostToDevice, st);
  conv_wgrad_launch(st, (int)tiles.size(), (const int2*)dt, (const mpde::Grid3*)dg, (const unsigned short*)x,
                    (const unsigned short*)dy, (float*)part, dw);
  hipError_t e = hipStreamSynchronize(st);
  (void)hipFree(dg);
  (void)hipFree(dt);
  (void)hipFree(part);
  return e == hipSuccess ? MPDE_OK : fail(MPDE_ERR_HIP, hipGetErrorString(e));
}

int mpde_autotune(mpde_problem* p, void* z, int32_t* chosen, double* best_ms) {
  g_err.clear();
  if (!p || !z) return fail(MPDE_ERR_INVALID_ARG, "problem or z_scratch is NULL");
  auto timed = [&](double& ms) -> int {
    int rc = 0;
    for (int rep = 0; rep < 2; ++rep) {        // first run captures graphs; time the second
      auto t0 = std::chrono::steady_clock::now();
      try {
        rc = p->dtype == MPDE_F32 ? solve_impl<float, float>(p, z, nullptr) : solve_impl<double, double>(p, z, nullptr);
      } catch (const HipError& h) {
        return hip_fail(h);
      }
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    return rc;
  };
  const mpde_options keep = p->opt;
  double best;
  int rc = timed(best);
  if (rc < 0) return rc;
  if (rc != MPDE_OK) best = 1e300;
  mpde_options cur = p->opt;
  const std::vector<double> tols = p->dtype == MPDE_F32 ? std::vector<double>{1e-2, 1e-3, 1e-4}
                                                         : std::vector<double>{1e-6, 1e-8, 1e-10};
  for (int pass = 0; pass < 3; ++pass) {
    std::vector<mpde_options> cands;
    for (int v : {1, 2, 3, 4}) if (pass == 0) { mpde_options o = cur; o.nu = v; cands.push_back(o); }
    for (double t : tols) if (pass == 1) { mpde_options o = cur; o.inner_tol = t; cands.push_back(o); }
    for (int c : {2, 4, 8, 16}) if (pass == 2) { mpde_options o = cur; o.check_every = c; cands.push_back(o); }
    for (const auto& o : cands) {
      p->opt = o;
      double ms;
      rc = timed(ms);
      if (rc < 0) { p->opt = keep; return rc; }
      if (rc == MPDE_OK && ms < best) { best = ms; cur = o; }
    }
    p->opt = cur;
  }
  p->opt = cur;
  p->opt.tol = keep.tol;
  if (chosen) {
    chosen[0] = cur.nu;
    chosen[1] = cur.check_every;
    chosen[2] = (int32_t)std::lround(cur.inner_tol * 1e9);   // 0: the adaptive default
  }
  if (best_ms) *best_ms = best;
  return MPDE_OK;
}

int mpde_time_operator(mpde_problem* p, int32_t mode, int32_t reps, double* us_per_launch,
                       double* bytes_per_launch) {
  g_err.clear();
  if (!p || !us_per_launch || !bytes_per_launch || mode < 0 || mode > 4 || reps < 1)
    return fail(MPDE_ERR_INVALID_ARG, "mpde_time_operator: bad argument");
  try {
    double us = 0, bytes = 0;
    if (p->dtype == MPDE_F32) {
      Solver<float, float> S(p);
      S.time_operator(mode, reps, us, bytes);
    } else {
      Solver<double, double> S(p);
      S.time_operator(mode, reps, us, bytes);
    }
    *us_per_launch = us;
    *bytes_per_launch = bytes;
    return MPDE_OK;
  } catch (const HipError& h) {
    return hip_fail(h);
  } catch (const std::string& m) {
    return fail(MPDE_ERR_UNSUPPORTED, m);
  }
}

int mpde_kernel_stats(const mpde_problem* p, mpde_kstat* out, int32_t max) {
  if (!p || !p->opt.profile) return 0;
  for (int i = 0; i < 3 && i < max; ++i)
    if (out) out[i] = p->kst[i];
  return 3;
}

int mpde_levels(const mpde_problem* p, int32_t b, int32_t* shapes) {
  if (!p || b < 0 || b >= p->B) return 0;
  const int nl = p->nlev[b];
  if (shapes)
    for (int l = 0; l < nl; ++l)
      for (int a = 0; a < p->D; ++a) shapes[l * p->D + a] = p->lshape[b][l][a];
  return nl;
}

}  // extern "C"
