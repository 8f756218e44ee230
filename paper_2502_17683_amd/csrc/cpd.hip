// C-ABI of libthccp.so: plan set-up, the matrix-free ALS sweep, fit,
// checkpointing, statistics, and the batched (grouped) form.
//
// A plan holds `count` independent CP-ALS problems (a single CPD is a
// batch of one).  Every step of a sweep is ONE grouped launch over all
// problems, driven by argument tables that live in the plan's workspace,
// and a whole sweep is captured once as a hipGraph and replayed.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/thccp.h"
#include "kernels.h"
#include "mixed.h"

namespace thccp {

static const int HIST_CAP = 4096;
static const int SPLIT_KPARTS_MAX = 4;  // split-K slices of the split-BF16 back-projection

static size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Carves a region; with base == nullptr only computes the size.
struct Layout {
  size_t off = 0;
  char* base = nullptr;
  void* take(size_t bytes) {
    void* p = base ? (void*)(base + off) : nullptr;
    off = align_up(off + bytes);
    return p;
  }
};

template <typename T>
struct Bufs {
  const T* X[4];
  const T* Z;
  T* W[4];
  T* Y;
  T* Msol;
  T* Msave;
  T* Mbak;      // right-hand side kept for a damped retry of a fused solve
  T* F[4];
  T* Fsave[4];  // factors at the start of the sweep (fast-path checkpoint)
  T* G[4];
  T* V;
  T* ldiag;
  T* diagL;
  T* lam;
  int32_t* flow;   // ready flags of the dataflow solves
  int32_t* cflow;  // ready flags of the dataflow factorisation
  T* dpart;        // partly updated diagonal blocks of the dataflow factorisation
};

struct Prob {
  cpd_desc d;
  int n[4], Rt, Rc, Tp, nblk, nmax;
  Bufs<double> b64;
  Bufs<float> b32;
  MixedBufs mx;
  DevState* st;
  DevState* st_save;
  double* fit_hist;
  double* inner_part;
  double* row_part;
  double* setup[3];
  double* partials;
  double* norm2;
  double* scratch64;
  float* spart;  // split BF16: split-K partial products of the back-projection (4 x nmax x Tp)
};

// One grouped launch: device table + workgroup prefix sums.
struct GroupOp {
  void* tab = nullptr;   // device: GemmArgs<T>[] / SplitArgs[]
  int* offs = nullptr;   // device: nprob + 1 prefix sums
  int total = 0;
  int count = 0;         // table entries
  int bm = 64;
  bool a_t = false, b_t = false, had = false, apair = false, bpair = false;
  bool wide = false;     // split BF16: bm x 256 tiles (gemm_split_wide_group)
  int kparts = 1;        // split BF16, wide tiles: K slices (split-K) summed by a reduce launch
  int maxm = 0, maxn = 0;
  // split BF16, direct-load 256 x 256 tiles of blocked operands: their own
  // argument table, and the pair splits that form a pair operand first
  bool dma = false;
  void* dtab = nullptr;  // device SplitArgs[] with the blocked operands (null: not available)
  void* ptab = nullptr;  // device PairJob[] (one per problem) or null
  size_t pchunks = 0;    // largest pair split, in 8-element chunks
  void* ttab = nullptr;  // device SplitTArgs[] (blocked transposes, one per problem) or null
  size_t tchunks = 0;
};

// One launch of a blocked solve: a step launch or a grouped panel GEMM.
struct SolveLaunch {
  int mode = -1;          // StepMode, or -1 for the GEMM
  StepCfg cfg{1, -1, 0, -1, 0};
  int* offs = nullptr;    // device, nprob + 1 prefix sums (step launches) or segment table
  int nseg = 0;           // segments of a dataflow launch (0: prefix sums)
  int total = 0;
  GroupOp gemm;
};
// The factorisation and solves of one mode.
struct StepOps {
  void* probs = nullptr;                // StepProb<T>[nprob]
  std::vector<SolveLaunch> cholfwd;     // factorisation fused with the forward solve
  std::vector<SolveLaunch> bwd;         // backward solve
  std::vector<SolveLaunch> chol_retry;  // damped-retry factorisation (retried problems only)
  std::vector<SolveLaunch> fwd_retry;   // forward solve of the retried problems only
  void* mkeep = nullptr;                // CkptArgs: Msol -> Mbak
  void* mrestore = nullptr;             // CkptArgs: Mbak -> Msol for retried problems
};

// Process-wide autotune cache: (kind, shapes) -> tile edge.
static std::mutex g_tune_mu;
// Test override of the split-BF16 launch shape (a SplitCfg code, 0: off);
// applied to every split product of plans built afterwards where that shape
// is available (split-K only where the product allows it).
static int g_split_force = 0;
static std::map<std::string, int> g_tune;

}  // namespace thccp

using namespace thccp;

struct cpd_plan_s {
  int count = 0;
  std::vector<Prob> P;
  int prec = 0;
  int fit_every = 1;
  int allow_fallback = 1;
  int use_graph = 0;
  int autotune = 0;
  double tol = 0.0, fit_floor = 0.0;
  long launched = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  hipGraphExec_t exec[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  bool have_graph = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t tables_off = 0;
  int maxR = 0, maxTp = 0, maxNblk = 0, maxN = 0;
  GroupOp core[4], back[4], gram[4], proj[4];  // FP64 / FP32 MTTKRP, Gram, projection
  GroupOp score[4], sback[4], sproj[4];         // split-BF16 core / back / projection
  void* ftt[4] = {nullptr, nullptr, nullptr, nullptr};  // SplitTArgs per mode
  GroupOp fproj[3], fcore, fback;               // mixed: FP64 mode-3 MTTKRP of fit sweeps
  GroupOp cproj[4];                             // mixed: FP64 projections of just-promoted problems
  void* cond = nullptr;                         // CondArgs<T>[nprob] (precision guard)
  int32_t* forced_dev = nullptr;                // nprob flags: problems promoted to the FP64 path
  std::vector<int32_t> forced;                  // host copy (sticky)
  double cond_limit = 1e5;
  int panel_width = 0;                          // blocks per solve panel; 0: one level
  int tied = 0;                                 // particle-tied model (F1 = F0, F3 = F2)
  bool tie_alias = true;                        // every problem has X1 = X0 and X3 = X2
  void* tie[2] = {nullptr, nullptr};            // CkptArgs: F, G (and W when aliased) n -> n + 1
  void* tinner = nullptr;                       // NormArgs: tied <G, G~> partials
  StepOps steps[4];
  void* formv[4] = {nullptr, nullptr, nullptr, nullptr};
  void* norm[4] = {nullptr, nullptr, nullptr, nullptr};
  void* norm_inner = nullptr;                   // mode 3 with the inner-product partials
  void* fit = nullptr;
  void* ckpt = nullptr;
  void* sts = nullptr;                          // DevState*[nprob]
  DevState* host_states = nullptr;              // pinned, nprob
  std::vector<std::pair<std::string, int>> tune_log;
};

namespace {

#define HIPCHK(x)                             \
  do {                                        \
    hipError_t e_ = (x);                      \
    if (e_ != hipSuccess) return CPD_ERR_HIP; \
  } while (0)

int check_desc(const cpd_desc* d) {
  if (!d) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m) {
    if (d->n[m] <= 0 || !d->X[m] || !d->init[m]) return CPD_ERR_INVALID_ARG;
  }
  if (d->r_thc <= 0 || d->r_cp <= 0 || !d->Z) return CPD_ERR_INVALID_ARG;
  if (d->r_thc > (1 << 20) || d->r_cp > (1 << 16)) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (d->n[m] > (1 << 24)) return CPD_ERR_INVALID_ARG;
  if (d->precision != CPD_FP64 && d->precision != CPD_FP32 && d->precision != CPD_MIXED_BF16)
    return CPD_ERR_INVALID_ARG;
  if (!(d->tol >= 0.0) || !(d->fit_floor >= 0.0) || !(d->fit_target >= 0.0)) return CPD_ERR_INVALID_ARG;
  return CPD_OK;
}

void fill_prob(Prob& q, const cpd_desc* d) {
  memset(&q, 0, sizeof(q));
  q.d = *d;
  for (int m = 0; m < 4; ++m) q.n[m] = d->n[m];
  q.Rt = d->r_thc;
  q.Rc = d->r_cp;
  q.nblk = (d->r_cp + 63) / 64;
  q.Tp = q.nblk * 64;
  q.nmax = 0;
  for (int m = 0; m < 4; ++m)
    if (q.n[m] > q.nmax) q.nmax = q.n[m];
}

template <typename T>
void carve_typed(Layout& L, Prob& q, Bufs<T>& b, bool own_inputs) {
  const int Rt = q.Rt, Tp = q.Tp;
  if (own_inputs) {
    for (int m = 0; m < 4; ++m) {
      int alias = -1;
      for (int r = 0; r < m; ++r)
        if (q.d.X[r] == q.d.X[m]) alias = r;
      b.X[m] = alias >= 0 ? b.X[alias] : (const T*)L.take(sizeof(T) * (size_t)q.n[m] * Rt);
    }
    b.Z = (const T*)L.take(sizeof(T) * (size_t)Rt * Rt);
  }
  for (int m = 0; m < 4; ++m) b.W[m] = (T*)L.take(sizeof(T) * (size_t)Rt * Tp);
  b.Y = (T*)L.take(sizeof(T) * (size_t)Rt * Tp);
  b.Msol = (T*)L.take(sizeof(T) * (size_t)q.nmax * Tp);
  b.Msave = (T*)L.take(sizeof(T) * (size_t)q.n[3] * Tp);
  b.Mbak = (T*)L.take(sizeof(T) * (size_t)q.nmax * Tp);
  for (int m = 0; m < 4; ++m) b.F[m] = (T*)L.take(sizeof(T) * (size_t)q.n[m] * Tp);
  for (int m = 0; m < 4; ++m) b.Fsave[m] = (T*)L.take(sizeof(T) * (size_t)q.n[m] * Tp);
  for (int m = 0; m < 4; ++m) b.G[m] = (T*)L.take(sizeof(T) * (size_t)Tp * Tp);
  b.V = (T*)L.take(sizeof(T) * (size_t)Tp * Tp);
  b.ldiag = (T*)L.take(sizeof(T) * (size_t)q.nblk * 64 * 64);
  b.diagL = (T*)L.take(sizeof(T) * (size_t)Tp);
  b.lam = (T*)L.take(sizeof(T) * (size_t)Tp);
  b.flow = (int32_t*)L.take(sizeof(int32_t) * (size_t)((q.nmax + 63) / 64) * q.nblk);
  b.cflow = (int32_t*)L.take(sizeof(int32_t) * ((size_t)(q.nblk + 2) * q.nblk + CU_SLOTS));
  b.dpart = (T*)L.take(sizeof(T) * (size_t)q.nblk * 64 * 64);
}

// Split-BF16 buffers; X and Z splits are shared between problems (and
// modes) that pass the same input pointer.
typedef std::map<const double*, std::pair<__bf16*, __bf16*>> SplitMap;
struct SplitShare {
  SplitMap x, xt, z, zt, xb, zb, ztb, xtb;
};

void carve_mixed(Layout& L, Prob& q, SplitShare& sh) {
  MixedBufs& mx = q.mx;
  const int Rt = q.Rt, Rc = q.Rc;
  mx.Rtp = (Rt + 31) / 32 * 32;
  mx.npad_max = 0;
  for (int m = 0; m < 4; ++m) {
    mx.npad[m] = (q.n[m] + 31) / 32 * 32;
    if (mx.npad[m] > mx.npad_max) mx.npad_max = mx.npad[m];
  }
  auto pair_for = [&](SplitMap& mp, const double* key, size_t elems) {
    auto it = mp.find(key);
    if (it != mp.end()) return it->second;
    std::pair<__bf16*, __bf16*> v((__bf16*)L.take(2 * elems), (__bf16*)L.take(2 * elems));
    mp[key] = v;
    return v;
  };
  for (int m = 0; m < 4; ++m) {
    auto a = pair_for(sh.x, q.d.X[m], (size_t)q.n[m] * mx.Rtp);
    auto b = pair_for(sh.xt, q.d.X[m], (size_t)Rt * mx.npad[m]);
    mx.Xh[m] = a.first;
    mx.Xl[m] = a.second;
    mx.XTh[m] = b.first;
    mx.XTl[m] = b.second;
  }
  auto z = pair_for(sh.z, q.d.Z, (size_t)Rt * mx.Rtp);
  auto zt = pair_for(sh.zt, q.d.Z, (size_t)Rt * mx.Rtp);
  mx.Zh = z.first;
  mx.Zl = z.second;
  mx.ZTh = zt.first;
  mx.ZTl = zt.second;
  for (int m = 0; m < 4; ++m) mx.WT[m] = (float*)L.take(4 * (size_t)Rc * mx.Rtp);
  mx.YT = (float*)L.take(4 * (size_t)Rc * mx.Rtp);
  mx.FTh = (__bf16*)L.take(2 * (size_t)Rc * mx.npad_max);
  mx.FTl = (__bf16*)L.take(2 * (size_t)Rc * mx.npad_max);
  for (int m = 0; m < 4; ++m) {
    auto xb = pair_for(sh.xb, q.d.X[m], blk_elems(q.n[m], mx.Rtp));
    mx.XBh[m] = xb.first;
    mx.XBl[m] = xb.second;
    auto xtb = pair_for(sh.xtb, q.d.X[m], blk_elems(Rt, mx.npad[m]));
    mx.XTBh[m] = xtb.first;
    mx.XTBl[m] = xtb.second;
  }
  mx.FTBh = (__bf16*)L.take(2 * blk_elems(Rc, mx.npad_max));
  mx.FTBl = (__bf16*)L.take(2 * blk_elems(Rc, mx.npad_max));
  auto zb = pair_for(sh.zb, q.d.Z, blk_elems(Rt, mx.Rtp));
  auto ztb = pair_for(sh.ztb, q.d.Z, blk_elems(Rt, mx.Rtp));
  mx.ZBh = zb.first;
  mx.ZBl = zb.second;
  mx.ZTBh = ztb.first;
  mx.ZTBl = ztb.second;
  mx.PWh = (__bf16*)L.take(2 * blk_elems(Rc, mx.Rtp));
  mx.PWl = (__bf16*)L.take(2 * blk_elems(Rc, mx.Rtp));
  q.spart = (float*)L.take(4 * (size_t)SPLIT_KPARTS_MAX * q.nmax * q.Tp);
}

void carve_prob(Layout& L, Prob& q, int prec, SplitShare& sh) {
  const int Rt = q.Rt, Tp = q.Tp;
  q.st = (DevState*)L.take(sizeof(DevState));
  q.st_save = (DevState*)L.take(sizeof(DevState));
  q.fit_hist = (double*)L.take(sizeof(double) * HIST_CAP);
  q.inner_part = (double*)L.take(sizeof(double) * Tp);
  q.row_part = (double*)L.take(sizeof(double) * Tp);
  q.norm2 = (double*)L.take(sizeof(double) * 8);
  const size_t nt = (size_t)((Rt + 63) / 64);
  q.partials = (double*)L.take(sizeof(double) * nt * nt);
  // the ||G||^2 set-up products (not needed when the caller supplies ||G||^2)
  size_t setup_elems = (size_t)Rt * Rt;
  if ((size_t)q.nmax * Tp > setup_elems) setup_elems = (size_t)q.nmax * Tp;
  if (q.d.norm2) setup_elems = 0;
  for (int i = 0; i < 3; ++i) q.setup[i] = (double*)L.take(sizeof(double) * setup_elems);
  q.scratch64 = (double*)L.take(sizeof(double) * (size_t)q.nmax * Tp);
  if (prec == CPD_FP32) {
    carve_typed<float>(L, q, q.b32, true);
  } else {
    carve_typed<double>(L, q, q.b64, false);
    for (int m = 0; m < 4; ++m) q.b64.X[m] = q.d.X[m];
    q.b64.Z = q.d.Z;
    if (prec == CPD_MIXED_BF16) carve_mixed(L, q, sh);
  }
}

// ---------------------------------------------------------- table building
// Tables are built on the host, laid out in the table region and uploaded
// once.  With base == nullptr only the sizes are accumulated.
struct TableBuilder {
  Layout L;
  std::vector<char> host;
  template <typename X>
  void* put(const std::vector<X>& v) {
    const size_t bytes = sizeof(X) * v.size();
    const size_t at = L.off;
    void* dev = L.take(bytes);
    if (L.base) {
      if (host.size() < L.off) host.resize(L.off);
      memcpy(host.data() + at, v.data(), bytes);
    }
    return dev;
  }
};

std::string tune_key(const std::string& kind, const std::vector<int>& dims) {
  std::string k(kind);
  for (int d : dims) k += "," + std::to_string(d);
  return k;
}

template <typename T>
GroupOp gemm_op(TableBuilder& tb, const std::vector<GemmArgs<T>>& v, bool at, bool had, const std::string& kind) {
  GroupOp op;
  op.a_t = at;
  op.had = had;
  // tile edge: autotune cache, else heuristic.  Register-staged tiles: 64
  // (three workgroups per compute unit; the staged 128 x 128 form holds
  // ~400 registers, one per unit), 128 only with thousands of tiles.
  std::vector<int> dims;
  long t128 = 0;
  for (auto& g : v) {
    dims.push_back(g.M);
    dims.push_back(g.N);
    dims.push_back(g.K);
    t128 += gemm_tile_count(g.M, g.N, 128, g.lower);
  }
  // FP64: 128 is the direct-load path (1.3-1.4x the 64-tiles at R = 4000),
  // taken when every entry qualifies and the 128-tiles cover the compute
  // units (the back-projection's 224 tiles at n = 800 stay on 64)
  bool dma = sizeof(T) == 8;
  for (auto& g : v) dma = dma && gemm_dma_ok(g, had);
  op.bm = dma ? (t128 >= 256 ? 128 : 64) : (t128 >= 4096 ? 128 : 64);
  op.count = (int)v.size();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(kind, dims));
    if (it != g_tune.end()) op.bm = it->second;
  }
  if (sizeof(T) == 8 && !dma) op.bm = 64;
  std::vector<int> offs(1, 0);
  for (auto& g : v) offs.push_back(offs.back() + gemm_tile_count(g.M, g.N, op.bm, g.lower));
  op.total = offs.back();
  op.tab = tb.put(v);
  op.offs = (int*)tb.put(offs);
  return op;
}

// Launch shape of a split-BF16 grouped product, as one integer (the
// autotune cache value): bm + 1000 wide + 10000 kparts.
struct SplitCfg {
  int bm = 128;
  bool wide = false;
  int kparts = 1;
  bool dma = false;  // direct-load 256 x 256 tiles (bm, wide unused)
  int code() const { return dma ? 100000 + 10000 * kparts : bm + (wide ? 1000 : 0) + 10000 * kparts; }
  static SplitCfg of(int c) {
    SplitCfg g;
    g.dma = c >= 100000;
    c %= 100000;
    g.kparts = c / 10000;
    c %= 10000;
    g.wide = c >= 1000;
    g.bm = g.dma ? 256 : c % 1000;
    if (g.kparts < 1) g.kparts = 1;
    return g;
  }
};

int split_cfg_count(const SplitArgs& g, const SplitCfg& c) {
  if (c.dma) return split_dma_tile_count(g.M, g.N) * c.kparts;
  return c.wide ? split_wide_tile_count(g.M, g.N, c.bm) * c.kparts : split_tile_count(g.M, g.N, c.bm);
}
long split_cfg_tiles(const std::vector<SplitArgs>& v, const SplitCfg& c) {
  long t = 0;
  for (auto& g : v) t += split_cfg_count(g, c);
  return t;
}

// Candidate launch shapes of a product; split-K only where a partial buffer
// exists (the back-projection).
std::vector<SplitCfg> split_candidates(bool splitk, bool dma) {
  std::vector<SplitCfg> c;
  for (int bm : {64, 128}) c.push_back({bm, false, 1});
  for (int bm : {128, 256}) {
    c.push_back({bm, true, 1});
    if (splitk)
      for (int k = 2; k <= SPLIT_KPARTS_MAX; k *= 2) c.push_back({bm, true, k});
  }
  if (dma) {
    c.push_back({256, false, 1, true});
    if (splitk)
      for (int k = 2; k <= SPLIT_KPARTS_MAX; k *= 2) c.push_back({256, false, k, true});
  }
  return c;
}

// Heuristic shape: wide 256 x 256 tiles when they alone cover most compute
// units and K is long; for a short-M back-projection, wide tiles with
// enough K slices to do so; otherwise the 128-column kernel with 64- or 128-row tiles (64 when
// 128-row tiles would pad a quarter more rows, as in the Laplace batch, or
// leave most compute units idle).
SplitCfg split_default(const std::vector<SplitArgs>& v, bool splitk, bool dma) {
  const long w256 = split_cfg_tiles(v, {256, true, 1});
  int kmin = 1 << 30;
  for (auto& g : v) kmin = g.K < kmin ? g.K : kmin;
  // The direct-load tiles wherever the blocked operands exist and the
  // tiles (times the K slices, for a split-K product) cover the compute
  // units with at least 256 of K per slice: measured faster than the other
  // shapes for the core product, the projection (K = n) and the
  // back-projection (4 K slices) alike.
  if (dma) {
    const long wd = split_cfg_tiles(v, {256, false, 1, true});
    for (int k = 1; k <= (splitk ? SPLIT_KPARTS_MAX : 1); k *= 2)
      if (wd * k >= 192 && kmin >= 256 * k) return {256, false, k, true};
  }
  if (w256 >= 192 && kmin >= 2048) return {256, true, 1};
  if (splitk) {
    for (int k = 2; k <= SPLIT_KPARTS_MAX; k *= 2)
      if (w256 * k >= 192) return {256, true, k};
  }
  long rows64 = 0, rows128 = 0;
  for (auto& g : v) {
    rows64 += (long)(g.M + 63) / 64 * 64;
    rows128 += (long)(g.M + 127) / 128 * 128;
  }
  const long t128 = split_cfg_tiles(v, {128, false, 1});
  return {(4 * rows128 >= 5 * rows64 || t128 < 128) ? 64 : 128, false, 1};
}

std::string split_key(const std::string& kind, const std::vector<SplitArgs>& v) {
  std::vector<int> dims;
  for (auto& g : v) {
    dims.push_back(g.M);
    dims.push_back(g.N);
    dims.push_back(g.K);
  }
  return tune_key(kind, dims);
}

void split_apply(GroupOp& op, const std::vector<SplitArgs>& v, const SplitCfg& c, std::vector<int>* offs_out) {
  op.bm = c.bm;
  op.wide = c.wide;
  op.kparts = c.kparts;
  op.dma = c.dma;
  std::vector<int> offs(1, 0);
  for (auto& g : v) offs.push_back(offs.back() + split_cfg_count(g, c));
  op.total = offs.back();
  if (offs_out) *offs_out = offs;
}

// vd (optional): the same products with blocked operands for the
// direct-load tiles, pj: the pair splits they need first.
GroupOp split_op(TableBuilder& tb, const std::vector<SplitArgs>& v, bool apair, bool bpair, const std::string& kind,
                 bool splitk, const std::vector<SplitArgs>* vd = nullptr, const std::vector<PairJob>* pj = nullptr,
                 const std::vector<SplitTArgs>* tj = nullptr) {
  GroupOp op;
  op.apair = apair;
  op.bpair = bpair;
  op.count = (int)v.size();
  for (auto& g : v) {
    if (g.M > op.maxm) op.maxm = g.M;
    if (g.N > op.maxn) op.maxn = g.N;
  }
  if (vd) {
    op.dtab = tb.put(*vd);
    if (pj && !pj->empty()) {
      op.ptab = tb.put(*pj);
      for (auto& j : *pj) {
        const size_t ch = (size_t)blk_rows(j.rows) * (j.Kp / 8);
        if (ch > op.pchunks) op.pchunks = ch;
      }
    }
    if (tj && !tj->empty()) {
      op.ttab = tb.put(*tj);
      for (auto& j : *tj) {
        const size_t ch = (size_t)blk_rows(j.cols) * (j.dcols / 8);
        if (ch > op.tchunks) op.tchunks = ch;
      }
    }
  }
  SplitCfg c = split_default(v, splitk, vd != nullptr);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(split_key(kind, v));
    if (it != g_tune.end()) c = SplitCfg::of(it->second);
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (g_split_force) {
      const SplitCfg f = SplitCfg::of(g_split_force);
      if ((!f.dma || vd) && (f.kparts == 1 || splitk)) c = f;
    }
  }
  if (c.dma && !vd) c = split_default(v, splitk, false);
  std::vector<int> offs;
  split_apply(op, v, c, &offs);
  // room for the prefix sums of any candidate shape (the autotuner rewrites them)
  offs.resize(v.size() + 1 > offs.size() ? v.size() + 1 : offs.size());
  op.tab = tb.put(v);
  op.offs = (int*)tb.put(offs);
  return op;
}

const int partner_of[4] = {1, 0, 3, 2};

// Device tables of one solve schedule.  gate_kind: 0 none, 1 skip problems
// whose factorisation failed, 2 only problems in the damped-retry pass.
template <typename T>
std::vector<SolveLaunch> build_sched(TableBuilder& tb, int sched, int max_nblk, int pw,
                                     const std::vector<StepProb<T>>& sp, int gate_kind, const std::string& kind) {
  std::vector<SolveLaunch> out;
  for (const SolveItem& it : solve_schedule(sched, max_nblk, pw)) {
    SolveLaunch L;
    L.mode = it.mode;
    L.cfg = it.cfg;
    if (it.mode >= 0 && is_flow_mode(it.mode)) {
      std::vector<int> nb, nr;
      for (auto& q : sp) {
        nb.push_back(q.nblk);
        nr.push_back(q.n);
      }
      const std::vector<int> seg = flow_segments(it.mode, nb, nr);
      L.nseg = (int)seg.size() / 3 - 1;
      L.total = seg[3 * L.nseg];
      L.offs = (int*)tb.put(seg);
    } else if (it.mode >= 0) {
      std::vector<int> offs(1, 0);
      for (auto& q : sp) offs.push_back(offs.back() + step_tiles(it.mode, q.nblk, q.n, it.cfg));
      L.total = offs.back();
      L.offs = (int*)tb.put(offs);
    } else {
      std::vector<GemmArgs<T>> v;
      bool bt = true;
      for (int h = 0; h < 2; ++h) {
        if (it.g_kind[h] < 0) continue;
        bt = it.g_kind[h] != PG_BWD;
        for (auto& q : sp) {
          GemmArgs<T> g;
          if (!panel_gemm<T>(it.g_kind[h], q, pw, it.g_panel[h], g)) continue;
          if (gate_kind == 1) {
            g.gate = &q.st->chol_fail;
            g.want = 0;
          } else if (gate_kind == 2) {
            g.gate = &q.st->retry_active;
            g.want = 1;
          }
          v.push_back(g);
        }
      }
      L.gemm = gemm_op<T>(tb, v, false, false, kind + "panel");
      L.gemm.b_t = bt;
    }
    out.push_back(L);
  }
  return out;
}

template <typename T>
void build_typed(TableBuilder& tb, cpd_plan_s* p, Bufs<T> Prob::*bufs, bool gated) {
  const int np = p->count;
  const std::string kind = sizeof(T) == 8 ? "f64" : "f32";
  for (int n = 0; n < 4; ++n) {
    std::vector<GemmArgs<T>> core, back, gram, proj;
    std::vector<StepProb<T>> sp;
    std::vector<FormVArgs<T>> fv;
    std::vector<NormArgs<T>> nm;
    for (int i = 0; i < np; ++i) {
      Prob& q = p->P[i];
      Bufs<T>& b = q.*bufs;
      const int32_t* done = &q.st->done;
      const int Rt = q.Rt, Rc = q.Rc, Tp = q.Tp;
      if (n == 0) core.push_back({Rt, Rc, Rt, b.Z, Rt, b.W[2], b.W[3], Tp, b.Y, Tp, nullptr, T(1), T(0), done});
      if (n == 2) core.push_back({Rt, Rc, Rt, b.Z, Rt, b.W[0], b.W[1], Tp, b.Y, Tp, nullptr, T(1), T(0), done});
      back.push_back({q.n[n], Rc, Rt, b.X[n], Rt, b.W[partner_of[n]], b.Y, Tp, b.Msol, Tp,
                      n == 3 ? b.Msave : nullptr, T(1), T(0), done});
      gram.push_back({Rc, Rc, q.n[n], b.F[n], Tp, b.F[n], nullptr, Tp, b.G[n], Tp, nullptr, T(1), T(0), done});
      gram.back().lower = 1;  // consumers read the lower triangle only
      proj.push_back({Rt, Rc, q.n[n], b.X[n], Rt, b.F[n], nullptr, Tp, b.W[n], Tp, nullptr, T(1), T(0), done});
      if (gated) {
        // split-BF16 plans: these FP64 products serve only problems promoted
        // to the FP64 path (the Gram always runs in FP64)
        for (auto* v : {&core, &back, &proj})
          if (!v->empty()) {
            v->back().gate = &q.st->path;
            v->back().want = 1;
          }
      }
      sp.push_back({b.V, b.ldiag, b.diagL, b.Msol, q.st, q.nblk, q.n[n], b.flow, b.cflow, b.dpart});
      const T* g[3];
      int c = 0;
      for (int m = 0; m < 4; ++m)
        if (m != n) g[c++] = b.G[m];
      fv.push_back({b.V, g[0], g[1], g[2], q.st, Tp, Rc});
      nm.push_back({b.Msol, b.F[n], b.lam, nullptr, nullptr, q.st, q.n[n], Rc, Tp});
    }
    if (n == 0 || n == 2) p->core[n] = gemm_op<T>(tb, core, n == 2, true, kind + "core");
    p->back[n] = gemm_op<T>(tb, back, false, true, kind + "back");
    p->gram[n] = gemm_op<T>(tb, gram, true, false, kind + "gram");
    p->proj[n] = gemm_op<T>(tb, proj, true, false, kind + "proj");
    StepOps& so = p->steps[n];
    so.probs = tb.put(sp);
    const int pw = p->panel_width > 0 ? p->panel_width : p->maxNblk;
    so.chol_retry = build_sched<T>(tb, SCHED_CHOL, p->maxNblk, pw, sp, 2, kind);
    so.cholfwd = build_sched<T>(tb, SCHED_CHOL_FWD, p->maxNblk, pw, sp, 1, kind);
    so.bwd = build_sched<T>(tb, SCHED_BWD, p->maxNblk, pw, sp, 0, kind);
    so.fwd_retry = build_sched<T>(tb, SCHED_FWD, p->maxNblk, pw, sp, 2, kind);
    {
      std::vector<CkptArgs> keep, restore;
      for (int i = 0; i < np; ++i) {
        Prob& q = p->P[i];
        Bufs<T>& b = q.*bufs;
        CkptArgs c{};
        c.a[0] = b.Msol;
        c.b[0] = b.Mbak;
        c.bytes[0] = sizeof(T) * (size_t)q.n[n] * q.Tp;
        keep.push_back(c);
        c.gate = &q.st->retry_active;
        c.want = 1;
        restore.push_back(c);
      }
      so.mkeep = tb.put(keep);
      so.mrestore = tb.put(restore);
    }
    p->formv[n] = tb.put(fv);
    p->norm[n] = tb.put(nm);
    if (n == 3) {
      for (int i = 0; i < np; ++i) {
        Bufs<T>& b = p->P[i].*bufs;
        nm[i].Msave = b.Msave;
        nm[i].inner_part = p->P[i].inner_part;
      }
      p->norm_inner = tb.put(nm);
    }
  }
  std::vector<FitArgs<T>> ft;
  std::vector<CkptArgs> ck;
  std::vector<CondArgs<T>> cd;
  for (int i = 0; i < np; ++i) {
    Prob& q = p->P[i];
    Bufs<T>& b = q.*bufs;
    cd.push_back({b.diagL, q.st, q.Rc});
    FitArgs<T> f;
    for (int m = 0; m < 4; ++m) f.g[m] = b.G[m];
    f.lam = b.lam;
    f.inner_part = q.inner_part;
    f.row_part = q.row_part;
    f.fit_hist = q.fit_hist;
    f.st = q.st;
    f.R = q.Rc;
    f.ld = q.Tp;
    ft.push_back(f);
    CkptArgs c{};
    for (int m = 0; m < 4; ++m) {
      c.a[m] = b.F[m];
      c.b[m] = b.Fsave[m];
      c.bytes[m] = sizeof(T) * (size_t)q.n[m] * q.Tp;
    }
    c.st = q.st;
    c.st_save = q.st_save;
    ck.push_back(c);
  }
  p->fit = tb.put(ft);
  p->ckpt = tb.put(ck);
  p->cond = tb.put(cd);
  if (p->tied) {
    // the tied copies after the updates of modes 0 and 2, and the <G, G~>
    // partials from the mode-3 MTTKRP of the tied factors
    std::vector<NormArgs<T>> ti;
    for (int h = 0; h < 2; ++h) {
      const int n = 2 * h;
      std::vector<CkptArgs> tc;
      for (int i = 0; i < np; ++i) {
        Prob& q = p->P[i];
        Bufs<T>& b = q.*bufs;
        CkptArgs c{};
        c.a[0] = b.F[n];
        c.b[0] = b.F[n + 1];
        c.bytes[0] = sizeof(T) * (size_t)q.n[n] * q.Tp;
        c.a[1] = b.G[n];
        c.b[1] = b.G[n + 1];
        c.bytes[1] = sizeof(T) * (size_t)q.Tp * q.Tp;
        if (p->tie_alias) {
          c.a[2] = b.W[n];
          c.b[2] = b.W[n + 1];
          c.bytes[2] = sizeof(T) * (size_t)q.Rt * q.Tp;
        }
        tc.push_back(c);
        if (h == 1) ti.push_back({b.F[3], nullptr, b.lam, b.Msave, q.inner_part, q.st, q.n[3], q.Rc, q.Tp});
      }
      p->tie[h] = tb.put(tc);
    }
    p->tinner = tb.put(ti);
  }
}

void build_mixed(TableBuilder& tb, cpd_plan_s* p) {
  const int np = p->count;
  for (int n = 0; n < 4; ++n) {
    std::vector<SplitArgs> core, back, proj, cored, backd, projd;
    std::vector<PairJob> corej, backj;
    std::vector<SplitTArgs> ftt, fttb;
    for (int i = 0; i < np; ++i) {
      Prob& q = p->P[i];
      MixedBufs& mx = q.mx;
      const int32_t* done = &q.st->done;
      const int Rt = q.Rt, Rc = q.Rc;
      if (n == 0 || n == 2) {
        const int a = n == 0 ? 2 : 0, b = n == 0 ? 3 : 1;
        SplitOperand A{nullptr, nullptr, mx.WT[a], mx.WT[b], mx.Rtp};
        SplitOperand B = n == 0 ? SplitOperand{mx.Zh, mx.Zl, nullptr, nullptr, mx.Rtp}
                                : SplitOperand{mx.ZTh, mx.ZTl, nullptr, nullptr, mx.Rtp};
        core.push_back({Rc, Rt, mx.Rtp, A, B, mx.YT, nullptr, nullptr, mx.Rtp, done, &q.st->path, 0, nullptr});
        // direct-load form: the pair product split into PW first
        SplitOperand Ad{mx.PWh, mx.PWl, nullptr, nullptr, mx.Rtp};
        SplitOperand Bd = n == 0 ? SplitOperand{mx.ZBh, mx.ZBl, nullptr, nullptr, mx.Rtp}
                                 : SplitOperand{mx.ZTBh, mx.ZTBl, nullptr, nullptr, mx.Rtp};
        cored.push_back({Rc, Rt, mx.Rtp, Ad, Bd, mx.YT, nullptr, nullptr, mx.Rtp, done, &q.st->path, 0, nullptr});
        corej.push_back({mx.WT[a], mx.WT[b], mx.Rtp, Rc, Rt, mx.PWh, mx.PWl, mx.Rtp, done, &q.st->path, 0});
      }
      SplitOperand A{mx.Xh[n], mx.Xl[n], nullptr, nullptr, mx.Rtp};
      SplitOperand B{nullptr, nullptr, mx.WT[partner_of[n]], mx.YT, mx.Rtp};
      back.push_back({q.n[n], Rc, mx.Rtp, A, B, nullptr, q.b64.Msol, nullptr, q.Tp, done, &q.st->path, 0, q.spart});
      SplitOperand Axd{mx.XBh[n], mx.XBl[n], nullptr, nullptr, mx.Rtp};
      SplitOperand Bpd{mx.PWh, mx.PWl, nullptr, nullptr, mx.Rtp};
      backd.push_back({q.n[n], Rc, mx.Rtp, Axd, Bpd, nullptr, q.b64.Msol, nullptr, q.Tp, done, &q.st->path, 0,
                       q.spart});
      backj.push_back({mx.WT[partner_of[n]], mx.YT, mx.Rtp, Rc, Rt, mx.PWh, mx.PWl, mx.Rtp, done, &q.st->path, 0});
      SplitOperand PA{mx.FTh, mx.FTl, nullptr, nullptr, mx.npad_max};
      SplitOperand PB{mx.XTh[n], mx.XTl[n], nullptr, nullptr, mx.npad[n]};
      proj.push_back({Rc, Rt, mx.npad[n], PA, PB, mx.WT[n], nullptr, nullptr, mx.Rtp, done, &q.st->path, 0,
                      nullptr});
      ftt.push_back({q.b64.F[n], mx.FTh, mx.FTl, done, &q.st->path, q.n[n], Rc, q.Tp, mx.npad_max, mx.npad[n]});
      SplitOperand PAd{mx.FTBh, mx.FTBl, nullptr, nullptr, mx.npad[n]};
      SplitOperand PBd{mx.XTBh[n], mx.XTBl[n], nullptr, nullptr, mx.npad[n]};
      projd.push_back({Rc, Rt, mx.npad[n], PAd, PBd, mx.WT[n], nullptr, nullptr, mx.Rtp, done, &q.st->path, 0,
                       nullptr});
      fttb.push_back({q.b64.F[n], mx.FTBh, mx.FTBl, done, &q.st->path, q.n[n], Rc, q.Tp, mx.npad[n], mx.npad[n]});
    }
    if (n == 0 || n == 2) p->score[n] = split_op(tb, core, true, false, "bf16core", false, &cored, &corej);
    p->sback[n] = split_op(tb, back, false, true, "bf16back", true, &backd, &backj);
    p->sproj[n] = split_op(tb, proj, false, false, "bf16proj", false, &projd, nullptr, &fttb);
    p->ftt[n] = tb.put(ftt);
  }
  // FP64 mode-3 MTTKRP for the fit of fit sweeps (split-path problems; a
  // promoted problem's FP64 back-projection already fills Msave), and the
  // FP64 projections that catch up a problem promoted in an asynchronous
  // sweep
  std::vector<GemmArgs<double>> fp[3], fc, fb, cp[4];
  for (int i = 0; i < np; ++i) {
    Prob& q = p->P[i];
    Bufs<double>& b = q.b64;
    const int32_t* done = &q.st->done;
    const int32_t* path = &q.st->path;
    const int Rt = q.Rt, Rc = q.Rc, Tp = q.Tp;
    for (int m = 0; m < 3; ++m)
      fp[m].push_back({Rt, Rc, q.n[m], b.X[m], Rt, b.F[m], nullptr, Tp, b.W[m], Tp, nullptr, 1.0, 0.0, done, path, 0});
    fc.push_back({Rt, Rc, Rt, b.Z, Rt, b.W[0], b.W[1], Tp, b.Y, Tp, nullptr, 1.0, 0.0, done, path, 0});
    fb.push_back({q.n[3], Rc, Rt, b.X[3], Rt, b.W[2], b.Y, Tp, b.Msave, Tp, nullptr, 1.0, 0.0, done, path, 0});
    for (int m = 0; m < 4; ++m)
      cp[m].push_back({Rt, Rc, q.n[m], b.X[m], Rt, b.F[m], nullptr, Tp, b.W[m], Tp, nullptr, 1.0, 0.0, done,
                       &q.st->promote, 1});
  }
  for (int m = 0; m < 3; ++m) p->fproj[m] = gemm_op<double>(tb, fp[m], true, false, "f64proj");
  p->fcore = gemm_op<double>(tb, fc, true, true, "f64core");
  p->fback = gemm_op<double>(tb, fb, false, true, "f64back");
  for (int m = 0; m < 4; ++m) p->cproj[m] = gemm_op<double>(tb, cp[m], true, false, "f64proj");
}

size_t build_tables(cpd_plan_s* p, char* base, std::vector<char>* host) {
  TableBuilder tb;
  tb.L.base = base;
  if (p->prec == CPD_FP32) build_typed<float>(tb, p, &Prob::b32, false);
  else build_typed<double>(tb, p, &Prob::b64, p->prec == CPD_MIXED_BF16);
  if (p->prec == CPD_MIXED_BF16) build_mixed(tb, p);
  std::vector<DevState*> sts;
  for (auto& q : p->P) sts.push_back(q.st);
  p->sts = tb.put(sts);
  std::vector<int32_t> forced(p->count, 0);
  p->forced_dev = (int32_t*)tb.put(forced);
  if (host) {
    tb.host.resize(tb.L.off);
    *host = tb.host;
  }
  return tb.L.off;
}

// Carves all problems and sizes the table region; returns total bytes
// (the last 4 KiB are autotuning scratch).
size_t layout_plan(cpd_plan_s* p, char* base) {
  Layout L;
  L.base = base;
  SplitShare sh;
  for (auto& q : p->P) carve_prob(L, q, p->prec, sh);
  p->tables_off = L.off;
  const size_t tables = build_tables(p, nullptr, nullptr);
  return L.off + align_up(tables) + 4096;
}

int init_shape(cpd_plan_s* p, const cpd_desc* descs, int count) {
  if (count <= 0 || count > 4096 || !descs) return CPD_ERR_INVALID_ARG;
  p->count = count;
  p->P.resize(count);
  for (int i = 0; i < count; ++i) {
    const int rc = check_desc(&descs[i]);
    if (rc != CPD_OK) return rc;
    if (descs[i].precision != descs[0].precision) return CPD_ERR_INVALID_ARG;
    fill_prob(p->P[i], &descs[i]);
  }
  p->prec = descs[0].precision;
  p->tied = descs[0].tied != 0;
  p->tie_alias = true;
  for (int i = 0; i < count; ++i) {
    if ((descs[i].tied != 0) != (p->tied != 0)) return CPD_ERR_INVALID_ARG;
    if (p->tied) {
      if (descs[i].n[1] != descs[i].n[0] || descs[i].n[3] != descs[i].n[2]) return CPD_ERR_INVALID_ARG;
      if (descs[i].X[1] != descs[i].X[0] || descs[i].X[3] != descs[i].X[2]) p->tie_alias = false;
    }
  }
  if (p->tied && p->prec == CPD_MIXED_BF16) return CPD_ERR_UNSUPPORTED;
  p->fit_every = descs[0].fit_every > 0 ? descs[0].fit_every : 1;
  p->allow_fallback = descs[0].chol_fallback;
  p->use_graph = descs[0].use_graph;
  p->autotune = descs[0].autotune;
  p->panel_width = descs[0].solve_panel;
  p->tol = descs[0].tol;
  p->fit_floor = descs[0].fit_floor;
  p->launched = 0;
  p->maxR = p->maxTp = p->maxNblk = p->maxN = 0;
  for (auto& q : p->P) {
    if (q.Rc > p->maxR) p->maxR = q.Rc;
    if (q.Tp > p->maxTp) p->maxTp = q.Tp;
    if (q.nblk > p->maxNblk) p->maxNblk = q.nblk;
    if (q.nmax > p->maxN) p->maxN = q.nmax;
  }
  return CPD_OK;
}

// ------------------------------------------------------------------ set-up
int setup_norm2(Prob& q, hipStream_t s) {
  if (q.d.norm2) {  // supplied by the caller (a DF input: ||B^T B||_F^2)
    HIPCHK(hipMemcpyAsync(q.norm2, q.d.norm2, sizeof(double), hipMemcpyDeviceToDevice, s));
    return CPD_OK;
  }
  const int Rt = q.Rt;
  double *A = q.setup[0], *B = q.setup[1], *C = q.setup[2];
  const double* const* X = q.d.X;
  auto syrk = [&](const double* x, int n, double* out) {
    GemmF64 g{Rt, Rt, n, x, Rt, true, x, nullptr, Rt, false, out, Rt, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  };
  const size_t cnt = (size_t)Rt * Rt;
  syrk(X[0], q.n[0], A);
  if (X[1] == X[0]) hadamard_inplace_f64(s, A, A, cnt);
  else {
    syrk(X[1], q.n[1], B);
    hadamard_inplace_f64(s, A, B, cnt);
  }
  {
    GemmF64 g{Rt, Rt, Rt, q.d.Z, Rt, true, A, nullptr, Rt, false, C, Rt, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  }
  if (!(X[2] == X[0] && X[3] == X[1])) {
    syrk(X[2], q.n[2], A);
    if (X[3] == X[2]) hadamard_inplace_f64(s, A, A, cnt);
    else {
      syrk(X[3], q.n[3], B);
      hadamard_inplace_f64(s, A, B, cnt);
    }
  }
  {
    GemmF64 g{Rt, Rt, Rt, q.d.Z, Rt, false, A, nullptr, Rt, false, B, Rt, nullptr, 1.0, 0.0, nullptr};
    gemm_f64(s, g);
  }
  transposed_dot_f64(s, C, B, Rt, Rt, q.partials, q.norm2);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

void split_inputs(Prob& q, hipStream_t s, std::map<const void*, int>& done_split) {
  MixedBufs& mx = q.mx;
  for (int m = 0; m < 4; ++m) {
    if (done_split.count(mx.Xh[m])) continue;
    done_split[mx.Xh[m]] = 1;
    split_rows_f64(s, q.d.X[m], q.n[m], q.Rt, q.Rt, mx.Xh[m], mx.Xl[m], mx.Rtp, mx.Rtp);
    split_transpose_f64(s, q.d.X[m], q.n[m], q.Rt, q.Rt, mx.XTh[m], mx.XTl[m], mx.npad[m], mx.npad[m]);
    split_blocked_f64(s, q.d.X[m], q.n[m], q.Rt, q.Rt, mx.XBh[m], mx.XBl[m], mx.Rtp);
    split_blocked_f64(s, q.d.X[m], q.Rt, q.n[m], q.Rt, mx.XTBh[m], mx.XTBl[m], mx.npad[m], true);
  }
  if (!done_split.count(mx.Zh)) {
    done_split[mx.Zh] = 1;
    split_rows_f64(s, q.d.Z, q.Rt, q.Rt, q.Rt, mx.Zh, mx.Zl, mx.Rtp, mx.Rtp);
    split_transpose_f64(s, q.d.Z, q.Rt, q.Rt, q.Rt, mx.ZTh, mx.ZTl, mx.Rtp, mx.Rtp);
    split_blocked_f64(s, q.d.Z, q.Rt, q.Rt, q.Rt, mx.ZBh, mx.ZBl, mx.Rtp, false);
    split_blocked_f64(s, q.d.Z, q.Rt, q.Rt, q.Rt, mx.ZTBh, mx.ZTBl, mx.Rtp, true);
  }
}

// --------------------------------------------------------- grouped launches
template <typename T>
void run_gemm(cpd_plan_s* p, hipStream_t s, const GroupOp& op) {
  (void)p;
  gemm_group<T>(s, (const GemmArgs<T>*)op.tab, op.offs, op.count, op.total, op.a_t, op.b_t, op.had, op.bm);
}
void run_split(cpd_plan_s* p, hipStream_t s, const GroupOp& op) {
  (void)p;
  const SplitArgs* tab = (const SplitArgs*)op.tab;
  if (op.dma) {
    const SplitArgs* dtab = (const SplitArgs*)op.dtab;
    if (op.ptab) pair_split_group(s, (const PairJob*)op.ptab, op.count, op.pchunks);
    if (op.ttab) split_transpose_blocked_group(s, (const SplitTArgs*)op.ttab, op.count, op.tchunks);
    gemm_split_dma_group(s, dtab, op.offs, op.count, op.total, op.kparts);
    if (op.kparts > 1) gemm_split_reduce_group(s, dtab, op.count, op.kparts, op.maxm, op.maxn);
    return;
  }
  if (!op.wide) {
    gemm_split_group(s, tab, op.offs, op.count, op.total, op.apair, op.bpair, op.bm);
    return;
  }
  gemm_split_wide_group(s, tab, op.offs, op.count, op.total, op.apair, op.bpair, op.bm, op.kparts);
  if (op.kparts > 1) gemm_split_reduce_group(s, tab, op.count, op.kparts, op.maxm, op.maxn);
}
template <typename T>
void run_sched(cpd_plan_s* p, hipStream_t s, int n, const std::vector<SolveLaunch>& sched, int retry_pass) {
  const StepProb<T>* probs = (const StepProb<T>*)p->steps[n].probs;
  for (const SolveLaunch& L : sched) {
    if (L.mode < 0) run_gemm<T>(p, s, L.gemm);
    else step_group<T>(s, L.mode, probs, L.offs, L.nseg > 0 ? L.nseg : p->count, L.total, L.cfg, retry_pass);
  }
}

template <typename T>
void solve_mode(cpd_plan_s* p, int n, hipStream_t s, bool with_inner, bool fast) {
  const FormVArgs<T>* fv = (const FormVArgs<T>*)p->formv[n];
  StepOps& so = p->steps[n];
  form_v_group<T>(s, fv, p->count, p->maxTp, 0);
  if (fast) {
    run_sched<T>(p, s, n, so.cholfwd, 0);
    run_sched<T>(p, s, n, so.bwd, 0);
  } else {
    // Asynchronous sweeps cannot be replayed from the host, so the damped
    // retry stays in the graph: the fused factorisation and forward solve
    // run on a copy-protected right-hand side; a problem whose pivot failed
    // is refactored from V + mu I, gets its right-hand side back and its
    // forward solve alone (launches that are no-ops without a failure).
    checkpoint_group(s, (const CkptArgs*)so.mkeep, p->count, 0);
    run_sched<T>(p, s, n, so.cholfwd, 0);
    retry_prepare_group<T>(s, fv, p->count, p->allow_fallback);
    form_v_group<T>(s, fv, p->count, p->maxTp, 1);
    run_sched<T>(p, s, n, so.chol_retry, 1);
    checkpoint_group(s, (const CkptArgs*)so.mrestore, p->count, 1);
    run_sched<T>(p, s, n, so.fwd_retry, 1);
    run_sched<T>(p, s, n, so.bwd, 0);
  }
  normalise_group<T>(s, (const NormArgs<T>*)(with_inner ? p->norm_inner : p->norm[n]), p->count, p->maxR);
}

// Particle-tied sweep (symmetric ALS): modes 0 and 2 are updated, each
// followed by its copy to the tied mode (factor, Gram, and the projection
// by copy when the two modes share X, else by product); <G, G~> comes from
// the mode-3 MTTKRP of the tied factors, X3 (W2 o Y'), with Y' of mode 2.
template <typename T>
void enqueue_sweep_tied(cpd_plan_s* p, hipStream_t s, bool fast) {
  if (fast) checkpoint_group(s, (const CkptArgs*)p->ckpt, p->count, 0);
  for (int n = 0; n < 4; n += 2) {
    run_gemm<T>(p, s, p->core[n]);
    run_gemm<T>(p, s, p->back[n]);
    solve_mode<T>(p, n, s, false, fast);
    run_gemm<T>(p, s, p->gram[n]);
    run_gemm<T>(p, s, p->proj[n]);
    checkpoint_group(s, (const CkptArgs*)p->tie[n / 2], p->count, 0);
    if (!p->tie_alias) run_gemm<T>(p, s, p->proj[n + 1]);
  }
  run_gemm<T>(p, s, p->back[3]);
  tied_inner_group<T>(s, (const NormArgs<T>*)p->tinner, p->count, p->maxR);
  fit_group<T>(s, (const FitArgs<T>*)p->fit, p->count, p->maxR, HIST_CAP, p->tol, p->fit_floor, 0, 0.0,
               p->fit_every);
}

template <typename T>
void enqueue_sweep_typed(cpd_plan_s* p, hipStream_t s, bool fast) {
  if (p->tied) {
    enqueue_sweep_tied<T>(p, s, fast);
    return;
  }
  if (fast) checkpoint_group(s, (const CkptArgs*)p->ckpt, p->count, 0);
  for (int n = 0; n < 4; ++n) {
    if (n == 0 || n == 2) run_gemm<T>(p, s, p->core[n]);
    run_gemm<T>(p, s, p->back[n]);
    solve_mode<T>(p, n, s, n == 3, fast);
    run_gemm<T>(p, s, p->gram[n]);
    run_gemm<T>(p, s, p->proj[n]);
  }
  fit_group<T>(s, (const FitArgs<T>*)p->fit, p->count, p->maxR, HIST_CAP, p->tol, p->fit_floor, 0, 0.0,
               p->fit_every);
}

// Mixed precision: the three MTTKRP products in split BF16, everything
// else in FP64.  On fit sweeps the mode-3 MTTKRP is ALSO formed in FP64
// (from the FP64 factors) for <G, G~>: the residual is first-order
// sensitive to that inner product, which split BF16 cannot deliver.
void mixed_refresh_mode(cpd_plan_s* p, hipStream_t s, int n, bool with_gram = true) {
  if (with_gram) run_gemm<double>(p, s, p->gram[n]);
  run_gemm<double>(p, s, p->proj[n]);  // FP64-path problems only (gated)
  int maxc = 0, maxd = 0;
  for (auto& q : p->P) {
    if (q.Rc > maxc) maxc = q.Rc;
    if (q.mx.npad[n] > maxd) maxd = q.mx.npad[n];
  }
  // (the direct-load projection splits its own blocked transpose)
  if (!p->sproj[n].dma) split_transpose_group(s, (const SplitTArgs*)p->ftt[n], p->count, maxc, maxd);
  run_split(p, s, p->sproj[n]);
}

// Precision guard: each problem runs either the split-BF16 MTTKRP (path 0)
// or the FP64 one (path 1); both grouped products are enqueued and every
// problem takes exactly one of them.  A problem is promoted to FP64 when
// its normal matrices get too ill-conditioned, it needs a damped retry, or
// its fit rises (see fit_final / sweep_tick).
void enqueue_sweep_mixed(cpd_plan_s* p, hipStream_t s, bool fit_sweep, bool fast) {
  if (fast) checkpoint_group(s, (const CkptArgs*)p->ckpt, p->count, 0);
  for (int m = 0; m < 4; ++m) run_gemm<double>(p, s, p->cproj[m]);  // promoted last sweep (async)
  guard_begin_group(s, (DevState* const*)p->sts, p->count);
  for (int n = 0; n < 4; ++n) {
    if (n == 0 || n == 2) {
      run_split(p, s, p->score[n]);
      run_gemm<double>(p, s, p->core[n]);
    }
    run_split(p, s, p->sback[n]);
    run_gemm<double>(p, s, p->back[n]);
    if (n == 3 && fit_sweep) {
      for (int m = 0; m < 3; ++m) run_gemm<double>(p, s, p->fproj[m]);
      run_gemm<double>(p, s, p->fcore);
      run_gemm<double>(p, s, p->fback);
    }
    solve_mode<double>(p, n, s, n == 3 && fit_sweep, fast);
    cond_track_group<double>(s, (const CondArgs<double>*)p->cond, p->count);
    mixed_refresh_mode(p, s, n);
  }
  if (fit_sweep)
    // fit sweeps are exactly the sweeps the stopping rule looks at
    fit_group<double>(s, (const FitArgs<double>*)p->fit, p->count, p->maxR, HIST_CAP, p->tol, p->fit_floor, 1,
                      p->cond_limit, 1);
  else
    sweep_tick_group(s, (DevState* const*)p->sts, p->count, 1, p->cond_limit);
}

void enqueue_sweep(cpd_plan_s* p, hipStream_t s, bool fit_sweep, bool fast) {
  if (p->prec == CPD_FP64) enqueue_sweep_typed<double>(p, s, fast);
  else if (p->prec == CPD_FP32) enqueue_sweep_typed<float>(p, s, fast);
  else enqueue_sweep_mixed(p, s, fit_sweep, fast);
}

bool is_fit_sweep(const cpd_plan_s* p, long index1) {
  return p->prec != CPD_MIXED_BF16 || p->fit_every <= 1 || index1 % p->fit_every == 0;
}

int refresh_all(cpd_plan_s* p, hipStream_t s) {
  for (int m = 0; m < 4; ++m) {
    if (p->prec == CPD_FP64) {
      run_gemm<double>(p, s, p->gram[m]);
      run_gemm<double>(p, s, p->proj[m]);
    } else if (p->prec == CPD_FP32) {
      run_gemm<float>(p, s, p->gram[m]);
      run_gemm<float>(p, s, p->proj[m]);
    } else {
      mixed_refresh_mode(p, s, m);
    }
  }
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

int capture(cpd_plan_s* p, bool fit_sweep, bool fast, hipGraph_t* g, hipGraphExec_t* e) {
  if (hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return CPD_ERR_HIP;
  enqueue_sweep(p, p->cap, fit_sweep, fast);
  if (hipStreamEndCapture(p->cap, g) != hipSuccess) return CPD_ERR_HIP;
  if (hipGraphInstantiate(e, *g, nullptr, nullptr, 0) != hipSuccess) return CPD_ERR_HIP;
  return CPD_OK;
}

__global__ void strided_to_dense_f32(const float* src, int rows, int cols, int ld, double* dst) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t r = e / cols, c = e % cols;
    dst[e] = (double)src[r * ld + c];
  }
}
__global__ void dense_to_strided_f32(const double* src, int rows, int cols, int ld, float* dst) {
  const size_t total = (size_t)rows * cols;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
    const size_t r = e / cols, c = e % cols;
    dst[r * ld + c] = (float)src[e];
  }
}
__global__ void state_set_kernel(DevState* st, double prev_fit, int sweeps) {
  if (threadIdx.x == 0) {
    st->fit_prev = prev_fit;
    st->fit_rule = prev_fit;
    st->sweeps = sweeps;
    st->done = 0;
    st->flags = 0;
    st->chol_fail = 0;
    st->retry_active = 0;
  }
}

int grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

int copy_out(cpd_plan_s* p, const Prob& q, const void* src_typed, int rows, int cols, double* dst,
             hipStream_t s) {
  if (p->prec == CPD_FP32) {
    hipLaunchKernelGGL(strided_to_dense_f32, dim3(grid_for((size_t)rows * cols)), dim3(256), 0, s,
                       (const float*)src_typed, rows, cols, q.Tp, dst);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpy2DAsync(dst, sizeof(double) * cols, src_typed, sizeof(double) * q.Tp, sizeof(double) * cols,
                            rows, hipMemcpyDeviceToDevice, s));
  }
  return CPD_OK;
}

int copy_in(cpd_plan_s* p, const Prob& q, const double* src, int rows, int cols, void* dst_typed, hipStream_t s) {
  if (p->prec == CPD_FP32) {
    hipLaunchKernelGGL(dense_to_strided_f32, dim3(grid_for((size_t)rows * cols)), dim3(256), 0, s, src, rows,
                       cols, q.Tp, (float*)dst_typed);
    HIPCHK(hipGetLastError());
  } else {
    HIPCHK(hipMemcpy2DAsync(dst_typed, sizeof(double) * q.Tp, src, sizeof(double) * cols, sizeof(double) * cols,
                            rows, hipMemcpyDeviceToDevice, s));
  }
  return CPD_OK;
}

int read_states(cpd_plan_s* p) {
  for (int i = 0; i < p->count; ++i)
    HIPCHK(hipMemcpyAsync(&p->host_states[i], p->P[i].st, sizeof(DevState), hipMemcpyDeviceToHost, p->stream));
  HIPCHK(hipStreamSynchronize(p->stream));
  return CPD_OK;
}

bool all_done(const cpd_plan_s* p) {
  for (int i = 0; i < p->count; ++i)
    if (!p->host_states[i].done) return false;
  return true;
}
bool any_chol_fail(const cpd_plan_s* p) {
  for (int i = 0; i < p->count; ++i)
    if (p->host_states[i].chol_fail) return true;
  return false;
}
bool any_stall(const cpd_plan_s* p) {
  for (int i = 0; i < p->count; ++i)
    if (p->host_states[i].flags & FLAG_SOLVE_STALL) return true;
  return false;
}
bool any_promote(const cpd_plan_s* p) {
  for (int i = 0; i < p->count; ++i)
    if (p->host_states[i].promote) return true;
  return false;
}
int status_from_flags(int flags) {
  if (flags & FLAG_SOLVE_STALL) return CPD_ERR_HIP;
  if (flags & FLAG_NOT_SPD) return CPD_ERR_NOT_SPD;
  if (flags & FLAG_NONFINITE) return CPD_ERR_NONFINITE;
  return CPD_OK;
}
int batch_status(const cpd_plan_s* p) {
  int f = 0;
  for (int i = 0; i < p->count; ++i) f |= p->host_states[i].flags;
  return status_from_flags(f);
}

int launch_sweep(cpd_plan_s* p, bool fit, bool fast) {
  if (p->have_graph) {
    HIPCHK(hipGraphLaunch(p->exec[fast ? 1 : 0][fit ? 1 : 0], p->stream));
  } else {
    enqueue_sweep(p, p->stream, fit, fast);
    HIPCHK(hipGetLastError());
  }
  return CPD_OK;
}

// Rewinds every problem to the checkpoint taken at the start of the last
// fast sweep and recomputes the projections / Grams from the restored
// factors (deterministic, so problems that did not fail are unchanged).
int rewind_sweep(cpd_plan_s* p) {
  checkpoint_group(p->stream, (const CkptArgs*)p->ckpt, p->count, 1);
  HIPCHK(hipGetLastError());
  if (p->prec == CPD_MIXED_BF16) {
    // the restored states predate any promotion: re-apply the sticky ones
    HIPCHK(hipMemcpyAsync(p->forced_dev, p->forced.data(), sizeof(int32_t) * p->count, hipMemcpyHostToDevice,
                          p->stream));
    set_path_group(p->stream, (DevState* const*)p->sts, p->count, p->forced_dev);
    HIPCHK(hipStreamSynchronize(p->stream));  // the host vector may change before the copy ran
  }
  return refresh_all(p, p->stream);
}

// Tile-size autotuning of the grouped FP64/FP32 GEMMs: times both tile
// edges of every group once and records the faster in the process cache
// (keyed by kind and shapes), which later table builds read.
template <typename T>
void autotune_ops(cpd_plan_s* p, hipStream_t s, bool gram_only = false) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return;
  }
  int* doffs = (int*)(p->ws + p->ws_bytes - 4096);
  auto tune = [&](GroupOp& op, const std::string& kind) {
    if (op.total == 0 || !op.tab || (size_t)(op.count + 1) * sizeof(int) > 4096) return;
    std::vector<GemmArgs<T>> host(op.count);
    if (hipMemcpy(host.data(), op.tab, sizeof(GemmArgs<T>) * op.count, hipMemcpyDeviceToHost) != hipSuccess)
      return;
    std::vector<int> dims;
    for (auto& g : host) {
      dims.push_back(g.M);
      dims.push_back(g.N);
      dims.push_back(g.K);
    }
    const std::string key = tune_key(kind, dims);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        p->tune_log.push_back({key, it->second});
        return;
      }
    }
    float best = 1e30f;
    int best_bm = op.bm;
    bool dma = sizeof(T) == 8;
    for (auto& g : host) dma = dma && gemm_dma_ok(g, op.had);
    for (int bm : {64, 128}) {
      if (bm == 128 && sizeof(T) == 8 && !dma) continue;
      std::vector<int> offs(1, 0);
      for (auto& g : host) offs.push_back(offs.back() + gemm_tile_count(g.M, g.N, bm, g.lower));
      if (hipMemcpy(doffs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice) != hipSuccess) return;
      float ms = 0.f;
      for (int w = 0; w < 2; ++w) {  // second pass is the timed one
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r)
          gemm_group<T>(s, (const GemmArgs<T>*)op.tab, doffs, op.count, offs.back(), op.a_t, op.b_t, op.had, bm);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
      }
      if (ms < best) {
        best = ms;
        best_bm = bm;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best_bm;
    p->tune_log.push_back({key, best_bm});
  };
  const std::string kind = sizeof(T) == 8 ? "f64" : "f32";
  for (int n = 0; n < 4; ++n) {
    if (!gram_only && (n == 0 || n == 2)) tune(p->core[n], kind + "core");
    if (!gram_only) tune(p->back[n], kind + "back");
    tune(p->gram[n], kind + "gram");
    if (!gram_only) tune(p->proj[n], kind + "proj");
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

// Launch-shape autotuning of the split-BF16 grouped products (core,
// back-projection, projection): every candidate shape (128-column tiles
// with 64 or 128 rows; wide bm x 256 tiles with bm = 128 or 256; for the
// back-projection also 2 or 4 K slices) is timed once on the plan's own
// tables and the fastest is kept in the process cache.
void autotune_split(cpd_plan_s* p, hipStream_t s) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return;
  }
  auto tune = [&](GroupOp& op, const std::string& kind, bool splitk) {
    if (op.total == 0 || !op.tab) return;
    std::vector<SplitArgs> host(op.count);
    if (hipMemcpy(host.data(), op.tab, sizeof(SplitArgs) * op.count, hipMemcpyDeviceToHost) != hipSuccess) return;
    const std::string key = split_key(kind, host);
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune.find(key);
      if (it != g_tune.end()) {
        p->tune_log.push_back({key, it->second});
        return;
      }
    }
    float best = 1e30f;
    SplitCfg best_c;
    best_c.bm = op.bm;
    best_c.wide = op.wide;
    best_c.kparts = op.kparts;
    best_c.dma = op.dma;
    for (const SplitCfg& c : split_candidates(splitk, op.dtab != nullptr)) {
      GroupOp t = op;
      std::vector<int> offs;
      split_apply(t, host, c, &offs);
      if (t.total <= 0) continue;
      if (hipMemcpy(op.offs, offs.data(), sizeof(int) * offs.size(), hipMemcpyHostToDevice) != hipSuccess) return;
      float ms = 0.f;
      for (int w = 0; w < 2; ++w) {  // second pass is the timed one
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < 3; ++r) run_split(p, s, t);
        (void)hipEventRecord(e1, s);
        (void)hipEventSynchronize(e1);
        (void)hipEventElapsedTime(&ms, e0, e1);
      }
      if (hipGetLastError() != hipSuccess) return;
      if (ms < best) {
        best = ms;
        best_c = c;
      }
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best_c.code();
    p->tune_log.push_back({key, best_c.code()});
  };
  for (int n = 0; n < 4; ++n) {
    if (n == 0 || n == 2) tune(p->score[n], "bf16core", false);
    tune(p->sback[n], "bf16back", true);
    tune(p->sproj[n], "bf16proj", false);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

int upload_tables(cpd_plan_s* p, hipStream_t s) {
  std::vector<char> host;
  build_tables(p, p->ws + p->tables_off, &host);
  if (host.empty()) return CPD_OK;
  HIPCHK(hipMemcpyAsync(p->ws + p->tables_off, host.data(), host.size(), hipMemcpyHostToDevice, s));
  // the host vector goes out of scope: wait for the copy
  HIPCHK(hipStreamSynchronize(s));
  return CPD_OK;
}

int plan_create(const cpd_desc* descs, int count, void* workspace, size_t ws_bytes, cpd_plan* out) {
  if (!out) return CPD_ERR_INVALID_ARG;
  *out = nullptr;
  cpd_plan_s* p = new (std::nothrow) cpd_plan_s();
  if (!p) return CPD_ERR_INVALID_ARG;
  int rc = init_shape(p, descs, count);
  if (rc != CPD_OK) {
    delete p;
    return rc;
  }
  const size_t need = layout_plan(p, nullptr);
  if (!workspace || ws_bytes < need) {
    delete p;
    return CPD_ERR_WORKSPACE;
  }
  p->ws = (char*)workspace;
  p->ws_bytes = ws_bytes;
  p->stream = (hipStream_t)descs[0].stream;
  p->forced.assign(count, 0);
  layout_plan(p, (char*)workspace);
  if (hipHostMalloc((void**)&p->host_states, sizeof(DevState) * count, hipHostMallocDefault) != hipSuccess) {
    delete p;
    return CPD_ERR_HIP;
  }
  if (hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess) {
    (void)hipHostFree(p->host_states);
    delete p;
    return CPD_ERR_HIP;
  }
  hipStream_t s = p->stream;
  fill_bytes(s, workspace, p->tables_off);
  rc = upload_tables(p, s);
  if (rc == CPD_OK && p->autotune) {
    // tuning launches write the plan's intermediate buffers; they are
    // cleared again below and recomputed by the set-up.  Split-BF16 plans
    // tune their split products and the FP64 Gram (their other FP64
    // products run only for problems the precision guard promotes).
    if (p->prec == CPD_FP64) autotune_ops<double>(p, s);
    else if (p->prec == CPD_FP32) autotune_ops<float>(p, s);
    else {
      autotune_split(p, s);
      autotune_ops<double>(p, s, true);
    }
    rc = upload_tables(p, s);
    fill_bytes(s, workspace, p->tables_off);
  }
  std::map<const void*, int> split_done;
  for (int i = 0; i < count && rc == CPD_OK; ++i) {
    Prob& q = p->P[i];
    rc = setup_norm2(q, s);
    if (rc != CPD_OK) break;
    if (p->prec == CPD_FP32) {
      for (int m = 0; m < 4; ++m) {
        bool first = true;
        for (int r = 0; r < m; ++r)
          if (q.d.X[r] == q.d.X[m]) first = false;
        if (first) cast_f64_to_f32(s, q.d.X[m], (float*)q.b32.X[m], (size_t)q.n[m] * q.Rt);
      }
      cast_f64_to_f32(s, q.d.Z, (float*)q.b32.Z, (size_t)q.Rt * q.Rt);
      for (int m = 0; m < 4; ++m) {
        // (tied: modes 1 and 3 start as copies of modes 0 and 2)
        copy_normalised_init(s, q.d.init[p->tied ? m & 2 : m], q.n[m], q.Rc, q.Tp, q.scratch64);
        cast_f64_to_f32(s, q.scratch64, q.b32.F[m], (size_t)q.n[m] * q.Tp);
      }
    } else {
      if (p->prec == CPD_MIXED_BF16) split_inputs(q, s, split_done);
      for (int m = 0; m < 4; ++m)
        copy_normalised_init(s, q.d.init[p->tied ? m & 2 : m], q.n[m], q.Rc, q.Tp, q.b64.F[m]);
    }
    state_reset(s, q.st, q.norm2, q.d.fit_target > 0.0 ? q.d.fit_target : 0.0);
  }
  if (rc == CPD_OK) rc = refresh_all(p, s);
  if (rc == CPD_OK && hipGetLastError() != hipSuccess) rc = CPD_ERR_HIP;
  if (rc == CPD_OK && p->use_graph) {
    const bool nofit = p->prec == CPD_MIXED_BF16 && p->fit_every > 1;
    for (int fast = 0; fast < 2 && rc == CPD_OK; ++fast)
      for (int fit = nofit ? 0 : 1; fit < 2 && rc == CPD_OK; ++fit)
        rc = capture(p, fit == 1, fast == 1, &p->graph[fast][fit], &p->exec[fast][fit]);
    if (rc == CPD_OK) p->have_graph = true;
  }
  if (rc != CPD_OK) {
    cpd_destroy(p);
    return rc;
  }
  *out = p;
  return CPD_OK;
}

// Runs up to nsweeps batched sweeps (see cpd_batch_sweep).
int batch_sweep(cpd_plan_s* p, int nsweeps, double* fits_host, int32_t* n_run) {
  if (nsweeps < 0) return CPD_ERR_INVALID_ARG;
  const bool sync = fits_host || n_run;
  int ran = 0;
  if (sync) {
    int rc = read_states(p);
    if (rc != CPD_OK) return rc;
    if (all_done(p)) {
      if (n_run) *n_run = 0;
      return batch_status(p);
    }
  }
  for (int i = 0; i < nsweeps; ++i) {
    const bool fit = is_fit_sweep(p, p->launched + 1);
    int rc;
    if (!sync) {
      // asynchronous: the damped retry must live inside the graph
      rc = launch_sweep(p, fit, false);
      if (rc != CPD_OK) return rc;
      p->launched += 1;
      ++ran;
      continue;
    }
    rc = launch_sweep(p, fit, true);
    if (rc == CPD_OK) rc = read_states(p);
    if (rc != CPD_OK) return rc;
    if (any_stall(p)) {
      // a dataflow wait gave up: the problem is marked done on the device
      // and the call reports CPD_ERR_HIP without running further sweeps
      p->launched += 1;
      ++ran;
      break;
    }
    // Replays: a failed pivot reruns the sweep with the damped-retry graph;
    // a precision promotion reruns it with the promoted problems on the
    // FP64 path.  Each problem can be promoted once, so this terminates.
    for (int attempt = 0; attempt < 2 * p->count + 2; ++attempt) {
      if (any_chol_fail(p)) {
        rc = rewind_sweep(p);
        if (rc == CPD_OK) rc = launch_sweep(p, fit, false);
        if (rc == CPD_OK) rc = read_states(p);
        if (rc != CPD_OK) return rc;
      }
      if (!any_promote(p)) break;
      for (int q = 0; q < p->count; ++q)
        if (p->host_states[q].promote) p->forced[q] = 1;
      rc = rewind_sweep(p);
      if (rc == CPD_OK) rc = launch_sweep(p, fit, true);
      if (rc == CPD_OK) rc = read_states(p);
      if (rc != CPD_OK) return rc;
    }
    p->launched += 1;
    ++ran;
    if (fits_host)
      for (int q = 0; q < p->count; ++q)
        fits_host[(size_t)q * nsweeps + (ran - 1)] = fit ? p->host_states[q].fit_prev : -1.0;
    if (all_done(p)) break;
  }
  if (n_run) *n_run = ran;
  if (sync) return batch_status(p);
  return CPD_OK;
}

int stats_of(cpd_plan_s* p, int idx, cpd_stats_t* out) {
  int rc = read_states(p);
  if (rc != CPD_OK) return rc;
  const DevState& h = p->host_states[idx];
  const Prob& q = p->P[idx];
  out->sweeps = h.sweeps;
  out->converged = h.done;
  out->fallbacks = h.fallbacks;
  out->flags = h.flags;
  out->fit = h.sweeps > 0 ? h.fit_prev : -1.0;
  out->norm2 = h.norm2;
  out->inner = h.inner;
  out->model2 = h.model2;
  std::vector<double> dg(q.Rc);
  if (p->prec == CPD_FP32) {
    std::vector<float> df(q.Rc);
    HIPCHK(hipMemcpy(df.data(), q.b32.diagL, sizeof(float) * q.Rc, hipMemcpyDeviceToHost));
    for (int i = 0; i < q.Rc; ++i) dg[i] = df[i];
  } else {
    HIPCHK(hipMemcpy(dg.data(), q.b64.diagL, sizeof(double) * q.Rc, hipMemcpyDeviceToHost));
  }
  double lo = INFINITY, hi = 0.0;
  for (int i = 0; i < q.Rc; ++i) {
    const double v = fabs(dg[i]);
    if (v < lo) lo = v;
    if (v > hi) hi = v;
  }
  out->cond_est = (lo > 0.0 && h.sweeps > 0) ? (hi / lo) * (hi / lo) : -1.0;
  out->fp64_path = h.path;
  out->reserved = 0;
  return CPD_OK;
}

int get_factors_of(cpd_plan_s* p, int idx, double* const F_dev[4], double* lambda_dev) {
  hipStream_t s = p->stream;
  const Prob& q = p->P[idx];
  for (int m = 0; m < 4; ++m) {
    if (!F_dev || !F_dev[m]) continue;
    const void* src = p->prec == CPD_FP32 ? (const void*)q.b32.F[m] : (const void*)q.b64.F[m];
    int rc = copy_out(p, q, src, q.n[m], q.Rc, F_dev[m], s);
    if (rc != CPD_OK) return rc;
  }
  if (lambda_dev) {
    const void* src = p->prec == CPD_FP32 ? (const void*)q.b32.lam : (const void*)q.b64.lam;
    int rc = copy_out(p, q, src, 1, q.Rc, lambda_dev, s);
    if (rc != CPD_OK) return rc;
  }
  return CPD_OK;
}

}  // namespace

extern "C" {

size_t cpd_batch_workspace_size(const cpd_desc* descs, int32_t count) {
  cpd_plan_s tmp;
  if (init_shape(&tmp, descs, count) != CPD_OK) return 0;
  return layout_plan(&tmp, nullptr);
}

size_t cpd_workspace_size(const cpd_desc* d) { return cpd_batch_workspace_size(d, 1); }

cpd_status cpd_init(const cpd_desc* d, cpd_plan* out) {
  if (!d) return CPD_ERR_INVALID_ARG;
  return plan_create(d, 1, d->workspace, d->workspace_bytes, out);
}

cpd_status cpd_batch_init(const cpd_desc* descs, int32_t count, void* workspace, size_t workspace_bytes,
                          cpd_plan* out) {
  return plan_create(descs, count, workspace, workspace_bytes, out);
}

cpd_status cpd_sweep(cpd_plan p, int32_t nsweeps, double* fits_host, int32_t* n_run) {
  if (!p) return CPD_ERR_INVALID_ARG;
  if (p->count == 1) return batch_sweep(p, nsweeps, fits_host, n_run);
  std::vector<double> all(fits_host ? (size_t)p->count * (nsweeps > 0 ? nsweeps : 1) : 0);
  int rc = batch_sweep(p, nsweeps, fits_host ? all.data() : nullptr, n_run);
  if (fits_host)
    for (int i = 0; i < nsweeps; ++i) fits_host[i] = all[i];
  return rc;
}

cpd_status cpd_batch_sweep(cpd_plan p, int32_t nsweeps, double* fits_host, int32_t* n_run) {
  if (!p) return CPD_ERR_INVALID_ARG;
  return batch_sweep(p, nsweeps, fits_host, n_run);
}

cpd_status cpd_batch_states(cpd_plan p, double* fits_host, int32_t* converged_host, int32_t* sweeps_host) {
  if (!p) return CPD_ERR_INVALID_ARG;
  int rc = read_states(p);
  if (rc != CPD_OK) return rc;
  for (int i = 0; i < p->count; ++i) {
    const DevState& h = p->host_states[i];
    if (fits_host) fits_host[i] = h.sweeps > 0 ? h.fit_prev : -1.0;
    if (converged_host) converged_host[i] = h.done;
    if (sweeps_host) sweeps_host[i] = h.sweeps;
  }
  return batch_status(p);
}

int32_t cpd_batch_count(cpd_plan p) { return p ? p->count : 0; }

cpd_status cpd_fit(cpd_plan p, double* fit_host) {
  if (!p || !fit_host) return CPD_ERR_INVALID_ARG;
  int rc = read_states(p);
  if (rc != CPD_OK) return rc;
  *fit_host = p->host_states[0].sweeps > 0 ? p->host_states[0].fit_prev : -1.0;
  return status_from_flags(p->host_states[0].flags);
}

cpd_status cpd_get_factors(cpd_plan p, double* const F_dev[4], double* lambda_dev) {
  if (!p) return CPD_ERR_INVALID_ARG;
  return get_factors_of(p, 0, F_dev, lambda_dev);
}

cpd_status cpd_batch_get_factors(cpd_plan p, int32_t idx, double* const F_dev[4], double* lambda_dev) {
  if (!p || idx < 0 || idx >= p->count) return CPD_ERR_INVALID_ARG;
  return get_factors_of(p, idx, F_dev, lambda_dev);
}

cpd_status cpd_set_factors(cpd_plan p, const double* const F_dev[4], const double* lambda_dev, double prev_fit,
                           int32_t sweeps) {
  if (!p || !F_dev || sweeps < 0 || p->count != 1) return CPD_ERR_INVALID_ARG;
  for (int m = 0; m < 4; ++m)
    if (!F_dev[m]) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  Prob& q = p->P[0];
  for (int m = 0; m < 4; ++m) {
    void* dst = p->prec == CPD_FP32 ? (void*)q.b32.F[m] : (void*)q.b64.F[m];
    int rc = copy_in(p, q, F_dev[m], q.n[m], q.Rc, dst, s);
    if (rc != CPD_OK) return rc;
  }
  if (lambda_dev) {
    void* dst = p->prec == CPD_FP32 ? (void*)q.b32.lam : (void*)q.b64.lam;
    int rc = copy_in(p, q, lambda_dev, 1, q.Rc, dst, s);
    if (rc != CPD_OK) return rc;
  }
  hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, q.st, prev_fit, (int)sweeps);
  HIPCHK(hipGetLastError());
  int rc = refresh_all(p, s);
  if (rc != CPD_OK) return rc;
  p->launched = sweeps;
  return CPD_OK;
}

cpd_status cpd_stats(cpd_plan p, cpd_stats_t* out) {
  if (!p || !out) return CPD_ERR_INVALID_ARG;
  return stats_of(p, 0, out);
}

cpd_status cpd_batch_stats(cpd_plan p, int32_t idx, cpd_stats_t* out) {
  if (!p || !out || idx < 0 || idx >= p->count) return CPD_ERR_INVALID_ARG;
  return stats_of(p, idx, out);
}

cpd_status cpd_mttkrp(cpd_plan p, int32_t mode, double* M_dev) {
  if (!p || mode < 0 || mode > 3 || !M_dev) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  const int core = mode < 2 ? 0 : 2;
  Prob& q = p->P[0];
  if (p->prec == CPD_FP64) {
    run_gemm<double>(p, s, p->core[core]);
    run_gemm<double>(p, s, p->back[mode]);
    return copy_out(p, q, q.b64.Msol, q.n[mode], q.Rc, M_dev, s);
  } else if (p->prec == CPD_FP32) {
    run_gemm<float>(p, s, p->core[core]);
    run_gemm<float>(p, s, p->back[mode]);
    return copy_out(p, q, q.b32.Msol, q.n[mode], q.Rc, M_dev, s);
  }
  run_split(p, s, p->score[core]);
  run_split(p, s, p->sback[mode]);
  return copy_out(p, q, q.b64.Msol, q.n[mode], q.Rc, M_dev, s);
}

cpd_status cpd_kernel_times(cpd_plan p, int32_t reps, double* ms_out) {
  if (!p || reps <= 0 || !ms_out) return CPD_ERR_INVALID_ARG;
  hipStream_t s = p->stream;
  for (auto& q : p->P) hipLaunchKernelGGL(state_set_kernel, dim3(1), dim3(64), 0, s, q.st, -1.0, 0);
  HIPCHK(hipGetLastError());
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool f32 = p->prec == CPD_FP32;
  for (int which = 0; which < 8; ++which) {
    auto body = [&]() {
      if (which == 7) {
        if (f32) form_v_group<float>(s, (const FormVArgs<float>*)p->formv[0], p->count, p->maxTp, 0);
        else form_v_group<double>(s, (const FormVArgs<double>*)p->formv[0], p->count, p->maxTp, 0);
        return;
      }
      if (which >= 4) {
        // normal-equation solve of mode 0: V, factorisation fused with the
        // forward solve, backward solve, normalisation
        if (f32) {
          if (which != 6) form_v_group<float>(s, (const FormVArgs<float>*)p->formv[0], p->count, p->maxTp, 0);
          if (which != 6) run_sched<float>(p, s, 0, p->steps[0].cholfwd, 0);
          if (which != 5) run_sched<float>(p, s, 0, p->steps[0].bwd, 0);
          if (which == 4) normalise_group<float>(s, (const NormArgs<float>*)p->norm[0], p->count, p->maxR);
        } else {
          if (which != 6) form_v_group<double>(s, (const FormVArgs<double>*)p->formv[0], p->count, p->maxTp, 0);
          if (which != 6) run_sched<double>(p, s, 0, p->steps[0].cholfwd, 0);
          if (which != 5) run_sched<double>(p, s, 0, p->steps[0].bwd, 0);
          if (which == 4) normalise_group<double>(s, (const NormArgs<double>*)p->norm[0], p->count, p->maxR);
        }
        return;
      }
      if (p->prec == CPD_MIXED_BF16) {
        if (which == 0) mixed_refresh_mode(p, s, 0, false);  // the Gram is timed on its own
        else if (which == 1) run_split(p, s, p->score[0]);
        else if (which == 2) run_split(p, s, p->sback[0]);
        else run_gemm<double>(p, s, p->gram[0]);
      } else {
        const GroupOp& op = which == 0 ? p->proj[0] : which == 1 ? p->core[0] : which == 2 ? p->back[0] : p->gram[0];
        if (f32) run_gemm<float>(p, s, op);
        else run_gemm<double>(p, s, op);
      }
    };
    body();  // warm-up
    HIPCHK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) body();
    HIPCHK(hipEventRecord(e1, s));
    HIPCHK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, e0, e1));
    ms_out[which] = (double)ms / reps;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return CPD_OK;
}

int32_t cpd_test_split_force(int32_t code) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  const int prev = g_split_force;
  g_split_force = code < 0 ? 0 : code;
  return prev;
}

int32_t cpd_autotune_log(cpd_plan p, char* buf, int32_t len) {
  if (!p) return -1;
  std::string out;
  for (auto& kv : p->tune_log) out += kv.first + "=" + std::to_string(kv.second) + "\n";
  if (buf && len > 0) {
    const size_t n = out.size() < (size_t)(len - 1) ? out.size() : (size_t)(len - 1);
    memcpy(buf, out.data(), n);
    buf[n] = 0;
  }
  return (int32_t)out.size();
}

cpd_status cpd_lt_scale_rows(const double* X, const double* eps, int32_t n, int32_t r, double t, double sign,
                             double* out, void* stream) {
  if (!X || !eps || !out || n <= 0 || r <= 0) return CPD_ERR_INVALID_ARG;
  lt_scale_rows((hipStream_t)stream, X, eps, n, r, t, sign, out);
  return hipGetLastError() == hipSuccess ? CPD_OK : CPD_ERR_HIP;
}

cpd_status cpd_destroy(cpd_plan p) {
  if (!p) return CPD_ERR_INVALID_ARG;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      if (p->exec[a][b]) (void)hipGraphExecDestroy(p->exec[a][b]);
      if (p->graph[a][b]) (void)hipGraphDestroy(p->graph[a][b]);
    }
  if (p->cap) (void)hipStreamDestroy(p->cap);
  if (p->host_states) (void)hipHostFree(p->host_states);
  delete p;
  return CPD_OK;
}

const char* cpd_status_string(cpd_status s) {
  switch (s) {
    case CPD_OK: return "ok";
    case CPD_ERR_INVALID_ARG: return "invalid argument";
    case CPD_ERR_HIP: return "HIP runtime error (or a dataflow solve wait gave up)";
    case CPD_ERR_NOT_SPD: return "normal matrix not positive definite";
    case CPD_ERR_NONFINITE: return "non-finite value in the fit";
    case CPD_ERR_WORKSPACE: return "workspace missing or too small";
    case CPD_ERR_UNSUPPORTED: return "unsupported option";
    default: return "unknown status";
  }
}

}  // extern "C"
