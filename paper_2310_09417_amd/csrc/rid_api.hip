// Host driver and C ABI of the randomized LUPP interpolative decomposition.
// Every step of the decomposition runs in the kernels of rid_kernels.hpp; the
// host only validates arguments, carves the caller's workspace, sizes the
// launches and enqueues them on the caller's stream (no host synchronisation).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <utility>
#include <vector>

#include "../../include/rid.h"
#include "rid_kernels.hpp"
#include "rid_sketch.hpp"
#include "rid_batched.hpp"
#include "rid_sketch_lp.hpp"
#include "rid_refine.hpp"
#include "rid_mlp.hpp"
#include "rid_resid.hpp"
#include "rid_rows.hpp"
#include "rid_sparse.hpp"

using namespace rid;

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxW = 128;        // widest sketch block per pass / panel
constexpr int kPanel = 64;        // panel width of the fixed-rank factorisation
constexpr int kGridCandidates = 3;  // persistent grids the batched autotuner times
constexpr size_t kMaxLds = 160 * 1024;

// LDS of the panel factorisation: the rows' panel values, two pivot rows of
// up to 128 values, and a flag per row.
size_t panel_lds(int64_t rows, int64_t w, size_t es) {
  return (size_t)rows * (size_t)panel_pitch((int)w, (int)es) * es + 256 * es + (size_t)rows * 4;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct DeviceInfo {
  int cu = 0;
  bool ok = false;
};

DeviceInfo device_info() {
  static std::mutex mu;
  static DeviceInfo cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DeviceInfo{};
  std::lock_guard<std::mutex> lk(mu);
  if (!cache[dev].ok) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return DeviceInfo{};
    cache[dev].cu = p.multiProcessorCount;
    cache[dev].ok = true;
  }
  return cache[dev];
}

inline size_t esize(rid_dtype t) { return t == RID_F64 ? 8 : 4; }

// ---- a second stream for work off the critical path --------------------------
// The growth of L1^{-1} after a panel is needed only by the next block's U2
// product, not by its sketch, so the adaptive loop runs it on a second stream
// (default priority) forked from the caller's stream by an event and joined
// back before that product.  Sets of (stream, fork event, join event) come from
// a per-process pool; a call holds one set while it enqueues, so calls from
// different host threads never share events.  Without a set (creation failed,
// pool exhausted) the work stays on the caller's stream.
struct SideSet {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  int dev = -1;
  bool busy = false;
};
std::mutex side_mu;
SideSet side_pool[32];

class SideLease {
 public:
  SideLease() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return;
    std::lock_guard<std::mutex> lk(side_mu);
    for (SideSet& e : side_pool)
      if (!e.busy && e.dev == dev) {
        e.busy = true;
        set_ = &e;
        return;
      }
    for (SideSet& e : side_pool)
      if (e.dev < 0) {
        if (hipStreamCreateWithFlags(&e.s, hipStreamNonBlocking) != hipSuccess) return;
        if (hipEventCreateWithFlags(&e.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&e.join, hipEventDisableTiming) != hipSuccess) {
          (void)hipGetLastError();
          return;  // the stream stays unused; this slot is not handed out
        }
        e.dev = dev;
        e.busy = true;
        set_ = &e;
        return;
      }
  }
  // An error return between a fork and its join leaves forked work running:
  // the caller's stream still waits for it here, before the set is released,
  // so nothing the caller enqueues next (e.g. freeing the workspace) overtakes it.
  ~SideLease() {
    if (!set_) return;
    if (pending) (void)hipStreamWaitEvent(caller, set_->join, 0);
    std::lock_guard<std::mutex> lk(side_mu);
    set_->busy = false;
  }
  SideLease(const SideLease&) = delete;
  SideLease& operator=(const SideLease&) = delete;
  SideSet* get() const { return set_; }
  bool pending = false;          // forked work not yet joined
  hipStream_t caller = nullptr;  // the stream the work was forked from

 private:
  SideSet* set_ = nullptr;
};

// ---- optional per-kernel-class timing (HIP events on the call's stream) ----
enum KClass {
  KC_SKETCH = 0, KC_REDUCE, KC_TRSM, KC_SCHUR, KC_LUPP, KC_TSOLVE, KC_LINV, KC_BATCHED, KC_OMEGA,
  KC_RESID, KC_SKETCH2, KC_N
};

struct Profiler {
  bool on = false;
  int override_class = -1;  // >= 0: every launch is counted in this class
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<std::pair<int, size_t>> marks;  // (class, index of start event)
};
Profiler& prof() {
  static Profiler p;
  return p;
}

// Records a start event before a launch of class c; returns the slot to close.
inline long prof_begin(int c, hipStream_t st) {
  Profiler& p = prof();
  if (!p.on) return -1;
  while (p.used + 2 > p.pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return -1;
    p.pool.push_back(e);
  }
  if (p.override_class >= 0) c = p.override_class;
  const size_t at = p.used;
  p.used += 2;
  if (hipEventRecord(p.pool[at], st) != hipSuccess) return -1;
  p.marks.emplace_back(c, at);
  return (long)at;
}
inline void prof_end(long at, hipStream_t st) {
  if (at >= 0) (void)hipEventRecord(prof().pool[(size_t)at + 1], st);
}

// Sketch launch geometry for a block of w <= 64 vectors: 128 (FP32) or 256
// (FP64) columns per workgroup, enough row splits for 2-8 rounds of
// workgroups.
struct SketchGeom {
  int mt, wp, kc;
  int64_t ncolg, nsplit, rows_per_split;
};

SketchGeom sketch_geom(int64_t m, int64_t n, int w, rid_dtype dt, int cu) {
  SketchGeom g;
  g.mt = w <= 16 ? 1 : w <= 32 ? 2 : 4;
  g.wp = g.mt * 16;
  g.kc = 32;
  g.ncolg = ceil_div(n, dt == RID_F64 ? SketchShape<double>::CPW : SketchShape<float>::CPW);
  // Resident workgroups: two per CU in FP32 (4 waves, ~78 KB of LDS each),
  // one in FP64 (8 waves).  Pick the number of row splits whose workgroup
  // count fills the last round best, between ~2 and ~8 rounds, preferring
  // fewer.  FP32 counts rounds of twice its resident workgroups: more,
  // shorter row splits measured faster for the split sketch at 50000 x 20000
  // (1.02 -> 0.94 ms per launch; the partials then take 1.2 -> 2.2 ms per
  // decomposition to reduce, before they were stored in FP32).
  const int64_t slots = (int64_t)cu * (dt == RID_F64 ? 1 : 4);
  const int64_t maxsplit = ceil_div(m, g.kc);
  const int64_t lo = std::max<int64_t>(1, std::min<int64_t>(maxsplit, ceil_div(2 * slots, g.ncolg)));
  const int64_t hi = std::max<int64_t>(lo, std::min<int64_t>(maxsplit, ceil_div(8 * slots, g.ncolg)));
  double best = -1.0;
  int64_t best_ns = lo;
  for (int64_t ns = lo; ns <= hi; ++ns) {
    const int64_t rps = ceil_div(ceil_div(m, ns), g.kc) * g.kc;
    const int64_t real_ns = ceil_div(m, rps);
    const int64_t items = g.ncolg * real_ns;
    const double eff = (double)items / (double)(ceil_div(items, slots) * slots);
    if (eff > best + 1e-3) {
      best = eff;
      best_ns = ns;
    }
  }
  g.rows_per_split = ceil_div(ceil_div(m, best_ns), g.kc) * g.kc;
  g.nsplit = ceil_div(m, g.rows_per_split);
  return g;
}

// Row-form sketch geometry (k_sketch_rows): 64 rows of A per workgroup and
// enough splits of the contraction (A's columns, in multiples of 32) for
// about four workgroups per CU, each split at least 256 columns long.
struct SketchGeomR {
  int mt, wp;
  int64_t ntile, nsplit, cols_per_split;
};

SketchGeomR sketch_geom_rows(int64_t mrows, int64_t ncols, int w, int cu) {
  SketchGeomR g;
  g.mt = w <= 16 ? 1 : w <= 32 ? 2 : 4;
  g.wp = g.mt * 16;
  g.ntile = ceil_div(mrows, 64);
  const int64_t maxsplit = std::max<int64_t>(1, ncols / 256);
  const int64_t ns = std::max<int64_t>(1, std::min<int64_t>(maxsplit, ceil_div(4 * cu, g.ntile)));
  g.cols_per_split = ceil_div(ceil_div(ncols, ns), 32) * 32;
  g.nsplit = ceil_div(ncols, g.cols_per_split);
  return g;
}

// Low-precision sketch geometry (k_sketch_lpr): 256 (BF16) or 512 (FP8)
// columns per 256-thread workgroup, two resident per CU.  The split count
// minimises the bytes of A each workgroup slot streams (rounds x rows per
// split x its row bytes) plus the FP32 partials written and read back per
// slot, counting four slots per CU, which gives about two workgroups per
// resident slot: the partials are a larger share of a pass over A here than
// in the FP32 sketch (one FP8 pass is 1 GB at 50000 x 20000).  Measured at
// that size (sketch + reduction per decomposition): one round of slots 17.8
// (BF16) / 10.4 ms (FP8), about two 15.9 / 10.1 ms, about eight 17.8 / 11.7 ms.
struct LpGeom {
  int64_t ncolg, nsplit, rows_per_split;
};

// vg = 2: k_sketch_lpw (half the columns per workgroup, 128 vectors).
LpGeom sketch_geom_lp(int64_t m, int64_t n, int fmt, int cu, int vg = 1) {
  LpGeom g;
  const int64_t cols = kLprCols(fmt) / vg, es = fmt == 1 ? 2 : 1, kc = 32;
  g.ncolg = ceil_div(n, cols);
  const int64_t slots = (int64_t)cu * 4;
  const int64_t maxsplit = ceil_div(m, kc);
  const int64_t hi = std::max<int64_t>(1, std::min<int64_t>(maxsplit, ceil_div(8 * slots, g.ncolg)));
  double best = -1.0;
  int64_t best_ns = 1;
  for (int64_t ns = 1; ns <= hi; ++ns) {
    const int64_t rps = ceil_div(ceil_div(m, ns), kc) * kc;
    const int64_t real_ns = ceil_div(m, rps);
    const int64_t items = g.ncolg * real_ns;
    const double cost = (double)ceil_div(items, slots) * (double)rps * (double)(cols * es) +
                        (double)items * (double)cols * 64.0 * vg * 4.0 * 2.0 / (double)slots;
    if (best < 0.0 || cost < best * (1.0 - 1e-3)) {
      best = cost;
      best_ns = ns;
    }
  }
  g.rows_per_split = ceil_div(ceil_div(m, best_ns), kc) * kc;
  g.nsplit = ceil_div(m, g.rows_per_split);
  return g;
}

// Bytes of the low-precision form's Omega records per 32 rows.
inline size_t lp_record_bytes(rid_dtype at) { return at == RID_BF16 ? 4096 : 2048; }

inline bool low_precision(rid_dtype t) { return t == RID_BF16 || t == RID_FP8_E4M3; }

// Everything a call needs, derived from its sizes.
struct Plan {
  int64_t m = 0, n = 0, kcap = 0, wmax = 0;
  rid_dtype dt = RID_F64;   // factor type
  rid_dtype at = RID_F64;   // storage type of A
  const float* scale = nullptr;  // FP8 column-tile scales (device)
  bool refine = false;           // FP64-residual refinement step on T
  bool refine_keep = false;      // keep the refined T without the choice (refine = 2)
  int est = 0;                   // rid_estimator of the stopping test
  int emb = 0;                   // rid_embedding of the sketch
  int resid_p = 0;               // set-aside sample width (adaptive, est > 0)
  int side = RID_COLUMNS;        // RID_ROWS: the column form of A^T, A read in place
  int64_t zr = 0;                // first Z column of the sample (adaptive, est > 0)
  int64_t zs = 0;                // first Z column of its copy that the private LU factors
  int64_t ldz = 0, ldu = 0, ldl = 0, ldg = 0;
  int cu = 0;
  int lupp_g = 0, lupp_rows = 0;
  size_t lupp_lds = 0;
  size_t part_bytes = 0, fro_count = 0;
  int64_t schur_wgs = 0;
  // offsets
  size_t xwords_end = 0;  // end of the panel exchange words (zeroed per call)
  size_t o_ctrl, o_pos, o_order, o_nonpiv, o_z, o_u2t, o_part, o_fro, o_norm, o_slots,
      o_slotrows, o_nonfinite, o_linv, o_mtmp, o_omega, o_yorig, o_tt, o_x, o_t1, o_posr, o_orderr,
      o_ctrlr, o_ytop, total;
};

// est > 0: a Remark-1 stopping estimate; sample_cols > 0 (adaptive calls)
// reserves that many Z columns after the decomposition's own for the sample.
bool make_plan(int64_t m, int64_t n, int64_t kcap, int64_t wmax, rid_dtype dt, rid_dtype at,
               bool refine, int est, int sample_cols, Plan& P, int side = RID_COLUMNS) {
  DeviceInfo di = device_info();
  if (!di.ok) return false;
  P.side = side;
  P.m = m;
  P.n = n;
  P.kcap = kcap;
  P.wmax = wmax;
  P.dt = dt;
  P.at = at;
  P.refine = refine;
  P.est = est;
  P.resid_p = sample_cols;
  P.cu = di.cu;
  const size_t es = esize(dt);
  P.ldz = (int64_t)align_up((size_t)(kcap + wmax), 4);
  P.zr = P.ldz;
  P.zs = P.zr + kResidPMax;
  if (sample_cols > 0) P.ldz = (int64_t)align_up((size_t)(P.zs + kResidPMax), 4);
  P.ldu = (int64_t)align_up((size_t)kcap, 16);
  P.ldl = (int64_t)align_up((size_t)kcap, 64);
  // Panel factorisation: each workgroup keeps up to 192 candidate rows in
  // LDS, one per thread of its three row waves (fewer when wide FP64 panels
  // would not fit; more per thread only when n needs more than one
  // workgroup per compute unit).
  {
    const int64_t cap =
        (int64_t)((kMaxLds - 256 * es) / ((size_t)panel_pitch((int)wmax, (int)es) * es + 4));
    const int64_t target = std::max<int64_t>(16, std::min<int64_t>(192, cap));
    P.lupp_g = (int)std::max<int64_t>(1, std::min<int64_t>(di.cu, ceil_div(n, target)));
  }
  P.lupp_rows = (int)ceil_div(n, P.lupp_g);
  P.lupp_g = (int)ceil_div(n, P.lupp_rows);
  P.lupp_lds = panel_lds(P.lupp_rows, wmax, es);
  // sketch partials: every launch covers <= 64 vectors with the same split
  size_t pb = 0, fc = 0;
  if (low_precision(at)) {
    LpGeom g = sketch_geom_lp(m, n, at == RID_BF16 ? 1 : 2, di.cu);
    LpGeom g2 = sketch_geom_lp(m, n, at == RID_BF16 ? 1 : 2, di.cu, 2);
    pb = std::max((size_t)g.nsplit * (size_t)n * 64 * 4, (size_t)g2.nsplit * (size_t)n * 128 * 4);
    fc = (size_t)(g.nsplit * g.ncolg);
  } else if (side == RID_ROWS) {
    // candidates are A's rows (n here), the contraction runs over its columns (m)
    SketchGeomR g = sketch_geom_rows(n, m, (int)std::min<int64_t>(wmax, 64), di.cu);
    pb = (size_t)g.nsplit * (size_t)n * g.wp * 8;
    fc = (size_t)(g.nsplit * g.ntile);
  } else {
    SketchGeom g = sketch_geom(m, n, (int)std::min<int64_t>(wmax, 64), dt, di.cu);
    pb = (size_t)g.nsplit * (size_t)n * g.wp * 8;
    fc = (size_t)(g.nsplit * g.ncolg);
  }
  P.part_bytes = pb;
  P.fro_count = fc;
  P.schur_wgs = ceil_div(n, 16);  // most Schur workgroups of any launch (16 rows each)
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, kAlign);
    return at;
  };
  P.o_ctrl = take(sizeof(Ctrl));
  P.o_nonfinite = take(4);
  P.o_pos = take((size_t)n * 4);
  P.o_order = take((size_t)(kcap + 1) * 4);
  P.o_nonpiv = take((size_t)n * 4);
  P.o_z = take((size_t)n * P.ldz * es);
  P.o_u2t = take((size_t)wmax * P.ldu * es);
  // the block's pivot rows, gathered for the U2 product (kcap x ldg)
  P.ldg = (int64_t)align_up((size_t)std::max<int64_t>(wmax, kResidPMax), 4);
  P.o_ytop = take((size_t)kcap * P.ldg * es);
  P.o_part = take(P.part_bytes);
  P.o_fro = take(P.fro_count * 8);
  P.o_norm = take((size_t)P.schur_wgs * 8);
  // panel exchange: tagged 64-bit words, es/4 per value, two buffers
  P.o_slots = take((size_t)2 * P.lupp_g * (es / 4 + 1) * 8);
  P.o_slotrows = take((size_t)2 * P.lupp_g * wmax * (es / 4) * 8);
  P.xwords_end = o;
  P.o_linv = take((size_t)kcap * P.ldl * es);
  P.o_mtmp = take((size_t)wmax * P.ldl * es);
  // Omega of one sketch launch (at most 64 vectors), rows padded to 64; in
  // FP32 followed by its three-part BF16 operand form (k_omega_split, 384
  // bytes per row)
  // (the low-precision forms: the FP32 Gaussian entries of up to 128
  // vectors, then their records in the format, lp_record_bytes per 32 rows
  // and 64 vectors)
  P.o_omega = take(low_precision(at)
                       ? (size_t)align_up((size_t)m, 64) * 128 * 4 +
                             (size_t)align_up((size_t)m, 64) / 32 * 2 * lp_record_bytes(at)
                       : (size_t)align_up((size_t)m, 64) * (64 * es + (es == 4 ? 384 : 0)));
  // refinement: the kept sketch (n x ldz), T^T and the residual rows (n x ldl)
  P.o_yorig = take(refine ? (size_t)n * P.ldz * es : 0);
  P.o_tt = take(refine ? (size_t)n * P.ldl * es : 0);
  P.o_x = take(refine ? (size_t)n * P.ldl * es : 0);
  P.o_t1 = take(refine ? (size_t)n * P.ldl * es : 0);  // the refined T, transposed
  // Remark-1 estimate: the private pivot state of the sample's factorisation
  P.o_posr = take(est > 0 ? (size_t)n * 4 : 0);
  P.o_orderr = take(est > 0 ? (size_t)(P.ldz + 1) * 4 : 0);
  P.o_ctrlr = take(est > 0 ? sizeof(Ctrl) : 0);
  P.total = o;
  return true;
}

// Plan of a call with rank cap kmax and block width b (fixed rank: kmax = k + p,
// b = p): kcap = min(kmax, m, n), widest block min(128, max(b, min(kcap, 64))): the
// adaptive blocks have b columns, the fixed-rank panels at most 64 and its
// estimate block p.
// sample: the call sets a Remark-1 sample aside (adaptive calls with an
// estimator).
bool plan_for(int64_t m, int64_t n, int64_t kmax, int64_t b, const rid_config* cfg, Plan& P,
              bool sample = false) {
  // the row form is the column form of A^T: n "rows" (A's columns) and m
  // candidates (A's rows)
  const int side = cfg->side;
  if (side == RID_ROWS) std::swap(m, n);
  const int64_t kcap = std::min<int64_t>(kmax, std::min(m, n));
  int64_t wmax =
      std::min<int64_t>(kMaxW, std::max<int64_t>({b, std::min<int64_t>(kcap, kPanel), 1}));
  const int est = cfg->estimator;
  if (sample && est > 0) wmax = std::max<int64_t>(wmax, cfg->resid_p);
  if (!make_plan(m, n, kcap, wmax, cfg->dtype, cfg->a_type, cfg->refine != 0, est,
                 sample && est > 0 ? cfg->resid_p : 0, P, side))
    return false;
  P.emb = cfg->embedding;
  P.scale = cfg->a_col_scale;
  P.refine_keep = cfg->refine == 2;
  return true;
}

// FP64 partials of the certificate products: kCertSplitMax ranges x p x n.
size_t cert_part_bytes(int64_t n, int64_t p) {
  return align_up((size_t)kCertSplitMax * (size_t)p * (size_t)n * 8, kAlign);
}

// Plan of the row-skeleton step: the m rows of A are the candidates, C has k
// columns; there is no sketch (one sketch row keeps its buffers minimal).
bool plan_rows(int64_t m, int64_t k, const rid_config* cfg, Plan& P) {
  const int64_t wmax = std::max<int64_t>(std::min<int64_t>(k, kPanel), 1);  // panels of <= 64
  return make_plan(1, m, k, wmax, cfg->dtype, cfg->dtype, false, 0, 0, P);
}

// Pointers into the caller's workspace.
struct Ws {
  Ctrl* ctrl;
  int* nonfinite;
  int* pos;
  int* order;
  int* nonpiv;
  void* z;
  void* u2t;
  void* ytop;
  double* part;
  double* fro;
  double* norm;
  xword* slots;
  xword* slotrows;
  void* linv;
  void* mtmp;
  void* omega;
  void* yorig;
  void* tt;
  void* xr;
  void* t1;
  int* pos_r;
  int* order_r;
  Ctrl* ctrl_r;
};

Ws carve(const Plan& P, void* work) {
  char* b = static_cast<char*>(work);
  Ws w;
  w.ctrl = reinterpret_cast<Ctrl*>(b + P.o_ctrl);
  w.nonfinite = reinterpret_cast<int*>(b + P.o_nonfinite);
  w.pos = reinterpret_cast<int*>(b + P.o_pos);
  w.order = reinterpret_cast<int*>(b + P.o_order);
  w.nonpiv = reinterpret_cast<int*>(b + P.o_nonpiv);
  w.z = b + P.o_z;
  w.u2t = b + P.o_u2t;
  w.ytop = b + P.o_ytop;
  w.part = reinterpret_cast<double*>(b + P.o_part);
  w.fro = reinterpret_cast<double*>(b + P.o_fro);
  w.norm = reinterpret_cast<double*>(b + P.o_norm);
  w.slots = reinterpret_cast<xword*>(b + P.o_slots);
  w.slotrows = reinterpret_cast<xword*>(b + P.o_slotrows);
  w.linv = b + P.o_linv;
  w.mtmp = b + P.o_mtmp;
  w.omega = b + P.o_omega;
  w.yorig = P.refine ? b + P.o_yorig : nullptr;
  w.tt = P.refine ? b + P.o_tt : nullptr;
  w.xr = P.refine ? b + P.o_x : nullptr;
  w.t1 = P.refine ? b + P.o_t1 : nullptr;
  w.pos_r = P.est > 0 ? reinterpret_cast<int*>(b + P.o_posr) : nullptr;
  w.order_r = P.est > 0 ? reinterpret_cast<int*>(b + P.o_orderr) : nullptr;
  w.ctrl_r = P.est > 0 ? reinterpret_cast<Ctrl*>(b + P.o_ctrlr) : nullptr;
  return w;
}

#define RID_LAUNCH_CHECK()                          \
  do {                                              \
    if (hipGetLastError() != hipSuccess) return RID_ERR_HIP; \
  } while (0)

#define RID_TRY(expr)             \
  do {                            \
    int rc_ = (expr);             \
    if (rc_ != RID_OK) return rc_; \
  } while (0)

// ---- sketch dispatch -------------------------------------------------------
// The method's draw that a launch belongs to: vectors [c0, c0 + w).  The
// sparse sign embedding is defined per draw, the Gaussian per vector.
struct Draw {
  int64_t c0;
  int w;
};

template <typename TC, int MT, int KC, bool VEC>
int launch_sketch_t(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                    int64_t c0, int w, const SketchGeom& g, bool norm, bool use_ctrl,
                    const Draw& dr, hipStream_t st) {
  dim3 grid((unsigned)g.ncolg, (unsigned)g.nsplit);
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const Ctrl* ctrl = use_ctrl ? W.ctrl : nullptr;
  TC* om = static_cast<TC*>(W.omega);
  const int64_t mpad = (int64_t)align_up((size_t)P.m, 64);
  // FP32 blocks of 64 vectors: the split operand form of Omega after it
  constexpr bool split = sizeof(TC) == 4 && MT == 4;
  uint32_t* oms = split ? reinterpret_cast<uint32_t*>(om + mpad * 64) : nullptr;
  long pm = prof_begin(KC_OMEGA, st);
  if (P.emb == RID_EMB_SPARSE_SIGN)
    hipLaunchKernelGGL(k_omega_ss<TC>, dim3((unsigned)ceil_div(mpad, 256)), dim3(256), 0, st, k0,
                       k1, (uint32_t)dr.c0, dr.w, (int)(c0 - dr.c0), w, g.wp, P.m, mpad, om, ctrl);
  else
    hipLaunchKernelGGL(k_omega<TC>, dim3((unsigned)ceil_div(mpad / 4 * g.wp, 256)), dim3(256), 0,
                       st, k0, k1, (uint32_t)c0, w, g.wp, P.m, mpad, om, ctrl);
  if (split)
    hipLaunchKernelGGL(k_omega_split<MT>, dim3((unsigned)ceil_div(mpad / 32 * MT * 64, 256)),
                       dim3(256), 0, st, reinterpret_cast<const float*>(om), mpad, oms, ctrl);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  pm = prof_begin(KC_SKETCH, st);
  if (norm)
    hipLaunchKernelGGL((k_sketch<TC, MT, KC, true, VEC>), grid, dim3(SketchShape<TC>::NT), 0, st,
                       static_cast<const TC*>(A), P.m, P.n, lda, om, oms, w, g.rows_per_split,
                       reinterpret_cast<TC*>(W.part), W.fro, W.nonfinite, ctrl);
  else
    hipLaunchKernelGGL((k_sketch<TC, MT, KC, false, VEC>), grid, dim3(SketchShape<TC>::NT), 0, st,
                       static_cast<const TC*>(A), P.m, P.n, lda, om, oms, w, g.rows_per_split,
                       reinterpret_cast<TC*>(W.part), W.fro, W.nonfinite, ctrl);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

template <typename TC, int KC, bool VEC>
int launch_sketch_mt(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                     int64_t c0, int w, const SketchGeom& g, bool norm, bool use_ctrl,
                     const Draw& dr, hipStream_t st) {
  switch (g.mt) {
    case 1:
      return launch_sketch_t<TC, 1, KC, VEC>(P, W, A, lda, seed, c0, w, g, norm, use_ctrl, dr, st);
    case 2:
      return launch_sketch_t<TC, 2, KC, VEC>(P, W, A, lda, seed, c0, w, g, norm, use_ctrl, dr, st);
    default:
      return launch_sketch_t<TC, 4, KC, VEC>(P, W, A, lda, seed, c0, w, g, norm, use_ctrl, dr, st);
  }
}

template <typename TC, int KC>
int launch_sketch(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                  int64_t c0, int w, const SketchGeom& g, bool norm, bool use_ctrl,
                  const Draw& dr, hipStream_t st) {
  // vector loads of NQ consecutive entries need lda % NQ == 0 and a base
  // aligned to 16 bytes (FP32: one 16-byte load; FP64: 16-byte pairs)
  constexpr int NQ = SketchShape<TC>::NQ;
  const bool vec = (lda % NQ == 0) && ((reinterpret_cast<uintptr_t>(A) & 15u) == 0);
  return vec ? launch_sketch_mt<TC, KC, true>(P, W, A, lda, seed, c0, w, g, norm, use_ctrl, dr, st)
             : launch_sketch_mt<TC, KC, false>(P, W, A, lda, seed, c0, w, g, norm, use_ctrl, dr,
                                               st);
}

// Row form: Omega over A's columns (P.m of them), then the row-form sketch.
template <typename TC, int MT, bool VEC>
int launch_sketch_rows_t(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                         int64_t c0, int w, const SketchGeomR& g, bool norm, bool use_ctrl,
                         const Draw& dr, hipStream_t st) {
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const Ctrl* ctrl = use_ctrl ? W.ctrl : nullptr;
  TC* om = static_cast<TC*>(W.omega);
  const int64_t mpad = (int64_t)align_up((size_t)P.m, 64);
  long pm = prof_begin(KC_OMEGA, st);
  if (P.emb == RID_EMB_SPARSE_SIGN)
    hipLaunchKernelGGL(k_omega_ss<TC>, dim3((unsigned)ceil_div(mpad, 256)), dim3(256), 0, st, k0,
                       k1, (uint32_t)dr.c0, dr.w, (int)(c0 - dr.c0), w, g.wp, P.m, mpad, om, ctrl);
  else
    hipLaunchKernelGGL(k_omega<TC>, dim3((unsigned)ceil_div(mpad / 4 * g.wp, 256)), dim3(256), 0,
                       st, k0, k1, (uint32_t)c0, w, g.wp, P.m, mpad, om, ctrl);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  dim3 grid((unsigned)g.ntile, (unsigned)g.nsplit);
  pm = prof_begin(KC_SKETCH, st);
  if (norm)
    hipLaunchKernelGGL((k_sketch_rows<TC, MT, true, VEC>), grid, dim3(256), 0, st,
                       static_cast<const TC*>(A), P.n, P.m, lda, om, w, g.cols_per_split, W.part,
                       W.fro, W.nonfinite, ctrl);
  else
    hipLaunchKernelGGL((k_sketch_rows<TC, MT, false, VEC>), grid, dim3(256), 0, st,
                       static_cast<const TC*>(A), P.n, P.m, lda, om, w, g.cols_per_split, W.part,
                       W.fro, W.nonfinite, ctrl);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

template <typename TC>
int launch_sketch_rows(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                       int64_t c0, int w, const SketchGeomR& g, bool norm, bool use_ctrl,
                       const Draw& dr, hipStream_t st) {
  // 4 consecutive entries per vector load: 16-byte aligned rows
  const bool vec = (lda % (16 / (int64_t)sizeof(TC)) == 0) &&
                   ((reinterpret_cast<uintptr_t>(A) & 15u) == 0);
#define RID_ROWS_MT(MTV)                                                                        \
  return vec ? launch_sketch_rows_t<TC, MTV, true>(P, W, A, lda, seed, c0, w, g, norm, use_ctrl, \
                                                    dr, st)                                      \
             : launch_sketch_rows_t<TC, MTV, false>(P, W, A, lda, seed, c0, w, g, norm,         \
                                                     use_ctrl, dr, st)
  switch (g.mt) {
    case 1: RID_ROWS_MT(1);
    case 2: RID_ROWS_MT(2);
    default: RID_ROWS_MT(4);
  }
#undef RID_ROWS_MT
}

template <int FMT, bool NORM>
int launch_sketch_lp(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                     int64_t c0, int w, const LpGeom& g, bool use_ctrl, hipStream_t st) {
  constexpr int ES = FMT == 1 ? 2 : 1;
  // the ring's 16-byte copies need 16-byte aligned rows
  const int aligned = ((lda * ES) % 16 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15u) == 0);
  const int vec8 = ((lda * ES) % 8 == 0) && ((reinterpret_cast<uintptr_t>(A) & 7u) == 0);
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const Ctrl* ctrl = use_ctrl ? W.ctrl : nullptr;
  const int64_t mpad = (int64_t)align_up((size_t)P.m, 64);
  float* om = static_cast<float*>(W.omega);
  unsigned char* rec = reinterpret_cast<unsigned char*>(om + mpad * 64);
  long pm = prof_begin(KC_OMEGA, st);
  hipLaunchKernelGGL(k_omega<float>, dim3((unsigned)ceil_div(mpad / 4 * 64, 256)), dim3(256), 0, st,
                     k0, k1, (uint32_t)c0, w, 64, P.m, mpad, om, ctrl);
  hipLaunchKernelGGL(k_omega_lp_records<FMT>, dim3((unsigned)ceil_div(mpad / 32 * 256, 256)),
                     dim3(256), 0, st, om, mpad, rec, ctrl);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  dim3 grid((unsigned)g.ncolg, (unsigned)g.nsplit);
  pm = prof_begin(KC_SKETCH, st);
  hipLaunchKernelGGL((k_sketch_lpr<FMT, NORM>), grid, dim3(kLprThreads), 0, st,
                     static_cast<const unsigned char*>(A), P.m, P.n, lda, P.scale, rec,
                     g.rows_per_split, reinterpret_cast<float*>(W.part), W.fro, W.nonfinite, ctrl,
                     aligned, vec8);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

// Two blocks of the low-precision forms in one pass (k_sketch_lpw): vectors
// [c0, c0 + w), 64 < w <= 128, Gaussian embedding, no norm pass.
template <int FMT>
int launch_sketch_lpw(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                      int64_t c0, int w, const LpGeom& g, bool use_ctrl, hipStream_t st) {
  constexpr int ES = FMT == 1 ? 2 : 1;
  const int aligned = ((lda * ES) % 16 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15u) == 0);
  const int vec8 = ((lda * ES) % 8 == 0) && ((reinterpret_cast<uintptr_t>(A) & 7u) == 0);
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  const Ctrl* ctrl = use_ctrl ? W.ctrl : nullptr;
  const int64_t mpad = (int64_t)align_up((size_t)P.m, 64);
  float* om = static_cast<float*>(W.omega);
  unsigned char* rec = reinterpret_cast<unsigned char*>(om + mpad * 128);
  long pm = prof_begin(KC_OMEGA, st);
  hipLaunchKernelGGL(k_omega<float>, dim3((unsigned)ceil_div(mpad / 4 * 128, 256)), dim3(256), 0,
                     st, k0, k1, (uint32_t)c0, w, 128, P.m, mpad, om, ctrl);
  hipLaunchKernelGGL((k_omega_lp_records<FMT, 8>), dim3((unsigned)ceil_div(mpad / 32 * 512, 256)),
                     dim3(256), 0, st, om, mpad, rec, ctrl);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  pm = prof_begin(KC_SKETCH2, st);
  hipLaunchKernelGGL((k_sketch_lpw<FMT>), dim3((unsigned)g.ncolg, (unsigned)g.nsplit),
                     dim3(kLprThreads), 0, st, static_cast<const unsigned char*>(A), P.m, P.n, lda,
                     rec, g.rows_per_split, reinterpret_cast<float*>(W.part), ctrl, aligned, vec8);
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

// Sketch vectors [c0, c0 + w) into columns [zcol, zcol + w) of `out`
// (n x ldo, dtype of the plan), in launches of at most 64 vectors (the
// low-precision forms: 128 after the first launch of a call's norm pass).
int sketch_block(const Plan& P, const Ws& W, const void* A, int64_t lda, uint64_t seed,
                 int64_t c0, int w, void* out, int64_t ldo, int zcol, bool first, bool use_ctrl,
                 hipStream_t st) {
  // the refinement step reads a copy of the sketch columns the factorisation
  // overwrites
  void* copy = (P.refine && out == W.z) ? W.yorig : nullptr;
  for (int off = 0, wc = 0; off < w; off += wc) {
    const bool norm = first && off == 0;
    wc = std::min(64, w - off);
    Ctrl* ctrl = use_ctrl ? W.ctrl : nullptr;
    if (low_precision(P.at) && !norm && w - off > 64 && P.emb == RID_EMB_GAUSSIAN) {
      wc = std::min(128, w - off);
      const int fmt = P.at == RID_BF16 ? 1 : 2;
      LpGeom g = sketch_geom_lp(P.m, P.n, fmt, P.cu, 2);
      RID_TRY(fmt == 1 ? launch_sketch_lpw<1>(P, W, A, lda, seed, c0 + off, wc, g, use_ctrl, st)
                       : launch_sketch_lpw<2>(P, W, A, lda, seed, c0 + off, wc, g, use_ctrl, st));
      const long pm = prof_begin(KC_REDUCE, st);
      hipLaunchKernelGGL(k_sketch_reduce_lp<float>, dim3((unsigned)ceil_div(P.n * wc, 256)),
                         dim3(256), 0, st, reinterpret_cast<const float*>(W.part), (int)g.nsplit,
                         P.n, 128, wc, fmt == 2 ? P.scale : nullptr, static_cast<float*>(out), ldo,
                         zcol + off, static_cast<float*>(copy), W.fro, 0, W.nonfinite, ctrl, 0);
      prof_end(pm, st);
      RID_LAUNCH_CHECK();
      continue;
    }
    const unsigned blocks = (unsigned)ceil_div(P.n * wc, 256);
    if (low_precision(P.at)) {
      // factor type is FP32 (checked by the caller)
      LpGeom g = sketch_geom_lp(P.m, P.n, P.at == RID_BF16 ? 1 : 2, P.cu);
      int rc;
      if (P.at == RID_BF16)
        rc = norm ? launch_sketch_lp<1, true>(P, W, A, lda, seed, c0 + off, wc, g, use_ctrl, st)
                  : launch_sketch_lp<1, false>(P, W, A, lda, seed, c0 + off, wc, g, use_ctrl, st);
      else
        rc = norm ? launch_sketch_lp<2, true>(P, W, A, lda, seed, c0 + off, wc, g, use_ctrl, st)
                  : launch_sketch_lp<2, false>(P, W, A, lda, seed, c0 + off, wc, g, use_ctrl, st);
      if (rc != RID_OK) return rc;
      const long pm = prof_begin(KC_REDUCE, st);
      hipLaunchKernelGGL(k_sketch_reduce_lp<float>, dim3(blocks), dim3(256), 0, st,
                         reinterpret_cast<const float*>(W.part), (int)g.nsplit, P.n, 64, wc,
                         P.at == RID_FP8_E4M3 ? P.scale : nullptr, static_cast<float*>(out), ldo,
                         zcol + off, static_cast<float*>(copy), W.fro, (int)(g.nsplit * g.ncolg),
                         W.nonfinite, ctrl, norm ? 1 : 0);
      prof_end(pm, st);
      RID_LAUNCH_CHECK();
      continue;
    }
    if (P.side == RID_ROWS) {
      SketchGeomR g = sketch_geom_rows(P.n, P.m, wc, P.cu);
      RID_TRY(P.dt == RID_F64 ? launch_sketch_rows<double>(P, W, A, lda, seed, c0 + off, wc, g,
                                                           norm, use_ctrl, Draw{c0, w}, st)
                              : launch_sketch_rows<float>(P, W, A, lda, seed, c0 + off, wc, g,
                                                          norm, use_ctrl, Draw{c0, w}, st));
      const long pm = prof_begin(KC_REDUCE, st);
      if (P.dt == RID_F64)
        hipLaunchKernelGGL((k_sketch_reduce<double, double>), dim3(blocks), dim3(256), 0, st,
                           W.part, (int)g.nsplit, P.n, g.wp, wc, static_cast<double*>(out), ldo,
                           zcol + off, static_cast<double*>(copy), W.fro,
                           (int)(g.nsplit * g.ntile), W.nonfinite, ctrl, norm ? 1 : 0);
      else
        hipLaunchKernelGGL((k_sketch_reduce<float, double>), dim3(blocks), dim3(256), 0, st, W.part,
                           (int)g.nsplit, P.n, g.wp, wc, static_cast<float*>(out), ldo,
                           zcol + off, static_cast<float*>(copy), W.fro,
                           (int)(g.nsplit * g.ntile), W.nonfinite, ctrl, norm ? 1 : 0);
      prof_end(pm, st);
      RID_LAUNCH_CHECK();
      continue;
    }
    SketchGeom g = sketch_geom(P.m, P.n, wc, P.dt, P.cu);
    int rc = (P.dt == RID_F64)
                 ? launch_sketch<double, 32>(P, W, A, lda, seed, c0 + off, wc, g, norm, use_ctrl,
                                             Draw{c0, w}, st)
                 : launch_sketch<float, 32>(P, W, A, lda, seed, c0 + off, wc, g, norm, use_ctrl,
                                            Draw{c0, w}, st);
    if (rc != RID_OK) return rc;
    const long pm = prof_begin(KC_REDUCE, st);
    if (P.dt == RID_F64)
      hipLaunchKernelGGL((k_sketch_reduce<double, double>), dim3(blocks), dim3(256), 0, st, W.part,
                         (int)g.nsplit, P.n, g.wp, wc, static_cast<double*>(out), ldo, zcol + off,
                         static_cast<double*>(copy), W.fro, (int)(g.nsplit * g.ncolg), W.nonfinite,
                         ctrl, norm ? 1 : 0);
    else
      hipLaunchKernelGGL((k_sketch_reduce<float, float>), dim3(blocks), dim3(256), 0, st,
                         reinterpret_cast<const float*>(W.part),
                         (int)g.nsplit, P.n, g.wp, wc, static_cast<float*>(out), ldo, zcol + off,
                         static_cast<float*>(copy), W.fro, (int)(g.nsplit * g.ncolg), W.nonfinite,
                         ctrl, norm ? 1 : 0);
    prof_end(pm, st);
    RID_LAUNCH_CHECK();
  }
  return RID_OK;
}

// ---- block update: U2 (triangular solve) then S (Schur GEMM) --------------
// K values per split of the split-K Schur update (k_schur_sk), at least.
constexpr int kSchurSplitMinK = 128;

// Column groups of a Schur launch for a block of w columns: split the
// workgroup's waves over columns when 64-row workgroups would leave the chip
// under-filled (fewer than 512 of them, two waves per SIMD).
int schur_cg(const Plan& P, int w) {
  const int nt = (w + 15) / 16;
  if (ceil_div(P.n, 64) >= 512 || nt < 2) return 1;
  if (ceil_div(P.n, 32) >= 512 || nt < 4) return 2;
  return 4;
}
// Workgroups (and FP64 norm partials) of that launch.
int64_t schur_parts(const Plan& P, int w) { return ceil_div(P.n, 64 / schur_cg(P, w)); }

// kb > 0 (the Remark-1 sample only): the columns already hold the Schur
// complement for the first kb pivots and are reduced by pivots kb..k-1.
template <typename TF>
int block_update_t(const Plan& P, const Ws& W, int kb, int k, int zcol, int w, bool norm,
                   hipStream_t st) {
  long pm = prof_begin(KC_TRSM, st);
  if (k > kb) {
    hipLaunchKernelGGL(k_gather_top<TF>, dim3((unsigned)ceil_div((int64_t)(k - kb) * w, 256)),
                       dim3(256), 0, st, static_cast<const TF*>(W.z), P.ldz, W.order, kb, k, zcol,
                       w, static_cast<TF*>(W.ytop), P.ldg, W.ctrl);
    RID_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_u2<TF>, dim3((unsigned)ceil_div(k - kb, 16), (unsigned)ceil_div(w, 64)),
                       dim3(512), 0, st, static_cast<const TF*>(W.ytop), P.ldg, kb, k, w,
                       static_cast<const TF*>(W.linv), P.ldl, static_cast<TF*>(W.u2t), P.ldu,
                       W.ctrl);
    RID_LAUNCH_CHECK();
  }
  if (P.refine && zcol < P.zr) {
    // keep U's block row in the pivot rows (the refinement solves with U)
    hipLaunchKernelGGL(k_store_u2<TF>, dim3((unsigned)ceil_div((int64_t)k * w, 256)), dim3(256),
                       0, st, static_cast<TF*>(W.z), P.ldz, W.order, k, zcol, w,
                       static_cast<const TF*>(W.u2t), P.ldu, W.ctrl);
    RID_LAUNCH_CHECK();
  }
  prof_end(pm, st);
  pm = prof_begin(KC_SCHUR, st);
  const int cg = schur_cg(P, w);
  const int nt = ((w + 15) / 16 + cg - 1) / cg;  // column tiles per wave
  dim3 grid((unsigned)schur_parts(P, w));
  // Long K: split-K form (about two workgroups per CU over the 64-row slabs,
  // measured faster than four or eight; each split at least 128 K values,
  // its FP64 partials in the sketch partials' buffer, which is free between
  // a sketch's reduction and the next sketch), then the in-place subtraction
  // with the same norm partials.
  if (kb == 0 && w <= 64 && k >= 2 * kSchurSplitMinK) {
    const int64_t slabs = ceil_div(P.n, 64);
    int64_t S = std::min<int64_t>(ceil_div(2 * (int64_t)P.cu, slabs), k / kSchurSplitMinK);
    S = std::min<int64_t>(S, (int64_t)(P.part_bytes / ((size_t)P.n * 64 * 8)));
    if (S >= 2) {
      const int ksplit = (int)(ceil_div(ceil_div(k, S), 64) * 64);
      S = ceil_div(k, ksplit);
      const int ntw = (w + 15) / 16;
      dim3 gsk((unsigned)slabs, (unsigned)S);
      // FP32: on the BF16 matrix cores through the three-part split
#define RID_SCHUR_SK(NTV)                                                                     \
  if constexpr (sizeof(TF) == 4)                                                             \
    hipLaunchKernelGGL((k_schur_skb<NTV>), gsk, dim3(256), 0, st,                              \
                       static_cast<const float*>(W.z), P.ldz, P.n, k, w,                      \
                       static_cast<const float*>(W.u2t), P.ldu, ksplit, W.part, W.ctrl);      \
  else                                                                                        \
    hipLaunchKernelGGL((k_schur_sk<TF, NTV>), gsk, dim3(256), 0, st,                           \
                       static_cast<const TF*>(W.z), P.ldz, P.n, k, w,                         \
                       static_cast<const TF*>(W.u2t), P.ldu, ksplit, W.part, W.ctrl)
      switch (ntw) {
        case 1: RID_SCHUR_SK(1); break;
        case 2: RID_SCHUR_SK(2); break;
        case 3: RID_SCHUR_SK(3); break;
        default: RID_SCHUR_SK(4); break;
      }
#undef RID_SCHUR_SK
      RID_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_schur_fin<TF>, grid, dim3(256), 0, st, static_cast<TF*>(W.z), P.ldz,
                         P.n, W.pos, zcol, w, W.part, (int)S, 64 / cg, W.norm, W.ctrl,
                         norm ? 1 : 0);
      prof_end(pm, st);
      RID_LAUNCH_CHECK();
      return RID_OK;
    }
  }
#define RID_SCHUR(NTV, CGV)                                                                   \
  hipLaunchKernelGGL((k_schur<TF, NTV, false, CGV>), grid, dim3(256), 0, st,                  \
                     static_cast<TF*>(W.z), P.ldz, P.n, W.pos, 0, k, zcol, w,                 \
                     static_cast<const TF*>(W.u2t), P.ldu, W.norm, W.ctrl, norm ? 1 : 0)
#define RID_SCHUR_FROM(NTV)                                                                   \
  hipLaunchKernelGGL((k_schur<TF, NTV, true, 1>), grid, dim3(256), 0, st,                     \
                     static_cast<TF*>(W.z), P.ldz, P.n, W.pos, kb, k, zcol, w,                \
                     static_cast<const TF*>(W.u2t), P.ldu, W.norm, W.ctrl, norm ? 1 : 0)
  if (kb > 0) {
    // the Remark-1 sample only (w <= 16, one column group)
    if (cg != 1 || nt != 1) return RID_ERR_ARG;
    RID_SCHUR_FROM(1);
  } else if (cg == 4) {
    if (nt == 1) RID_SCHUR(1, 4); else RID_SCHUR(2, 4);
  } else if (cg == 2) {
    switch (nt) {
      case 1: RID_SCHUR(1, 2); break;
      case 2: RID_SCHUR(2, 2); break;
      case 3: RID_SCHUR(3, 2); break;
      default: RID_SCHUR(4, 2); break;
    }
  } else {
    switch (nt) {
      case 1: RID_SCHUR(1, 1); break;
      case 2: RID_SCHUR(2, 1); break;
      case 3: RID_SCHUR(3, 1); break;
      case 4: RID_SCHUR(4, 1); break;
      case 5: RID_SCHUR(5, 1); break;
      case 6: RID_SCHUR(6, 1); break;
      case 7: RID_SCHUR(7, 1); break;
      default: RID_SCHUR(8, 1); break;
    }
  }
#undef RID_SCHUR
#undef RID_SCHUR_FROM
  prof_end(pm, st);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int block_update(const Plan& P, const Ws& W, int k, int zcol, int w, bool norm, hipStream_t st,
                 int kb = 0) {
  return P.dt == RID_F64 ? block_update_t<double>(P, W, kb, k, zcol, w, norm, st)
                         : block_update_t<float>(P, W, kb, k, zcol, w, norm, st);
}

int estimate(const Plan& P, const Ws& W, int w, double tol, int rel, int k, bool fixed,
             hipStream_t st) {
  hipLaunchKernelGGL(k_estimate, dim3(1), dim3(256), 0, st, W.ctrl, W.norm, (int)schur_parts(P, w), w,
                     tol, rel, k, (int)P.kcap, fixed ? 1 : 0);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

// ---- panel factorisation ---------------------------------------------------
template <typename TF>
int panel_state_t(const Plan& P, const Ws& W, int zcol, int w, int f, bool stop_full, int* pos,
                  int* order, Ctrl* ctrl, hipStream_t st) {
  const size_t lds = panel_lds(P.lupp_rows, w, sizeof(TF));
  // each of the 192 row threads keeps the flags of its rows in 32 bits
  if (lds > kMaxLds || w > P.wmax || P.lupp_rows > 192 * 32) return RID_ERR_ARG;
  const void* fn = (const void*)k_panel_lupp<TF>;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return RID_ERR_HIP;
  TF* z = static_cast<TF*>(W.z);
  int64_t ldz = P.ldz, n = P.n, mn = std::min(P.m, P.n);
  xword* xslot = W.slots;
  xword* xrow = W.slotrows;
  int wmax = (int)P.wmax;
  int rows = P.lupp_rows;
  int sf = stop_full ? 1 : 0;
  void* args[] = {&z, &ldz, &n, &zcol, &w, &f, &pos, &order, &ctrl,
                  &xslot, &xrow, &wmax, &rows, &mn, &sf};
  const long pm = prof_begin(KC_LUPP, st);
  const hipError_t e =
      hipLaunchCooperativeKernel(fn, dim3(P.lupp_g), dim3(256), args, (unsigned)lds, st);
  prof_end(pm, st);
  return e == hipSuccess ? RID_OK : RID_ERR_HIP;
}

template <typename TF>
int panel_t(const Plan& P, const Ws& W, int zcol, int w, int f, bool stop_full, hipStream_t st) {
  return panel_state_t<TF>(P, W, zcol, w, f, stop_full, W.pos, W.order, W.ctrl, st);
}

// Linv grows by the block row of the pivots just taken at k0 (at most f;
// the kernels read the actual count from the control block).
template <typename TF>
int linv_update_t(const Plan& P, const Ws& W, int k0, int f, hipStream_t st) {
  const long pm = prof_begin(KC_LINV, st);
  const size_t lds1 = (size_t)f * (f + 1) * sizeof(TF);
  const int x_in_lds = (2 * lds1 <= kMaxLds) ? 1 : 0;
  const size_t lds = x_in_lds ? 2 * lds1 : lds1;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_linv_diag<TF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)lds) != hipSuccess)
    return RID_ERR_HIP;
  hipLaunchKernelGGL(k_linv_diag<TF>, dim3(1), dim3(256), lds, st, static_cast<const TF*>(W.z),
                     P.ldz, W.order, k0, static_cast<TF*>(W.linv), P.ldl, W.ctrl, x_in_lds);
  RID_LAUNCH_CHECK();
  if (k0 > 0) {
    dim3 grid((unsigned)ceil_div(f, 16), (unsigned)ceil_div(k0, 64));
    hipLaunchKernelGGL(k_linv_b1<TF>, grid, dim3(256), 0, st, static_cast<const TF*>(W.z), P.ldz,
                       W.order, k0, static_cast<const TF*>(W.linv), P.ldl,
                       static_cast<TF*>(W.mtmp), W.ctrl);
    RID_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_linv_b2<TF>, grid, dim3(256), 0, st, static_cast<const TF*>(W.mtmp), k0,
                       static_cast<TF*>(W.linv), P.ldl, W.ctrl);
    RID_LAUNCH_CHECK();
  }
  prof_end(pm, st);
  return RID_OK;
}

// The caller's stream waits for the work forked to the side stream.
int side_join(SideLease& side, hipStream_t st) {
  if (!side.pending) return RID_OK;
  side.pending = false;
  return hipStreamWaitEvent(st, side.get()->join, 0) == hipSuccess ? RID_OK : RID_ERR_HIP;
}

// Panel on the caller's stream, then the growth of L1^{-1} forked to the side
// stream (on the caller's stream when there is none).  The caller joins
// before anything reads L1^{-1}.
int panel_fork(const Plan& P, const Ws& W, int zcol, int w, int f, bool stop_full, hipStream_t st,
               SideLease& side) {
  int rc = P.dt == RID_F64 ? panel_t<double>(P, W, zcol, w, f, stop_full, st)
                           : panel_t<float>(P, W, zcol, w, f, stop_full, st);
  if (rc != RID_OK) return rc;
  SideSet* ss = side.get();
  if (!ss)
    return P.dt == RID_F64 ? linv_update_t<double>(P, W, zcol, f, st)
                           : linv_update_t<float>(P, W, zcol, f, st);
  RID_TRY(side_join(side, st));  // at most one forked update at a time
  if (hipEventRecord(ss->fork, st) != hipSuccess || hipStreamWaitEvent(ss->s, ss->fork, 0) != hipSuccess)
    return RID_ERR_HIP;
  // from here on the side stream holds this call's work (joined by the lease
  // on an error return)
  side.caller = st;
  side.pending = true;
  rc = P.dt == RID_F64 ? linv_update_t<double>(P, W, zcol, f, ss->s)
                       : linv_update_t<float>(P, W, zcol, f, ss->s);
  const bool recorded = hipEventRecord(ss->join, ss->s) == hipSuccess;
  if (rc != RID_OK) return rc;
  return recorded ? RID_OK : RID_ERR_HIP;
}

int panel(const Plan& P, const Ws& W, int zcol, int w, int f, bool stop_full,
          hipStream_t st) {
  int rc = P.dt == RID_F64 ? panel_t<double>(P, W, zcol, w, f, stop_full, st)
                           : panel_t<float>(P, W, zcol, w, f, stop_full, st);
  if (rc != RID_OK) return rc;
  return P.dt == RID_F64 ? linv_update_t<double>(P, W, zcol, f, st)
                         : linv_update_t<float>(P, W, zcol, f, st);
}

// Panel exchange words: tag 0 never matches a step.
int zero_xwords(const Plan& P, const Ws& W, hipStream_t st) {
  const int64_t xw = (int64_t)(P.xwords_end - P.o_slots) / 4;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>(4096, ceil_div(xw, 256))), dim3(256),
                     0, st, reinterpret_cast<unsigned int*>(W.slots), xw);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

// ---- Remark-1 estimate of the current rank k (Sec. 3.2) --------------------
// Adaptive calls keep the sample's Schur complement S_r in Z columns
// [zr, zr+p): after the block that took pivots kb..k-1 the U2 and Schur
// kernels reduce it by those pivots only (K = k - kb), its non-pivot rows are
// copied to columns [zs, zs+p), and the panel kernel factors that copy with
// the private pivot state (pos_r, order_r, ctrl_r; its exchange words carry
// tags zs + s + 1, which repeat from one estimate to the next, hence the
// zeroing).  Fixed-rank calls factor their oversampling block (columns
// [k, k+p), already reduced by the caller) in place.  k_resid_est then forms
// the estimates and applies the stopping test.  Counted as one profiler
// class.
template <typename TF>
int resid_estimate_body(const Plan& P, const Ws& W, int kb, int k, int p, bool adaptive,
                        double tol, int rel, double* est_out, hipStream_t st) {
  const int zcol = adaptive ? (int)P.zs : k;
  if (adaptive) RID_TRY(block_update(P, W, k, (int)P.zr, p, true, st, kb));
  hipLaunchKernelGGL(k_resid_prep<TF>, dim3((unsigned)ceil_div(P.n, 256)), dim3(256), 0, st,
                     static_cast<TF*>(W.z), P.ldz, adaptive ? (int)P.zr : -1, zcol, p, P.n, W.pos,
                     W.pos_r, W.ctrl, W.ctrl_r);
  RID_LAUNCH_CHECK();
  const int f = (int)std::min<int64_t>(p, P.n - k);
  if (f < 1) return RID_OK;  // k = n: the decomposition is exact and done
  RID_TRY(zero_xwords(P, W, st));
  RID_TRY(panel_state_t<TF>(P, W, zcol, p, f, false, W.pos_r, W.order_r, W.ctrl_r, st));
  hipLaunchKernelGGL(k_resid_est<TF>, dim3(1), dim3(256), 0, st, W.ctrl, W.ctrl_r, W.order_r,
                     static_cast<const TF*>(W.z), P.ldz, zcol, p, W.norm, (int)schur_parts(P, p), P.n,
                     P.est, tol, rel, (int)P.kcap, adaptive ? 0 : 1, est_out);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int resid_estimate(const Plan& P, const Ws& W, int kb, int k, int p, bool adaptive, double tol,
                   int rel, double* est_out, hipStream_t st) {
  Profiler& pr = prof();
  const int saved = pr.override_class;
  pr.override_class = KC_RESID;
  const int rc =
      P.dt == RID_F64
          ? resid_estimate_body<double>(P, W, kb, k, p, adaptive, tol, rel, est_out, st)
          : resid_estimate_body<float>(P, W, kb, k, p, adaptive, tol, rel, est_out, st);
  pr.override_class = saved;
  return rc;
}

// ---- interpolation matrix and outputs --------------------------------------
// we, klim: the estimate block of the refinement choice (we vectors at Z
// column k, drawn when k < klim; see k_refine_pick).
template <typename TF>
int finish_t(const Plan& P, const Ws& W, void* T, int64_t ldt, int64_t* J, int32_t* k_out,
             double* err_est, int32_t* status, hipStream_t st, int we, int64_t klim) {
  hipLaunchKernelGGL(k_nonpiv, dim3(1), dim3(1024), 0, st, W.pos, P.n, W.nonpiv);
  RID_LAUNCH_CHECK();
  {
    const long pm = prof_begin(KC_TSOLVE, st);
    dim3 grid((unsigned)std::max<int64_t>(1, ceil_div(P.n, 64)),
              (unsigned)std::max<int64_t>(1, ceil_div(P.kcap, 64)));
    const TF* z = static_cast<const TF*>(W.z);
    const TF* linv = static_cast<const TF*>(W.linv);
    if (!P.refine) {
      hipLaunchKernelGGL((k_tgemm<TF, 0>), grid, dim3(256), 0, st, z, P.ldz, W.nonpiv, P.n, linv,
                         P.ldl, static_cast<TF*>(T), ldt, static_cast<const TF*>(nullptr),
                         (int64_t)0, W.ctrl);
      RID_LAUNCH_CHECK();
    } else {
      TF* tt = static_cast<TF*>(W.tt);
      TF* xr = static_cast<TF*>(W.xr);
      // T^T = L2 L1^{-1} (rows in ascending J^c order)
      hipLaunchKernelGGL((k_tgemm<TF, 1>), grid, dim3(256), 0, st, z, P.ldz, W.nonpiv, P.n, linv,
                         P.ldl, tt, P.ldl, static_cast<const TF*>(nullptr), (int64_t)0, W.ctrl);
      RID_LAUNCH_CHECK();
      // residual of the kept sketch in FP64, solve x U = R^T, T^T += x L1^{-1}
      hipLaunchKernelGGL(k_refine_resid, grid, dim3(256), 0, st,
                         static_cast<const float*>(W.yorig), P.ldz, W.order, W.nonpiv, P.n,
                         static_cast<const float*>(W.tt), P.ldl, static_cast<float*>(W.xr), P.ldl,
                         W.ctrl);
      RID_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_refine_solve, dim3((unsigned)std::max<int64_t>(1, ceil_div(P.n, 64))),
                         dim3(256), 0, st, static_cast<const float*>(W.z), P.ldz, W.order, P.n,
                         static_cast<float*>(W.xr), P.ldl, W.ctrl);
      RID_LAUNCH_CHECK();
      // the refined T, transposed, beside the unrefined one
      hipLaunchKernelGGL((k_tgemm<TF, 3>), grid, dim3(256), 0, st, static_cast<const TF*>(xr),
                         P.ldl, W.nonpiv, P.n, linv, P.ldl, static_cast<TF*>(W.t1), P.ldl,
                         static_cast<const TF*>(tt), P.ldl, W.ctrl);
      RID_LAUNCH_CHECK();
      // keep the one with the smaller residual on the last estimate block
      const int nparts = (int)std::max<int64_t>(1, ceil_div(P.n, 64));
      const int klim_i = P.refine_keep ? 0 : (int)std::min<int64_t>(klim, INT32_MAX);
      hipLaunchKernelGGL(k_refine_pick, dim3((unsigned)nparts), dim3(256), 0, st,
                         static_cast<const float*>(W.yorig), P.ldz, W.order, W.nonpiv, P.n, we,
                         klim_i, static_cast<const float*>(W.tt), static_cast<const float*>(W.t1),
                         P.ldl, W.part, W.ctrl);
      RID_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_refine_emit, grid, dim3(256), 0, st, static_cast<float*>(T), ldt,
                         static_cast<const float*>(W.tt), static_cast<const float*>(W.t1), P.ldl,
                         P.n, W.part, nparts, we, klim_i, W.ctrl);
      RID_LAUNCH_CHECK();
    }
    prof_end(pm, st);
  }
  const unsigned og = (unsigned)std::max<int64_t>(1, ceil_div(P.kcap, 256));
  hipLaunchKernelGGL(k_outputs, dim3(og), dim3(256), 0, st, W.ctrl, W.order, J, k_out, err_est,
                     status);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int finish(const Plan& P, const Ws& W, void* T, int64_t ldt, int64_t* J, int32_t* k_out,
           double* err_est, int32_t* status, hipStream_t st, int we = 0, int64_t klim = 0) {
  return P.dt == RID_F64
             ? finish_t<double>(P, W, T, ldt, J, k_out, err_est, status, st, we, klim)
             : finish_t<float>(P, W, T, ldt, J, k_out, err_est, status, st, we, klim);
}

int init(const Plan& P, const Ws& W, hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3((unsigned)ceil_div(P.n, 256)), dim3(256), 0, st, W.ctrl, W.pos,
                     P.n, W.nonfinite);
  RID_LAUNCH_CHECK();
  const int64_t words = P.kcap * P.ldl * (int64_t)esize(P.dt) / 4;
  hipLaunchKernelGGL(k_zero, dim3((unsigned)std::min<int64_t>(4096, ceil_div(words, 256))), dim3(256),
                     0, st, static_cast<unsigned int*>(W.linv), words);
  RID_LAUNCH_CHECK();
  return zero_xwords(P, W, st);
}

// est_out (nullable, device): -1 until an estimate is taken.
int init_est_out(double* est_out, hipStream_t st) {
  if (!est_out) return RID_OK;
  hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, st, est_out, 3, -1.0);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

bool valid_cfg(const rid_config* cfg) {
  if (!cfg || (cfg->dtype != RID_F64 && cfg->dtype != RID_F32)) return false;
  if (cfg->side != RID_COLUMNS && cfg->side != RID_ROWS) return false;
  // the row form reads A in the factor type
  if (cfg->side == RID_ROWS && cfg->a_type != cfg->dtype) return false;
  if (cfg->estimator < RID_EST_SCHUR || cfg->estimator > RID_EST_UR_MAX) return false;
  if (cfg->embedding != RID_EMB_GAUSSIAN && cfg->embedding != RID_EMB_SPARSE_SIGN) return false;
  // the low-precision sketch generates Gaussian entries inside its kernel
  if (cfg->embedding == RID_EMB_SPARSE_SIGN && cfg->a_type != cfg->dtype) return false;
  if (cfg->a_type != cfg->dtype) {
    if (cfg->dtype != RID_F32 || !low_precision(cfg->a_type)) return false;
    if (cfg->a_type == RID_FP8_E4M3 && !cfg->a_col_scale) return false;
  }
  return cfg->refine == 0 || ((cfg->refine == 1 || cfg->refine == 2) && cfg->dtype == RID_F32);
}

// The batched path reads A in the factor type, or FP32 blocks under an FP64
// factorisation.
bool valid_batched_cfg(const rid_config* cfg) {
  if (!cfg || cfg->refine != 0 || cfg->embedding != RID_EMB_GAUSSIAN || cfg->estimator != 0 ||
      cfg->side != RID_COLUMNS)
    return false;
  if (cfg->dtype == RID_F64 && cfg->a_type == RID_F32) return true;
  return valid_cfg(cfg) && cfg->a_type == cfg->dtype;
}

// The row-skeleton step reads A in the factor type, with no refinement or
// estimator.
bool valid_rows_cfg(const rid_config* cfg) {
  return valid_cfg(cfg) && cfg->a_type == cfg->dtype && cfg->refine == 0 && cfg->estimator == 0 &&
         cfg->side == RID_COLUMNS;
}

int64_t lds_kcap_limit(rid_dtype dt) { return (int64_t)(kMaxLds / esize(dt)); }

// ---- batched path ------------------------------------------------------------
struct BPlan {
  rid::BLayout L{};
  size_t total = 0;
  int G = 0;
};

// Persistent grid of the batched kernel chosen per (device, storage type,
// factor type, b, max_n rounded up to a power of two): the number of
// workgroups taking blocks from the queue (0 = one per compute unit).
struct GridKey {
  int dev, dt, at, b, nbucket;
  bool operator<(const GridKey& o) const {
    return std::tie(dev, dt, at, b, nbucket) < std::tie(o.dev, o.dt, o.at, o.b, o.nbucket);
  }
};
std::mutex grid_mu;
std::map<GridKey, int> grid_cache;

GridKey grid_key(const rid_config* cfg, int32_t b, int32_t max_n) {
  int dev = 0;
  (void)hipGetDevice(&dev);
  int nb = 64;
  while (nb < max_n) nb *= 2;
  return GridKey{dev, (int)cfg->dtype, (int)cfg->a_type, b, nb};
}

int batched_grid(const rid_config* cfg, int32_t b, int32_t max_n) {
  std::lock_guard<std::mutex> lk(grid_mu);
  auto it = grid_cache.find(grid_key(cfg, b, max_n));
  return it == grid_cache.end() ? 0 : it->second;
}

void set_batched_grid(const rid_config* cfg, int32_t b, int32_t max_n, int grid) {
  std::lock_guard<std::mutex> lk(grid_mu);
  grid_cache[grid_key(cfg, b, max_n)] = grid;
}

bool bplan(int32_t maxn, int32_t maxk, int32_t b, rid_dtype dt, BPlan& P) {
  DeviceInfo di = device_info();
  if (!di.ok) return false;
  // the same layout function gives the kernel its slice carving
  P.L = rid::batched_layout(maxn, maxk, b, (int64_t)esize(dt), 0);
  P.G = di.cu;
  P.total = kAlign + (size_t)P.G * (size_t)P.L.slice;
  return true;
}

// ---- workspace for callers that cannot allocate ------------------------------
// A file-scope device array serves as the fixed-rank call's workspace for
// callers that cannot call hipMalloc.  Each device that loads the library
// holds its own copy until the process ends.  In host code the array's name is
// only a stand-in for the device symbol: its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) and only that
// address is ever handed to kernels.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* scratch_addr[64] = {};
std::mutex scratch_mu;

// Device address of the current device's copy of `scratch` (nullptr on error).
void* scratch_address() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    scratch_addr[dev] = p;
  }
  return scratch_addr[dev];
}

}  // namespace


extern "C" {

size_t rid_workspace_bytes(int64_t m, int64_t n, int64_t kmax, int64_t b, const rid_config* cfg) {
  if (m < 1 || n < 1 || kmax < 1 || b < 0 || !valid_cfg(cfg)) return 0;
  Plan P;
  // with a Remark-1 estimator and a sample width, the adaptive call's layout
  // (a superset of the fixed-rank call's)
  const bool sample = cfg->estimator > 0 && cfg->resid_p >= 1 && cfg->resid_p <= kResidPMax;
  if (!plan_for(m, n, kmax, b, cfg, P, sample)) return 0;
  return P.total;
}

const char* rid_status_string(int s) {
  switch (s) {
    case RID_OK: return "RID_OK";
    case RID_NOT_CONVERGED: return "RID_NOT_CONVERGED";
    case RID_RANK_DEFICIENT: return "RID_RANK_DEFICIENT";
    case RID_ERR_ARG: return "RID_ERR_ARG";
    case RID_ERR_NONFINITE: return "RID_ERR_NONFINITE";
    case RID_ERR_HIP: return "RID_ERR_HIP";
    case RID_ERR_WORKSPACE: return "RID_ERR_WORKSPACE";
    default: return "RID_UNKNOWN";
  }
}

int rid_lupp_fixed_rank(const void* A, int64_t m, int64_t n, int64_t lda, int64_t k, int64_t p,
                        const rid_config* cfg, int64_t* J, void* T, int64_t ldt, int32_t* k_out,
                        double* err_est, int32_t* status, void* work, size_t work_bytes,
                        hipStream_t stream) {
  if (!A || !J || !T || !k_out || !err_est || !status || !work || !valid_cfg(cfg))
    return RID_ERR_ARG;
  // T has a column per candidate: A's columns, or its rows in the row form
  const int64_t ncand = cfg->side == RID_ROWS ? m : n;
  if (m < 1 || n < 1 || lda < n || ldt < ncand || k < 1 || k > std::min(m, n) || p < 0 ||
      p > kMaxW || m > INT32_MAX || n > INT32_MAX)
    return RID_ERR_ARG;
  if (k > lds_kcap_limit(cfg->dtype)) return RID_ERR_ARG;
  if (cfg->estimator > 0 && p < 1) return RID_ERR_ARG;
  Plan P;
  if (!plan_for(m, n, k + p, p, cfg, P)) return RID_ERR_HIP;
  if (work_bytes < P.total) return RID_ERR_WORKSPACE;
  if (P.lupp_lds > kMaxLds) return RID_ERR_ARG;
  Ws W = carve(P, work);
  RID_TRY(init(P, W, stream));
  RID_TRY(init_est_out(cfg->estimator > 0 ? cfg->est_out : nullptr, stream));
  // all k + p vectors up front, as two draws of the method (k for the
  // pivots, p for the estimate); each sketch launch covers <= 64 vectors
  RID_TRY(sketch_block(P, W, A, lda, cfg->seed, 0, (int)k, W.z, P.ldz, 0, true, true, stream));
  if (p > 0)
    RID_TRY(sketch_block(P, W, A, lda, cfg->seed, k, (int)p, W.z, P.ldz, (int)k, false, true,
                         stream));
  for (int64_t k0 = 0; k0 < k; k0 += kPanel) {
    const int f = (int)std::min<int64_t>(kPanel, k - k0);
    if (k0 > 0) RID_TRY(block_update(P, W, (int)k0, (int)k0, f, false, stream));
    RID_TRY(panel(P, W, (int)k0, f, f, false, stream));
  }
  if (p > 0) {
    RID_TRY(block_update(P, W, (int)k, (int)k, (int)p, true, stream));
    if (cfg->estimator > 0)
      RID_TRY(resid_estimate(P, W, 0, (int)k, (int)p, false, 0.0, 0, cfg->est_out, stream));
    else
      RID_TRY(estimate(P, W, (int)p, 0.0, 0, (int)k, true, stream));
  }
  // the p estimate vectors sit at Z column k (ctrl->k = k)
  return finish(P, W, T, ldt, J, k_out, err_est, status, stream, (int)p, p > 0 ? k + 1 : 0);
}

size_t rid_noalloc_max_bytes(void) { return kScratchBytes; }

int rid_lupp_fixed_rank_noalloc(const void* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                                int64_t p, const rid_config* cfg, int64_t* J, void* T,
                                int64_t ldt, int32_t* k_out, double* err_est, int32_t* status,
                                hipStream_t stream) {
  if (!A || !J || !T || !k_out || !err_est || !status || !valid_cfg(cfg)) return RID_ERR_ARG;
  if (m < 1 || n < 1 || k < 1 || k > std::min(m, n) || p < 0 || p > kMaxW) return RID_ERR_ARG;
  Plan P;  // the plan rid_lupp_fixed_rank makes for these sizes
  if (!plan_for(m, n, k + p, p, cfg, P)) return RID_ERR_HIP;
  if (P.total > kScratchBytes) return RID_ERR_WORKSPACE;
  void* ws = scratch_address();
  if (!ws) return RID_ERR_HIP;
  // the same enqueue as the workspace form; init() clears what must start at zero
  return rid_lupp_fixed_rank(A, m, n, lda, k, p, cfg, J, T, ldt, k_out, err_est, status, ws,
                             kScratchBytes, stream);
}

int rid_lupp_adaptive(const void* A, int64_t m, int64_t n, int64_t lda, int64_t b, double tol,
                      int64_t kmax, const rid_config* cfg, int64_t* J, void* T, int64_t ldt,
                      int32_t* k_out, double* err_est, int32_t* status, void* work,
                      size_t work_bytes, hipStream_t stream) {
  if (!A || !J || !T || !k_out || !err_est || !status || !work || !valid_cfg(cfg))
    return RID_ERR_ARG;
  const int64_t ncand = cfg->side == RID_ROWS ? m : n;
  if (m < 1 || n < 1 || lda < n || ldt < ncand || b < 1 || b > kMaxW || kmax < 1 ||
      !(tol >= 0.0) || m > INT32_MAX || n > INT32_MAX)
    return RID_ERR_ARG;
  const int64_t mn = std::min(m, n);
  const int64_t kcap = std::min(kmax, mn);
  if (kcap > lds_kcap_limit(cfg->dtype)) return RID_ERR_ARG;
  const int est = cfg->estimator;
  if (est > 0 && (cfg->resid_p < 1 || cfg->resid_p > kResidPMax)) return RID_ERR_ARG;
  Plan P;
  if (!plan_for(m, n, kmax, b, cfg, P, true)) return RID_ERR_HIP;
  if (work_bytes < P.total) return RID_ERR_WORKSPACE;
  if (P.lupp_lds > kMaxLds) return RID_ERR_ARG;
  Ws W = carve(P, work);
  RID_TRY(init(P, W, stream));
  const int w0 = (int)std::min<int64_t>(b, kcap);
  RID_TRY(sketch_block(P, W, A, lda, cfg->seed, 0, w0, W.z, P.ldz, 0, true, true, stream));
  int64_t k = w0, cnext = w0;
  if (est > 0) {
    // Remark 1: the sample is drawn once; every factored block is followed
    // by the estimate of its rank, and no block is drawn only to measure.
    // The next block is sketched while L1^{-1} grows on the side stream (a
    // pass that is wasted only when the estimate then stops the call).
    const int p = cfg->resid_p;
    SideLease side;
    RID_TRY(init_est_out(cfg->est_out, stream));
    RID_TRY(panel_fork(P, W, 0, w0, w0, true, stream, side));
    RID_TRY(sketch_block(P, W, A, lda, cfg->seed, kResidC0, p, W.z, P.ldz, (int)P.zr, false, true,
                         stream));
    if (k < kcap) {
      RID_TRY(sketch_block(P, W, A, lda, cfg->seed, cnext, (int)b, W.z, P.ldz, (int)k, false,
                           true, stream));
      cnext += b;
    }
    RID_TRY(side_join(side, stream));
    RID_TRY(resid_estimate(P, W, 0, (int)k, p, true, tol, cfg->tol_relative, cfg->est_out,
                           stream));
    while (k < kcap) {
      RID_TRY(block_update(P, W, (int)k, (int)k, (int)b, false, stream));
      const int f = (int)std::min<int64_t>(b, kcap - k);
      RID_TRY(panel_fork(P, W, (int)k, (int)b, f, true, stream, side));
      const int64_t k0 = k;
      k += f;
      if (k < kcap) {
        RID_TRY(sketch_block(P, W, A, lda, cfg->seed, cnext, (int)b, W.z, P.ldz, (int)k, false,
                             true, stream));
        cnext += b;
      }
      RID_TRY(side_join(side, stream));
      RID_TRY(resid_estimate(P, W, (int)k0, (int)k, p, true, tol, cfg->tol_relative,
                             cfg->est_out, stream));
    }
    RID_TRY(side_join(side, stream));
    // a stop below kcap has the next block sketched at column k
    return finish(P, W, T, ldt, J, k_out, err_est, status, stream, (int)b, kcap);
  }
  // Alg. 1 with the growth of L1^{-1} overlapping the next block's sketch.
  // The low-precision forms (Gaussian embedding, b <= 64) draw two blocks
  // per pass over A after the first (k_sketch_lpw), the second into the Z
  // columns after the first, where the next block starts once the first is
  // fully factored; Omega's entries depend only on (seed, vector, row), so
  // each block's sketch is the one a pass of its own would give.  `ahead`
  // counts the sketched columns from column k on.
  SideLease side;
  RID_TRY(panel_fork(P, W, 0, w0, w0, true, stream, side));
  const bool pairs = low_precision(P.at) && P.emb == RID_EMB_GAUSSIAN && b <= 64;
  int64_t ahead = 0;
  while (k < mn) {
    if (ahead == 0) {
      // a second block is factored or estimated only if this one takes b pivots
      const int64_t nb = (pairs && kcap - k >= b && k + b < mn) ? 2 : 1;
      RID_TRY(sketch_block(P, W, A, lda, cfg->seed, cnext, (int)(nb * b), W.z, P.ldz, (int)k,
                           false, true, stream));
      cnext += nb * b;
      ahead = nb * b;
    }
    RID_TRY(side_join(side, stream));
    RID_TRY(block_update(P, W, (int)k, (int)k, (int)b, true, stream));
    RID_TRY(estimate(P, W, (int)b, tol, cfg->tol_relative, (int)k, false, stream));
    if (k >= kcap) break;
    const int f = (int)std::min<int64_t>(b, kcap - k);
    RID_TRY(panel_fork(P, W, (int)k, (int)b, f, true, stream, side));
    ahead -= b;
    if (f < b && ahead > 0) {
      // (not reached: a pair is drawn only when f = b) the next block would
      // start at column k + f; draw its vectors again there
      cnext -= ahead;
      ahead = 0;
    }
    k += f;
  }
  RID_TRY(side_join(side, stream));
  // every estimate of Alg. 1 measures the block at column k (none at k = min(m, n))
  return finish(P, W, T, ldt, J, k_out, err_est, status, stream, (int)b, mn);
}

size_t rid_rows_workspace_bytes(int64_t m, int64_t k, const rid_config* cfg) {
  if (m < 1 || k < 1 || k > m || !valid_rows_cfg(cfg)) return 0;
  Plan P;
  if (!plan_rows(m, k, cfg, P)) return 0;
  return P.total;
}

int rid_lupp_rows(const void* A, int64_t m, int64_t n, int64_t lda, const int64_t* J, int64_t k,
                  const rid_config* cfg, int64_t* I, void* Tr, int64_t ldtr, int32_t* k_out,
                  int32_t* status, void* work, size_t work_bytes, hipStream_t stream) {
  if (!A || !J || !I || !Tr || !k_out || !status || !work || !cfg || !valid_rows_cfg(cfg))
    return RID_ERR_ARG;
  if (m < 1 || n < 1 || lda < n || k < 1 || k > std::min(m, n) || ldtr < m || m > INT32_MAX ||
      n > INT32_MAX)
    return RID_ERR_ARG;
  if (k > lds_kcap_limit(cfg->dtype)) return RID_ERR_ARG;
  Plan P;
  if (!plan_rows(m, k, cfg, P)) return RID_ERR_HIP;
  if (work_bytes < P.total) return RID_ERR_WORKSPACE;
  if (P.lupp_lds > kMaxLds) return RID_ERR_ARG;
  Ws W = carve(P, work);
  RID_TRY(init(P, W, stream));
  const bool f64 = P.dt == RID_F64;
  if (f64)
    hipLaunchKernelGGL(k_gather_cols<double>, dim3((unsigned)m), dim3(256), 0, stream,
                       static_cast<const double*>(A), lda, m, n, J, (int)k,
                       static_cast<double*>(W.z), P.ldz, W.ctrl);
  else
    hipLaunchKernelGGL(k_gather_cols<float>, dim3((unsigned)m), dim3(256), 0, stream,
                       static_cast<const float*>(A), lda, m, n, J, (int)k,
                       static_cast<float*>(W.z), P.ldz, W.ctrl);
  RID_LAUNCH_CHECK();
  for (int64_t k0 = 0; k0 < k; k0 += kPanel) {
    const int f = (int)std::min<int64_t>(kPanel, k - k0);
    if (k0 > 0) RID_TRY(block_update(P, W, (int)k0, (int)k0, f, false, stream));
    RID_TRY(panel(P, W, (int)k0, f, f, false, stream));
  }
  // Tr = W(I^c, :)^T = (L2 L1^{-1})^T: k_out rows of ldtr, column q for the
  // q-th non-skeleton row in ascending index (the layout of T)
  hipLaunchKernelGGL(k_nonpiv, dim3(1), dim3(1024), 0, stream, W.pos, P.n, W.nonpiv);
  RID_LAUNCH_CHECK();
  {
    const long pm = prof_begin(KC_TSOLVE, stream);
    dim3 grid((unsigned)ceil_div(m, 64), (unsigned)ceil_div(k, 64));
    if (f64)
      hipLaunchKernelGGL((k_tgemm<double, 0>), grid, dim3(256), 0, stream,
                         static_cast<const double*>(W.z), P.ldz, W.nonpiv, P.n,
                         static_cast<const double*>(W.linv), P.ldl, static_cast<double*>(Tr), ldtr,
                         static_cast<const double*>(nullptr), (int64_t)0, W.ctrl);
    else
      hipLaunchKernelGGL((k_tgemm<float, 0>), grid, dim3(256), 0, stream,
                         static_cast<const float*>(W.z), P.ldz, W.nonpiv, P.n,
                         static_cast<const float*>(W.linv), P.ldl, static_cast<float*>(Tr), ldtr,
                         static_cast<const float*>(nullptr), (int64_t)0, W.ctrl);
    prof_end(pm, stream);
    RID_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_outputs, dim3((unsigned)std::max<int64_t>(1, ceil_div(k, 256))), dim3(256),
                     0, stream, W.ctrl, W.order, I, k_out, W.norm, status);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

size_t rid_certificate_workspace_bytes(int64_t m, int64_t n, int64_t p, const rid_config* cfg) {
  // the sketch's plan, then the FP64 partials of the split certificate products
  if (m < 1 || n < 1 || p < 1 || p > kCertPMax || !valid_cfg(cfg) || cfg->side != RID_COLUMNS)
    return 0;
  rid_config c = *cfg;
  c.estimator = 0;
  c.embedding = RID_EMB_GAUSSIAN;  // the certificate draws Gaussian vectors
  Plan P;
  if (!plan_for(m, n, p, p, &c, P)) return 0;
  return align_up(P.total, kAlign) + cert_part_bytes(n, p);
}

int rid_certificate(const void* A, int64_t m, int64_t n, int64_t lda, const int64_t* J, int64_t k,
                    const void* T, int64_t ldt, int64_t p, int64_t c0, const rid_config* cfg,
                    double* cert, void* work, size_t work_bytes, hipStream_t stream) {
  if (!A || (k > 0 && !J) || (k > 0 && k < n && !T) || !cert || !work || !valid_cfg(cfg) ||
      cfg->side != RID_COLUMNS)
    return RID_ERR_ARG;
  if (m < 1 || n < 1 || lda < n || k < 0 || k > n || p < 1 || p > kCertPMax || c0 < 0 ||
      c0 + p > (int64_t(1) << 32) || (k > 0 && ldt < n - k) || m > INT32_MAX || n > INT32_MAX)
    return RID_ERR_ARG;
  rid_config c = *cfg;
  c.estimator = 0;
  c.embedding = RID_EMB_GAUSSIAN;  // the certificate draws Gaussian vectors
  Plan P;
  if (!plan_for(m, n, p, p, &c, P)) return RID_ERR_HIP;
  if (work_bytes < align_up(P.total, kAlign) + cert_part_bytes(n, p)) return RID_ERR_WORKSPACE;
  Ws W = carve(P, work);
  double* cpart = reinterpret_cast<double*>(static_cast<char*>(work) + align_up(P.total, kAlign));
  const unsigned gn = (unsigned)ceil_div(n, 256);
  hipLaunchKernelGGL(k_cert_clear, dim3(gn), dim3(256), 0, stream, W.pos, n, W.ctrl);
  RID_LAUNCH_CHECK();
  // Yc^T in Z's first p columns
  RID_TRY(sketch_block(P, W, A, lda, cfg->seed, c0, (int)p, W.z, P.ldz, 0, false, true, stream));
  if (k > 0) {
    hipLaunchKernelGGL(k_cert_mark, dim3((unsigned)ceil_div(k, 256)), dim3(256), 0, stream, J, k,
                       W.pos, n, W.ctrl);
    RID_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_nonpiv, dim3(1), dim3(1024), 0, stream, W.pos, n, W.nonpiv);
  RID_LAUNCH_CHECK();
  const int64_t nr = n - k;
  // squared residual sums: one per 256 non-skeleton columns, in the Schur
  // partials' buffer (ceil(n/16) entries)
  const int nparts = (int)std::max<int64_t>(1, ceil_div(nr, 256));
  const bool f64 = P.dt == RID_F64;
  if (nr > 0) {
    // skeleton ranges of about 128 each, so that the products fill the chip
    const int S = (int)std::max<int64_t>(1, std::min<int64_t>(kCertSplitMax, ceil_div(k, 128)));
    dim3 gp((unsigned)nparts, (unsigned)S);
    if (f64) {
      hipLaunchKernelGGL((k_cert<double, kCertPMax>), gp, dim3(256), 0, stream,
                         static_cast<const double*>(W.z), P.ldz, (int)p, J, k, nr,
                         static_cast<const double*>(T), ldt, cpart, W.ctrl);
      RID_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_cert_resid<double>, dim3((unsigned)nparts), dim3(256), 0, stream,
                         static_cast<const double*>(W.z), P.ldz, (int)p, W.nonpiv, nr, cpart, S,
                         W.norm, W.ctrl);
    } else {
      hipLaunchKernelGGL((k_cert<float, kCertPMax>), gp, dim3(256), 0, stream,
                         static_cast<const float*>(W.z), P.ldz, (int)p, J, k, nr,
                         static_cast<const float*>(T), ldt, cpart, W.ctrl);
      RID_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_cert_resid<float>, dim3((unsigned)nparts), dim3(256), 0, stream,
                         static_cast<const float*>(W.z), P.ldz, (int)p, W.nonpiv, nr, cpart, S,
                         W.norm, W.ctrl);
    }
    RID_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, stream, W.norm, 1, 0.0);
    RID_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_cert_reduce, dim3(1), dim3(256), 0, stream, W.norm, nparts, (int)p, W.ctrl,
                     cert);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_debug_gaussian(uint64_t seed, int64_t c0, int64_t w, int64_t m, int dtype, void* out,
                       hipStream_t stream) {
  if (!out || w < 1 || m < 1 || c0 < 0 || (dtype != RID_F64 && dtype != RID_F32))
    return RID_ERR_ARG;
  const int64_t nq = (m + 3) / 4;
  const unsigned blocks = (unsigned)ceil_div(nq * w, 256);
  const uint32_t k0 = (uint32_t)(seed & 0xffffffffu), k1 = (uint32_t)(seed >> 32);
  if (dtype == RID_F64)
    hipLaunchKernelGGL(k_gaussian<double>, dim3(blocks), dim3(256), 0, stream, k0, k1, c0, w, m,
                       static_cast<double*>(out));
  else
    hipLaunchKernelGGL(k_gaussian<float>, dim3(blocks), dim3(256), 0, stream, k0, k1, c0, w, m,
                       static_cast<float*>(out));
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_debug_sketch(const void* A, int64_t m, int64_t n, int64_t lda, int64_t c0, int64_t w,
                     const rid_config* cfg, void* Yt, int64_t ldy, void* work, size_t work_bytes,
                     hipStream_t stream) {
  if (!A || !Yt || !work || !valid_cfg(cfg) || m < 1 || n < 1 || lda < n || w < 1 ||
      w > kMaxW || ldy < w || c0 < 0)
    return RID_ERR_ARG;
  Plan P;
  if (!plan_for(m, n, w, w, cfg, P)) return RID_ERR_HIP;
  if (work_bytes < P.total) return RID_ERR_WORKSPACE;
  Ws W = carve(P, work);
  RID_TRY(init(P, W, stream));
  // the norm pass rides on the sketch of vectors from 0, as in a decomposition
  return sketch_block(P, W, A, lda, cfg->seed, c0, (int)w, Yt, ldy, 0, c0 == 0, true, stream);
}

size_t rid_batched_workspace_bytes(int32_t max_n, int32_t max_kmax, int32_t b,
                                   const rid_config* cfg) {
  if (max_n < 1 || max_n > rid::kBMaxN || max_kmax < 1 || b < 1 || b > rid::kBPW ||
      !valid_batched_cfg(cfg))
    return 0;
  BPlan P;
  if (!bplan(max_n, std::min(max_kmax, max_n), b, cfg->dtype, P)) return 0;
  return P.total;
}

int rid_lupp_batched(int32_t nblk, const void* const* A, const int64_t* lda, const int32_t* m,
                     const int32_t* n, int32_t b, double tol, const int32_t* kmax,
                     const int32_t* k_hint, const rid_config* cfg, int32_t* const* J,
                     void* const* T, const int64_t* ldt, int32_t* k_out, double* err_est,
                     int32_t* status, int32_t* passes, const int32_t* order, int32_t max_n,
                     int32_t max_kmax, void* work, size_t work_bytes, hipStream_t stream) {
  if (nblk < 0 || !valid_batched_cfg(cfg) || b < 1 || b > rid::kBPW || !(tol >= 0.0) || max_n < 1 ||
      max_n > rid::kBMaxN || max_kmax < 1 || !work)
    return RID_ERR_ARG;
  if (nblk == 0) return RID_OK;
  if (!A || !lda || !m || !n || !kmax || !J || !T || !ldt || !k_out || !err_est || !status)
    return RID_ERR_ARG;
  BPlan P;
  const int32_t maxk = std::min(max_kmax, max_n);
  if (!bplan(max_n, maxk, b, cfg->dtype, P)) return RID_ERR_HIP;
  if (work_bytes < P.total) return RID_ERR_WORKSPACE;
  // FP32 batches that need a workgroup to take a second block from the queue
  // ended twice with a GPU memory fault whose cause is not known; until it is,
  // an FP32 call takes at most one block per resident workgroup.
  if (cfg->dtype == RID_F32 && nblk > P.G) return RID_ERR_ARG;
  unsigned* queue = static_cast<unsigned*>(work);
  unsigned char* base = static_cast<unsigned char*>(work) + kAlign;
  hipLaunchKernelGGL(k_batched_init, dim3(1), dim3(1), 0, stream, queue);
  RID_LAUNCH_CHECK();
  // persistent workgroups: one per compute unit unless a smaller grid was
  // chosen for this key (rid_batched_autotune / rid_batched_set_grid; FP64
  // factorisations only: an FP32 one keeps one block per workgroup)
  const int g_set = cfg->dtype == RID_F64 ? batched_grid(cfg, b, max_n) : 0;
  const int grid = std::min<int>(g_set > 0 ? std::min(g_set, P.G) : P.G, nblk);
  const long pm = prof_begin(KC_BATCHED, stream);
#define RID_BATCHED(TFV, TAV)                                                                  \
  hipLaunchKernelGGL((k_batched<rid::kBT, TFV, TAV>), dim3(grid), dim3(rid::kBT), 0, stream,    \
                     nblk, A, lda, m, n, b, tol, cfg->tol_relative, kmax, k_hint, cfg->seed, J, T, \
                     ldt, k_out, err_est, status, passes, order, queue, base, P.L, max_n, maxk)
  if (cfg->dtype == RID_F64 && cfg->a_type == RID_F32)
    RID_BATCHED(double, float);
  else if (cfg->dtype == RID_F64)
    RID_BATCHED(double, double);
  else
    RID_BATCHED(float, float);
#undef RID_BATCHED
  prof_end(pm, stream);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_batched_set_grid(const rid_config* cfg, int32_t b, int32_t max_n, int32_t grid) {
  if (!valid_batched_cfg(cfg) || cfg->dtype != RID_F64 || b < 1 || b > rid::kBPW || max_n < 1 ||
      max_n > rid::kBMaxN || grid < 0)
    return RID_ERR_ARG;
  set_batched_grid(cfg, b, max_n, grid);
  return RID_OK;
}

int rid_batched_autotune(int32_t nblk, const void* const* A, const int64_t* lda, const int32_t* m,
                         const int32_t* n, int32_t b, double tol, const int32_t* kmax,
                         const int32_t* k_hint, const rid_config* cfg, int32_t* const* J,
                         void* const* T, const int64_t* ldt, int32_t* k_out, double* err_est,
                         int32_t* status, int32_t* passes, const int32_t* order, int32_t max_n,
                         int32_t max_kmax, void* work, size_t work_bytes, hipStream_t stream,
                         int32_t* grid_out, float* ms_out) {
  if (!valid_batched_cfg(cfg) || nblk < 1 || b < 1 || b > rid::kBPW || max_n < 1 ||
      max_n > rid::kBMaxN)
    return RID_ERR_ARG;
  DeviceInfo di = device_info();
  if (!di.ok) return RID_ERR_HIP;
  // candidates: all compute units, three quarters, half (FP32 factorisations
  // never take more blocks than workgroups, so their grid is not tuned)
  const int G = di.cu;
  const int cand[kGridCandidates] = {G, (3 * G) / 4, G / 2};
  const int ncand = cfg->dtype == RID_F64 ? kGridCandidates : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return RID_ERR_HIP;
  }
  const int saved = batched_grid(cfg, b, max_n);
  float best = -1.0f;
  int best_g = 0;
  int rc = RID_OK;
  for (int i = 0; i < ncand && rc == RID_OK; ++i) {
    set_batched_grid(cfg, b, max_n, cand[i]);
    float ts[3] = {0.f, 0.f, 0.f};
    // one untimed call, then the median of three timed ones
    for (int rep = 0; rep < 4 && rc == RID_OK; ++rep) {
      float t = 0.0f;
      if (hipEventRecord(e0, stream) != hipSuccess) rc = RID_ERR_HIP;
      if (rc == RID_OK)
        rc = rid_lupp_batched(nblk, A, lda, m, n, b, tol, kmax, k_hint, cfg, J, T, ldt, k_out,
                              err_est, status, passes, order, max_n, max_kmax, work, work_bytes,
                              stream);
      if (rc == RID_OK && (hipEventRecord(e1, stream) != hipSuccess ||
                           hipEventSynchronize(e1) != hipSuccess ||
                           hipEventElapsedTime(&t, e0, e1) != hipSuccess))
        rc = RID_ERR_HIP;
      if (rep > 0) ts[rep - 1] = t;
    }
    if (rc != RID_OK) break;
    std::sort(ts, ts + 3);
    if (ms_out) ms_out[i] = ts[1];
    if (best < 0.0f || ts[1] < best) {
      best = ts[1];
      best_g = cand[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != RID_OK) {
    set_batched_grid(cfg, b, max_n, saved);
    return rc;
  }
  for (int i = ncand; ms_out && i < kGridCandidates; ++i) ms_out[i] = -1.0f;
  set_batched_grid(cfg, b, max_n, best_g == G ? 0 : best_g);
  if (grid_out) *grid_out = best_g;
  return RID_OK;
}

int rid_rank_features(int32_t nblk, const void* const* A, const int64_t* lda, const int32_t* m,
                      const int32_t* n, double tol, const rid_config* cfg, float* features,
                      hipStream_t stream) {
  if (nblk < 0 || !cfg || (cfg->dtype != RID_F64 && cfg->dtype != RID_F32) || !(tol >= 0.0))
    return RID_ERR_ARG;
  if (nblk == 0) return RID_OK;
  if (!A || !lda || !m || !n || !features) return RID_ERR_ARG;
  if (cfg->dtype == RID_F64)
    hipLaunchKernelGGL(k_rank_features<double>, dim3((unsigned)nblk), dim3(256), 0, stream, nblk,
                       A, lda, m, n, tol, cfg->tol_relative, cfg->seed, features);
  else
    hipLaunchKernelGGL(k_rank_features<float>, dim3((unsigned)nblk), dim3(256), 0, stream, nblk,
                       A, lda, m, n, tol, cfg->tol_relative, cfg->seed, features);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int32_t rid_mlp_param_count(void) { return rid::kNParams; }

static int mlp_groups(int32_t B) {
  const int tiles = (B + rid::kMlpTile - 1) / rid::kMlpTile;
  return tiles < 256 ? tiles : 256;
}

size_t rid_mlp_workspace_bytes(int32_t B) {
  if (B < 1) return 0;
  const size_t G = (size_t)mlp_groups(B);
  return align_up(G * rid::kNParams * sizeof(float), kAlign) + G * sizeof(double);
}

int rid_mlp_forward(int32_t B, const float* X, const float* xnorm, const float* params, float* y,
                    float* z1, float* z2, hipStream_t stream) {
  if (B < 0 || (B > 0 && (!X || !params || !y))) return RID_ERR_ARG;
  if (B == 0) return RID_OK;
  const unsigned g = (unsigned)((B + rid::kMlpTile - 1) / rid::kMlpTile);
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(rid::kHid), 0, stream, B, X, xnorm, params, y,
                     z1, z2);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_mlp_backward(int32_t B, const float* X, const float* xnorm, const float* z1,
                     const float* z2, const float* y, const float* target, float q,
                     const float* params, float* grad, double* loss, void* work,
                     size_t work_bytes, hipStream_t stream) {
  if (B < 1 || !X || !z1 || !z2 || !y || !target || !params || !grad || !work ||
      !(q > 0.f && q < 1.f))
    return RID_ERR_ARG;
  if (work_bytes < rid_mlp_workspace_bytes(B)) return RID_ERR_WORKSPACE;
  const int G = mlp_groups(B);
  float* part = static_cast<float*>(work);
  double* lpart = reinterpret_cast<double*>(static_cast<char*>(work) +
                                            align_up((size_t)G * rid::kNParams * sizeof(float), kAlign));
  hipLaunchKernelGGL(k_mlp_backward, dim3((unsigned)G), dim3(rid::kHid), 0, stream, B, X, xnorm,
                     z1, z2, y, target, q, params, part, lpart);
  RID_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)ceil_div(rid::kNParams, 256)), dim3(256), 0,
                     stream, G, part, lpart, grad, loss);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_mlp_adamw(float* params, const float* grad, float* m1, float* m2, int32_t step, float lr,
                  float beta1, float beta2, float eps, float weight_decay, hipStream_t stream) {
  if (!params || !grad || !m1 || !m2 || step < 1) return RID_ERR_ARG;
  hipLaunchKernelGGL(k_mlp_adamw, dim3((unsigned)ceil_div(rid::kNParams, 256)), dim3(256), 0,
                     stream, params, grad, m1, m2, step, lr, beta1, beta2, eps, weight_decay);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_rank_hint(int32_t B, const float* y, float margin, const int32_t* kcap, int32_t* k_hint,
                  hipStream_t stream) {
  if (B < 0 || (B > 0 && (!y || !kcap || !k_hint))) return RID_ERR_ARG;
  if (B == 0) return RID_OK;
  hipLaunchKernelGGL(k_rank_hint, dim3((unsigned)ceil_div(B, 256)), dim3(256), 0, stream, B, y,
                     margin, kcap, k_hint);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_debug_mfma_probe(int kind, const void* A, const void* B, float* D, hipStream_t stream) {
  if (kind < 0 || kind > 3 || !A || !B || !D) return RID_ERR_ARG;
  hipLaunchKernelGGL(k_mfma_probe, dim3(1), dim3(64), 0, stream, kind,
                     static_cast<const unsigned char*>(A), static_cast<const unsigned char*>(B), D);
  RID_LAUNCH_CHECK();
  return RID_OK;
}

int rid_profile_start(void) {
  Profiler& p = prof();
  p.on = true;
  p.used = 0;
  p.marks.clear();
  return RID_OK;
}

int rid_profile_stop(double* ms, int64_t* launches, int nclass) {
  Profiler& p = prof();
  p.on = false;
  if (!ms || !launches || nclass < 1) return RID_ERR_ARG;
  for (int c = 0; c < nclass; ++c) {
    ms[c] = 0.0;
    launches[c] = 0;
  }
  for (auto& mk : p.marks) {
    if (hipEventSynchronize(p.pool[mk.second + 1]) != hipSuccess) return RID_ERR_HIP;
    float t = 0.f;
    if (hipEventElapsedTime(&t, p.pool[mk.second], p.pool[mk.second + 1]) != hipSuccess)
      return RID_ERR_HIP;
    if (mk.first < nclass) {
      ms[mk.first] += t;
      launches[mk.first] += 1;
    }
  }
  p.marks.clear();
  p.used = 0;
  return RID_OK;
}

int rid_release(void) {
  int dev0 = 0;
  if (hipGetDevice(&dev0) != hipSuccess) return RID_ERR_HIP;
  int rc = RID_OK;
  {
    std::lock_guard<std::mutex> lk(side_mu);
    for (SideSet& e : side_pool) {
      if (e.dev < 0) continue;
      if (e.busy) {  // a call still holds this set
        rc = RID_ERR_ARG;
        continue;
      }
      if (hipSetDevice(e.dev) != hipSuccess) {
        rc = RID_ERR_HIP;
        continue;
      }
      if (hipStreamSynchronize(e.s) != hipSuccess || hipEventDestroy(e.fork) != hipSuccess ||
          hipEventDestroy(e.join) != hipSuccess || hipStreamDestroy(e.s) != hipSuccess)
        rc = RID_ERR_HIP;
      e = SideSet{};
    }
  }
  Profiler& p = prof();
  p.on = false;
  for (hipEvent_t ev : p.pool)
    if (hipEventDestroy(ev) != hipSuccess) rc = RID_ERR_HIP;
  p.pool.clear();
  p.marks.clear();
  p.used = 0;
  if (hipSetDevice(dev0) != hipSuccess) rc = RID_ERR_HIP;
  return rc;
}

}  // extern "C"
