// lk_runtime.hip -- the C ABI of liblk.so (include/lk.h): contexts, workspace,
// argument checking, the kernel sequence of each call and its HIP-graph cache,
// the autotuner, and the pass loop of lk_discretize.
//
// lk_direct_sum enqueues, on the caller's stream:
//   preparation (xi partials, per-loop validity) -> plan (items per pair) ->
//   schedule (LPT order, scan) -> persistent direct-sum kernel, which also
//   rounds, flags and queues refits for pairs of one work item -> the same for
//   pairs split over several items
//   [MIXED only: plan -> schedule -> FP64 direct-sum -> split pairs, on the
//   refit list]
// CROSSINGS replaces the FP32 direct sum by the crossing count (with its FP64
// count and the FP64 direct sum for undecided pairs); BARNES_HUT by the trees,
// the breadth-first traversal (twice with the adaptive beta) and the leaf
// pairs.  Every launch has a host-known shape; data-dependent counts live in
// device memory.  The first call with a given argument set is captured into a
// HIP graph (when the stream allows capture) and replayed by later identical
// calls.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <fstream>
#include <map>
#include <sstream>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lk.h"
#include "lk_internal.h"
#include "lk_dz.h"

namespace {

// Device buffer that only grows; growing invalidates captured graphs.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

using GraphKey = std::tuple<const void*, int, const void*, int32_t, const void*, int64_t, int,
                            void*, void*, void*, int, int, int, int, int64_t, const void*, void*,
                            int>;

}  // namespace

struct lk_ctx {
  int device = 0;
  int n_cu = 0;
  std::string err;
  // options
  double refit_thr = 0.05;
  bool use_graph = true;
  bool timing = false;
  int opt_tile = 0, opt_chunk = 0, opt_waves = 0, opt_atan = 0, opt_segs = 0, opt_segs64 = 0;
  int opt_batch = 0;
  // crossing count: view direction (largest component magnitude 1) and the
  // multiplier of its certainty bounds
  float view[3] = {0.0f, 0.0f, 0.0f};
  int cc_tol = 1;
  bool cc_cull = true;
  // vertex count of the last offsets array seen in CROSSINGS mode (sizes the
  // culling boxes; read from the device once per offsets pointer and length)
  const void* cc_off_key = nullptr;
  int32_t cc_loops_key = -1;
  int64_t cc_vertices = 0;
  // workspace
  DevBuf loop_flags, minseg2, xi, recs, big_prefix, meta, acc, flags, refit_list;
  DevBuf boxes, vcounts, vprefix;
  DevBuf cc_blk, cc_sup;  // crossing count: projected block and superblock boxes
  DevBuf bh_nodes, bh_lists, bh_counts;  // Barnes-Hut trees, node-pair lists, counts
  DevBuf bh_adapt;  // adaptive beta: per-pair error estimate (fixed point) and beta
  DevBuf pls_grid;  // grid pair search: parameters, cell counts and starts, bins
  int pair_search = 0;  // 0 auto, 1 all pairs, 2 grid
  // discretization: two piece arrays and two unprocessed lists (swapped every
  // pass), piece and group boxes, marks, split prefixes, per-pair item
  // prefixes, scan partials, and the small per-loop arrays
  DevBuf dz_piece[2], dz_list[2], dz_pbox, dz_gbox, dz_mark, dz_pre, dz_pair_pre, dz_pair_ab,
      dz_part, dz_loops;
  int dz_max_passes = 64;
  double bh_beta = 4.0;
  int bh_order = 2;
  bool bh_adaptive = false;      // Sec. 3.4.4's second evaluation at a larger beta
  double bh_beta_max = 10.0;
  double bh_target = 0.2;
  uint64_t ws_epoch = 0;  // bumped whenever a workspace buffer moves
  // completion of the context's last enqueued work (calls on one context do
  // not overlap, so it covers every earlier call): a buffer that grows waits
  // for it instead of for the whole device
  hipEvent_t done = nullptr;
  bool done_pending = false;
  // graphs
  struct Cached {
    hipGraphExec_t exec = nullptr;
    uint64_t epoch = 0;
  };
  std::map<GraphKey, Cached> graphs;
  // timing: a ring of event quadruples (main start/stop, refit start/stop),
  // one per timed call, so a run of calls can be averaged without syncing
  std::vector<hipEvent_t> ring;
  int ring_pos = 0, ring_count = 0;
  lk_stats stats;
  hipStream_t last_stream = nullptr;
  bool last_mixed = false;
  bool last_crossings = false;
  bool last_bh = false;
  int64_t last_bh_list_cap = 0;
  bool last_timed = false;

  lk_status fail(lk_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    err = buf;
    return st;
  }
};

#define LK_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ctx->fail(LK_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));       \
  } while (0)

namespace {

lk_status ensure(lk_ctx* ctx, DevBuf& b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return LK_OK;
  size_t want = bytes + bytes / 4;
  if (b.p) {
    // the buffer may be referenced by this context's work still in flight
    if (ctx->done_pending) {
      if (hipEventSynchronize(ctx->done) != hipSuccess)
        return ctx->fail(LK_EDEVICE, "sync before realloc");
      ctx->done_pending = false;
    }
    (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (hipMalloc(&b.p, want) != hipSuccess) {
    b.p = nullptr;
    return ctx->fail(LK_ENOMEM, "hipMalloc(%zu) failed", want);
  }

  b.bytes = want;
  ctx->ws_epoch++;
  return LK_OK;
}

// Mark the end of the work just enqueued on `s` (not while `s` is being
// captured: that work runs when the caller launches its graph).
void mark_done(lk_ctx* ctx, hipStream_t s) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (s && hipStreamIsCapturing(s, &cs) != hipSuccess) return;
  if (cs != hipStreamCaptureStatusNone || !ctx->done) return;
  if (hipEventRecord(ctx->done, s) == hipSuccess) ctx->done_pending = true;
}

int default_tile(bool f64) { return f64 ? 256 : 512; }
int default_chunk(bool f64) { return f64 ? 2048 : 4096; }

struct Plan {
  bool in_f64;
  bool mixed;      // FP32 main pass + FP64 refit (MIXED, CROSSINGS, BARNES_HUT)
  bool crossings;  // main pass counts crossings
  bool bh;         // main pass is the Barnes-Hut traversal
  int tile, chunk, grid, grid64, grid_refit, atan_form;
  int segs, segs64;  // segments of loop B per lane, FP32 and FP64 kernels
  int grid_cc64;     // CROSSINGS: grid of the FP64 crossing count
  bool unpacked;     // few pairs: every small pair on a whole wave
};

constexpr int kDefaultSegs32 = 4;
constexpr int kDefaultSegs64 = 2;
constexpr int kDefaultBatch = 4;
constexpr int kFormCrossings = 3;  // term form of the crossing-count kernel
// Certainty factors of the crossing count in units of 2^-24 (twice the
// first-order error bounds of the side predicates and of the crossing sign).
constexpr double kCcTau = 128.0 / 16777216.0, kCcTauP = 512.0 / 16777216.0;
constexpr double kCcTau64 = kCcTau / 536870912.0, kCcTauP64 = kCcTauP / 536870912.0;  // 2^-29

// Small device-side counters of one call, in one buffer (byte offsets).
constexpr size_t kMetaCountsMain = 0;    // int32[2]: n_small, n_big (main pass)
constexpr size_t kMetaCountsRefit = 8;   // int32[2]: n_small, n_big (refit pass)
constexpr size_t kMetaRefitN = 16;       // int32: pairs queued for refit (follows the above)
constexpr size_t kMetaBigTotalMain = 24; // int64
constexpr size_t kMetaBigTotalRefit = 32;
constexpr size_t kMetaCounterMain = 40;  // uint64 work counters
constexpr size_t kMetaCounterRefit = 48;
constexpr size_t kMetaStop = 56;         // int32: fused check's stop flag
// CROSSINGS: the FP64 crossing count refits first and queues what it cannot
// decide for the FP64 direct sum (a second refit pass)
constexpr size_t kMetaCountsRefit2 = 64; // int32[2]
constexpr size_t kMetaRefitN2 = 72;      // int32 (follows the above)
constexpr size_t kMetaBigTotalRefit2 = 80;
constexpr size_t kMetaCounterRefit2 = 88;
constexpr size_t kMetaOffsetsBad = 96;  // int32: offsets that decrease (set by a check)
constexpr size_t kMetaBytes = 104;

// Fused certificate check of a call (lk_direct_sum_check); empty for
// lk_direct_sum.
struct Check {
  const int32_t* expected = nullptr;
  int early_exit = 0;
  int64_t* n_mismatch = nullptr;
};

template <typename T>
T* meta_at(lk_ctx* ctx, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ctx->meta.p) + off);
}

// Device workspace of one direct-sum call in the PLAIN_F64 and MIXED modes:
// the context's buffers, or a carve of the no-allocation entry point's static
// array.  (CROSSINGS and BARNES_HUT also use the context's boxes and trees.)
struct Ws {
  uint32_t* loop_flags;     // [L]
  double* minseg2;          // [L]
  double* xi;               // [kPrepMaxBlocks + 1]
  lk::WorkRec* recs;        // [3 P]
  int64_t* big_prefix;      // [P + 1]
  char* meta;               // [kMetaBytes]
  unsigned long long* acc;  // [2 P]
  int32_t* refit_list;      // [2 P]
  template <typename T>
  T* at(size_t off) const {
    return reinterpret_cast<T*>(meta + off);
  }
};

Ws ctx_ws(lk_ctx* ctx) {
  Ws w;
  w.loop_flags = (uint32_t*)ctx->loop_flags.p;
  w.minseg2 = (double*)ctx->minseg2.p;
  w.xi = (double*)ctx->xi.p;
  w.recs = (lk::WorkRec*)ctx->recs.p;
  w.big_prefix = (int64_t*)ctx->big_prefix.p;
  w.meta = (char*)ctx->meta.p;
  w.acc = (unsigned long long*)ctx->acc.p;
  w.refit_list = (int32_t*)ctx->refit_list.p;
  return w;
}

// pass: 0 main, 1 refit, 2 second refit (CROSSINGS)
lk::Sched make_sched(const Ws& W, int64_t n_pairs, int pass) {
  lk::Sched S;
  lk::WorkRec* recs = W.recs;
  S.small = recs;
  S.big_in = recs + n_pairs;
  S.big = recs + 2 * n_pairs;
  S.big_prefix = W.big_prefix;
  const size_t counts[3] = {kMetaCountsMain, kMetaCountsRefit, kMetaCountsRefit2};
  const size_t totals[3] = {kMetaBigTotalMain, kMetaBigTotalRefit, kMetaBigTotalRefit2};
  const size_t counters[3] = {kMetaCounterMain, kMetaCounterRefit, kMetaCounterRefit2};
  S.counts = W.at<int32_t>(counts[pass]);
  S.big_total = W.at<int64_t>(totals[pass]);
  S.counter = W.at<unsigned long long>(counters[pass]);
  return S;
}

// Two directions spanning the plane orthogonal to the view direction.
lk::CcProj cc_projection(const float* view) {
  double n[3] = {view[0], view[1], view[2]};
  const double nn = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  for (double& c : n) c /= nn;
  // the coordinate axis least aligned with n
  int ax = 0;
  for (int q = 1; q < 3; ++q)
    if (std::fabs(n[q]) < std::fabs(n[ax])) ax = q;
  double a[3] = {0.0, 0.0, 0.0};
  a[ax] = 1.0;
  double e1[3] = {n[1] * a[2] - n[2] * a[1], n[2] * a[0] - n[0] * a[2], n[0] * a[1] - n[1] * a[0]};
  const double l1 = std::sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
  for (double& c : e1) c /= l1;
  const double e2[3] = {n[1] * e1[2] - n[2] * e1[1], n[2] * e1[0] - n[0] * e1[2],
                        n[0] * e1[1] - n[1] * e1[0]};
  lk::CcProj P;
  for (int q = 0; q < 3; ++q) {
    P.e1[q] = (float)e1[q];
    P.e2[q] = (float)e2[q];
  }
  return P;
}

// Barnes-Hut: tree levels, node slots and list capacities for the call's
// vertex count (read as for the crossing count).  The trees need levels up
// to the one whose node spans the longest possible loop (the vertex count).
struct BhLayout {
  int levels = 1;
  int64_t base[lk::kBhMaxLevels] = {}, cap[lk::kBhMaxLevels] = {};
  int64_t nodes = 0, list_cap = 0, near_cap = 0;
};

BhLayout bh_layout(int64_t v, int32_t n_loops, int64_t n_pairs) {
  BhLayout Y;
  int64_t span = lk::kBhLeaf;
  while (span < v && Y.levels < lk::kBhMaxLevels) {
    span *= lk::kBhArity;
    ++Y.levels;
  }
  span = lk::kBhLeaf;
  for (int h = 0; h < Y.levels; ++h) {
    Y.base[h] = Y.nodes;
    Y.cap[h] = v / span + n_loops + 1;
    Y.nodes += Y.cap[h];
    span *= lk::kBhArity;
  }
  // generous (measured: a step of the long-loop and knit workloads holds up
  // to 2 and 12 node pairs per leaf, the leaf list up to 330 per leaf of the
  // knit workload at beta 8); a pair whose entries do not fit is refitted,
  // not lost
  const int64_t leaves = v / lk::kBhLeaf + n_loops;
  Y.list_cap = 32 * leaves + 8 * n_pairs + 65536;
  Y.near_cap = 512 * leaves + 4 * n_pairs + 65536;
  return Y;
}

// Enqueue the whole direct-sum sequence (no graph logic here).
lk_status enqueue_direct_sum(lk_ctx* ctx, const Ws& W, const Plan& P, const void* xyz,
                             const int64_t* off, int32_t n_loops, const int32_t* pairs,
                             int64_t n_pairs, double* lk_real, int32_t* lk_int, uint32_t* flags,
                             hipStream_t s, hipEvent_t* ev /* 4 events or NULL */,
                             const Check& ck = Check()) {
  const bool timed = ev != nullptr;
  using namespace lk;
  uint32_t* lf = W.loop_flags;
  double* xi = W.xi;  // [kPrepMaxBlocks] partial sums of |coordinate|
  int32_t* rlist = W.refit_list;
  int32_t* rn = W.at<int32_t>(kMetaRefitN);
  unsigned long long* acc = W.acc;

  LoopInfo li;
  li.lf = lf;
  li.minseg2 = W.minseg2;
  li.part = xi;
  // the vertex count is known (and the boxes sized for it) only in CROSSINGS
  const bool cull = P.crossings && ctx->cc_cull;
  li.n_part = prep_blocks(n_loops, (cull || P.bh) && ctx->cc_off_key == off &&
                                           ctx->cc_loops_key == n_loops
                                       ? ctx->cc_vertices
                                       : 0);
  li.eps = P.in_f64 ? 2.220446049250313080847e-16 : 1.1920928955078125e-07;

  Outs out{};
  out.lk_real = lk_real;
  out.lk_int = lk_int;
  out.flags = flags;
  out.refit_list = P.mixed ? rlist : nullptr;
  out.refit_n = P.mixed ? rn : nullptr;
  out.thr = ctx->refit_thr;
  out.refit_pass = 0;
  out.expected = ck.expected;
  out.n_mismatch = ck.expected ? (unsigned long long*)ck.n_mismatch : nullptr;
  out.stop = ck.expected ? W.at<int32_t>(kMetaStop) : nullptr;
  out.early_exit = ck.expected ? ck.early_exit : 0;

  PlanArgs M{};
  M.off = off;
  M.pairs = pairs;
  M.list = nullptr;
  M.n_list_dev = nullptr;
  M.n_list = n_pairs;
  M.acc = acc;
  M.chunk = P.chunk;
  M.bblock = lk::kWave * (P.mixed ? P.segs : P.segs64);
  M.cc_sup = cull ? (const float4*)ctx->cc_sup.p : nullptr;
  M.cc_nsup = cull ? (int64_t)(ctx->cc_sup.bytes / 16) : 0;
  M.out = out;
  DsArgs A{};
  A.xyz = xyz;
  A.s = make_sched(W, n_pairs, 0);
  A.acc = acc;
  A.tile = P.tile;
  A.chunk = P.chunk;
  A.batch = ctx->opt_batch ? ctx->opt_batch : kDefaultBatch;
  // R small pairs share a wave in the FP32 kernel: a batch below R idles lanes
  if (P.mixed && A.batch < P.segs) A.batch = P.segs;
  // A call with few pairs is latency-bound: unpacked, one pair per work
  // item; up to R pairs per persistent wave, one packed round per item.
  // Either way the pairs spread over the most waves.  (The batch only groups
  // pairs; a pair's lane layout, and so its value, does not depend on it.)
  if (P.unpacked) {
    A.batch = 1;
  } else {
    const int waves = P.mixed ? P.grid : P.grid64;
    const int r = P.mixed ? P.segs : P.segs64;
    if (n_pairs <= (int64_t)waves * r && A.batch > r) A.batch = r;
  }
  A.view[0] = ctx->view[0];
  A.view[1] = ctx->view[1];
  A.view[2] = ctx->view[2];
  A.cc_tau = (float)(kCcTau * ctx->cc_tol);
  A.cc_tau_p = (float)(kCcTauP * ctx->cc_tol);
  A.cc_blk = cull ? (const float4*)ctx->cc_blk.p : nullptr;
  A.cc_sup = cull ? (const float4*)ctx->cc_sup.p : nullptr;
  A.cc_nblk = cull ? (int64_t)(ctx->cc_blk.bytes / 16) : 0;
  A.cc_nsup = cull ? (int64_t)(ctx->cc_sup.bytes / 16) : 0;
  A.pairs = pairs;
  A.off = off;
  A.out = out;

  // the crossing count's box kernel and the Barnes-Hut leaf kernel validate
  // the loops in parallel; the preparation kernel then only initialises.  A
  // direct sum with few pairs prepares, plans and schedules in one launch.
  const bool one_launch_start = P.unpacked && !cull && !P.bh;
  if (!one_launch_start)
    LK_HIP(launch_prep(xyz, P.in_f64, off, n_loops, xi, lf, W.minseg2, A.s.counts,
                       out.n_mismatch, out.stop, !cull && !P.bh, li.n_part, s));
  if (cull)
    LK_HIP(launch_cc_boxes(xyz, P.in_f64, off, n_loops, cc_projection(ctx->view),
                           (float4*)ctx->cc_blk.p, A.cc_nblk, (float4*)ctx->cc_sup.p, A.cc_nsup,
                           lf, W.minseg2, s));
  if (P.bh) {
    // Barnes-Hut: the plan validates, flags and zeroes (every pair one item);
    // the trees, the breadth-first traversal and the leaf pairs replace the
    // direct-sum kernel
    PlanArgs Mb = M;
    Mb.chunk = 1 << 24;
    Mb.bblock = 1 << 30;
    const int64_t v = ctx->cc_off_key == off && ctx->cc_loops_key == n_loops ? ctx->cc_vertices : 0;
    const BhLayout Y = bh_layout(v, n_loops, n_pairs);
    BhArgs H{};
    H.xyz = xyz;
    H.off = off;
    H.pairs = pairs;
    H.n_loops = n_loops;
    H.nodes = (BhNode*)ctx->bh_nodes.p;
    const int64_t node_room = (int64_t)(ctx->bh_nodes.bytes / sizeof(BhNode));
    for (int h = 0; h < kBhMaxLevels; ++h) {
      H.level_base[h] = h < Y.levels ? Y.base[h] : 0;
      // a level that does not fit the buffer (a capture before the vertex
      // count was read) gets no slots: its pairs fail and are refitted
      H.level_cap[h] = h < Y.levels && Y.base[h] + Y.cap[h] <= node_room ? Y.cap[h] : 0;
    }
    H.levels = Y.levels;
    BhPair* lists = (BhPair*)ctx->bh_lists.p;
    const int64_t room = (int64_t)(ctx->bh_lists.bytes / sizeof(BhPair));
    const bool fits = 2 * Y.list_cap + Y.near_cap <= room;
    H.list[0] = lists;
    H.list[1] = lists + (fits ? Y.list_cap : 0);
    H.near = lists + (fits ? 2 * Y.list_cap : 0);
    H.list_cap = fits ? Y.list_cap : 0;
    ctx->last_bh_list_cap = H.list_cap;
    H.near_cap = fits ? Y.near_cap : 0;
    H.counts = (int32_t*)ctx->bh_counts.p;
    H.acc = acc;
    H.lf = lf;
    H.minseg2 = W.minseg2;
    H.beta = ctx->bh_beta;
    H.order = ctx->bh_order;
    H.out = out;
    const bool adaptive = ctx->bh_adaptive && ctx->bh_adapt.bytes >= 24 * (size_t)n_pairs;
    if (adaptive) H.est = (unsigned long long*)ctx->bh_adapt.p;
    if (timed) LK_HIP(hipEventRecord(ev[0], s));
    // the leaf kernel also validates the loops, so the plan follows it
    LK_HIP(launch_bh_leaves(H, P.in_f64, s));
    for (int h = 1; h < Y.levels; ++h) LK_HIP(launch_bh_level(H, h, s));
    LK_HIP(launch_plan(Mb, n_loops, li, A.s, false, s));
    LK_HIP(launch_sched(A.s, W.at<int32_t>(kMetaCountsRefit), s));
    LK_HIP(launch_bh_roots(H, n_pairs, s));
    for (int it = 0; it < 2 * (Y.levels - 1) + 1; ++it) LK_HIP(launch_bh_expand(H, it, s));
    LK_HIP(launch_bh_near(H, P.in_f64, s));
    if (adaptive) {
      // pairs whose error estimate asks for a larger beta are evaluated again
      // from their roots at that beta (their first values are discarded)
      H.beta_p = (double*)((char*)ctx->bh_adapt.p + 16 * (size_t)n_pairs);
      LK_HIP(launch_bh_adapt(H, n_pairs, ctx->bh_target, ctx->bh_beta_max, s));
      H.est = nullptr;
      LK_HIP(launch_bh_roots(H, n_pairs, s));
      for (int it = 0; it < 2 * (Y.levels - 1) + 1; ++it) LK_HIP(launch_bh_expand(H, it, s));
      LK_HIP(launch_bh_near(H, P.in_f64, s));
    }
    if (timed) LK_HIP(hipEventRecord(ev[1], s));
    LK_HIP(launch_bh_finalize(H, n_pairs, s));
  } else {
    if (one_launch_start) {
      LK_HIP(launch_prep_plan(xyz, P.in_f64, M, n_loops, li, lf, W.minseg2, A.s, out.n_mismatch,
                              out.stop, W.at<int32_t>(kMetaCountsRefit), s));
    } else {
      LK_HIP(launch_plan(M, n_loops, li, A.s, false, s));
      LK_HIP(launch_sched(A.s, W.at<int32_t>(kMetaCountsRefit), s));
    }
    if (timed) LK_HIP(hipEventRecord(ev[0], s));
    LK_HIP(launch_direct_sum(A, P.in_f64, !P.mixed, P.atan_form, P.mixed ? P.segs : P.segs64,
                             P.mixed ? P.grid : P.grid64, s, P.unpacked));
    if (timed) LK_HIP(hipEventRecord(ev[1], s));
    // a mixed call finalises its split pairs in the launch that plans the
    // refit pass (below)
    if (!P.mixed) LK_HIP(launch_finalize_split(A.s, acc, out, n_pairs, s));
  }
  if (P.mixed) {
    // refit: the FP64 direct sum (MIXED), or the FP64 crossing count
    // (CROSSINGS), which queues what it cannot decide for the FP64 direct sum
    int32_t* rlist2 = rlist + n_pairs;
    int32_t* rn2 = W.at<int32_t>(kMetaRefitN2);
    Outs ro = out;
    ro.refit_list = P.crossings ? rlist2 : nullptr;
    ro.refit_n = P.crossings ? rn2 : nullptr;
    ro.refit_pass = 1;
    PlanArgs R = M;
    R.list = rlist;
    R.n_list_dev = rn;
    R.chunk = P.crossings ? P.chunk : default_chunk(true);
    R.bblock = lk::kWave * P.segs64;
    R.cc_sup = nullptr;
    R.out = ro;
    DsArgs B = A;
    if (!P.crossings) B.cc_blk = B.cc_sup = nullptr;
    B.cc_tau = (float)(kCcTau64 * ctx->cc_tol);
    B.cc_tau_p = (float)(kCcTauP64 * ctx->cc_tol);
    B.s = make_sched(W, n_pairs, 1);
    B.tile = default_tile(true);
    B.chunk = R.chunk;
    // refits are few and latency-bound: one pair per work index spreads them
    // over the most waves
    B.batch = 1;
    B.out = ro;
    int32_t* zero_next = P.crossings ? W.at<int32_t>(kMetaCountsRefit2) : nullptr;
    if (P.bh) {
      // the Barnes-Hut pass finalised its pairs itself
      LK_HIP(launch_plan(R, n_loops, li, B.s, true, s));
      LK_HIP(launch_sched(B.s, zero_next, s));
    } else {
      LK_HIP(launch_finalize_replan(A.s, acc, out, R, n_loops, li, B.s, zero_next, s));
    }
    if (timed) LK_HIP(hipEventRecord(ev[2], s));
    // the FP64 crossing count gets the whole grid: its pairs are the ones
    // with shallow crossings, often the largest
    LK_HIP(launch_direct_sum(B, P.in_f64, true, P.crossings ? kFormCrossings : 0, P.segs64,
                             P.crossings ? P.grid_cc64 : P.grid_refit, s, P.unpacked));
    if (timed) LK_HIP(hipEventRecord(ev[3], s));
    if (!P.crossings) LK_HIP(launch_finalize_split(B.s, acc, ro, n_pairs, s));
    if (P.crossings) {
      Outs r2 = out;
      r2.refit_list = nullptr;
      r2.refit_n = nullptr;
      r2.refit_pass = 1;
      PlanArgs R2 = R;
      R2.list = rlist2;
      R2.n_list_dev = rn2;
      R2.chunk = default_chunk(true);
      R2.out = r2;
      DsArgs B2 = B;
      B2.cc_blk = B2.cc_sup = nullptr;
      B2.s = make_sched(W, n_pairs, 2);
      B2.chunk = R2.chunk;
      B2.out = r2;
      // the FP64 crossing count's split pairs are finalised (queuing what it
      // cannot decide) in the launch that plans the direct sum of those
      LK_HIP(launch_finalize_replan(B.s, acc, ro, R2, n_loops, li, B2.s, nullptr, s));
      LK_HIP(launch_direct_sum(B2, P.in_f64, true, 0, P.segs64, P.grid_refit, s, P.unpacked));
      LK_HIP(launch_finalize_split(B2.s, acc, r2, n_pairs, s));
    }
  }
  return LK_OK;
}

// Kernel configuration of a call from the context's options (0 = default).
// Up to two pairs per compute unit a call is latency-bound: every small pair
// then gets a whole wave (64 lanes, so each walks a quarter or less of loop
// A) instead of sharing one with R - 1 others.  The choice depends only on
// the pair count and the device, and both passes of a call make it, so a
// pair's lane layout, and with it its value, is the same in the plain mode
// and in a refit.
bool few_pairs(const lk_ctx* ctx, int64_t n_pairs) { return n_pairs <= 2 * (int64_t)ctx->n_cu; }

Plan make_plan(lk_ctx* ctx, bool in_f64, int mode, int64_t n_pairs) {
  const bool mixed = mode != LK_PLAIN_F64;
  Plan P;
  P.unpacked = few_pairs(ctx, n_pairs);
  P.in_f64 = in_f64;
  P.mixed = mixed;
  P.crossings = mode == LK_CROSSINGS;
  P.bh = mode == LK_BARNES_HUT;
  P.atan_form = P.crossings ? kFormCrossings : ctx->opt_atan;
  const int tmax = mixed ? lk::kMaxTileF32 : lk::kMaxTileF64;
  P.tile = ctx->opt_tile ? (ctx->opt_tile < tmax ? ctx->opt_tile : tmax) : default_tile(!mixed);
  P.chunk = ctx->opt_chunk ? ctx->opt_chunk : default_chunk(!mixed);
  if (P.chunk % P.tile) P.chunk = ((P.chunk + P.tile - 1) / P.tile) * P.tile;
  P.segs = lk::segs_supported(false, ctx->opt_segs ? ctx->opt_segs : kDefaultSegs32, P.crossings);
  P.segs64 = lk::segs_supported(true, ctx->opt_segs64 ? ctx->opt_segs64 : kDefaultSegs64);
  P.grid = lk::direct_sum_grid(in_f64, false, P.atan_form, P.segs, P.tile, ctx->n_cu,
                               ctx->opt_waves, P.unpacked);
  P.grid64 = lk::direct_sum_grid(in_f64, true, 0, P.segs64, mixed ? default_tile(true) : P.tile,
                                 ctx->n_cu, ctx->opt_waves, P.unpacked);
  // refits of the direct sum are rare: one wave per CU keeps the empty refit
  // pass cheap (4.7 instead of 7.8 us on chainmail).  Barnes-Hut sends every
  // pair whose far-field error estimate stays too large there (hundreds of
  // big pairs on knit with adaptive beta), so its refit pass gets the whole
  // grid.
  P.grid_refit = P.bh || ctx->n_cu >= P.grid64 ? P.grid64 : ctx->n_cu;
  P.grid_cc64 = P.crossings ? lk::direct_sum_grid(in_f64, true, kFormCrossings, P.segs64,
                                                  default_tile(true), ctx->n_cu, 0)
                            : 0;
  return P;
}

lk_status ensure_workspace(lk_ctx* ctx, int32_t n_loops, int64_t n_pairs) {
  lk_status st;
  if ((st = ensure(ctx, ctx->loop_flags, 4 * (size_t)n_loops)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->minseg2, 8 * (size_t)n_loops)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->xi, 8 * (size_t)(lk::kPrepMaxBlocks + 1))) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->recs, 3 * sizeof(lk::WorkRec) * (size_t)n_pairs)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->big_prefix, 8 * (size_t)(n_pairs + 1))) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->meta, kMetaBytes)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->acc, 16 * (size_t)n_pairs)) != LK_OK) return st;
  // two refit lists: the second is the CROSSINGS mode's FP64 direct-sum pass
  if ((st = ensure(ctx, ctx->refit_list, 8 * (size_t)n_pairs)) != LK_OK) return st;
  return LK_OK;
}

// Crossing count: size the culling boxes for the call's vertex count, which
// is read from the device (one synchronisation) the first time an offsets
// array is seen.  Inside a stream capture nothing is read and the boxes keep
// their size; the kernels never cull through a slot beyond it.
lk_status read_vertices(lk_ctx* ctx, const int64_t* off, int32_t n_loops, hipStream_t s,
                        bool can_sync, int64_t* v) {
  if (can_sync && (ctx->cc_off_key != off || ctx->cc_loops_key != n_loops)) {
    // the block and node slots are computed from the offsets, so offsets that
    // decrease are rejected here, in the same synchronisation
    int64_t ends[2] = {0, 0};
    int32_t bad = 0;
    int32_t* bad_d = meta_at<int32_t>(ctx, kMetaOffsetsBad);
    LK_HIP(hipMemsetAsync(bad_d, 0, 4, s));
    LK_HIP(lk::launch_dz_check(off, n_loops, bad_d, s));
    LK_HIP(hipMemcpyAsync(&bad, bad_d, 4, hipMemcpyDeviceToHost, s));
    LK_HIP(hipMemcpyAsync(&ends[0], off, 8, hipMemcpyDeviceToHost, s));
    LK_HIP(hipMemcpyAsync(&ends[1], off + n_loops, 8, hipMemcpyDeviceToHost, s));
    LK_HIP(hipStreamSynchronize(s));
    if (bad) return ctx->fail(LK_EINVAL, "loop offsets decrease");
    ctx->cc_off_key = off;
    ctx->cc_loops_key = n_loops;
    ctx->cc_vertices = ends[1] - ends[0] > 0 ? ends[1] - ends[0] : 0;
  }
  *v = ctx->cc_off_key == off && ctx->cc_loops_key == n_loops ? ctx->cc_vertices : 0;
  return LK_OK;
}

lk_status cc_prepare(lk_ctx* ctx, const int64_t* off, int32_t n_loops, hipStream_t s,
                     bool can_sync) {
  int64_t v = 0;
  lk_status st;
  if ((st = read_vertices(ctx, off, n_loops, s, can_sync, &v)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->cc_blk, 16 * (size_t)(v / lk::kCcBlock + n_loops + 1))) != LK_OK)
    return st;
  return ensure(ctx, ctx->cc_sup, 16 * (size_t)(v / lk::kCcSuper + n_loops + 1));
}

lk_status bh_prepare(lk_ctx* ctx, const int64_t* off, int32_t n_loops, int64_t n_pairs,
                     hipStream_t s, bool can_sync) {
  int64_t v = 0;
  lk_status st;
  if ((st = read_vertices(ctx, off, n_loops, s, can_sync, &v)) != LK_OK) return st;
  const BhLayout Y = bh_layout(v, n_loops, n_pairs);
  if ((st = ensure(ctx, ctx->bh_nodes, sizeof(lk::BhNode) * (size_t)Y.nodes)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->bh_lists,
                   sizeof(lk::BhPair) * (size_t)(2 * Y.list_cap + Y.near_cap))) != LK_OK)
    return st;
  if ((st = ensure(ctx, ctx->bh_adapt, 24 * (size_t)(n_pairs + 1))) != LK_OK) return st;
  return ensure(ctx, ctx->bh_counts, 4 * (size_t)(lk::kBhMaxIters + 3));
}

bool check_dtype(int d) { return d == LK_F32 || d == LK_F64; }

lk_status set_device(lk_ctx* ctx) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return ctx->fail(LK_EDEVICE, "hipGetDevice failed");
  if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
    return ctx->fail(LK_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  return LK_OK;
}

// ------------------------------------------------ no-allocation workspace
// lk_direct_sum_noalloc runs the PLAIN_F64 / MIXED kernel sequence with its
// workspace carved from one static device array instead of the context's
// buffers.  Its limits size that array.
constexpr int32_t kNoallocMaxLoops = 65536;
constexpr int64_t kNoallocMaxPairs = 131072;

constexpr size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Byte offsets of the workspace arrays for L loops and P pairs (each aligned
// to 256 bytes; the same arrays and sizes as ensure_workspace, plus flags).
struct NoallocLayout {
  size_t lf, minseg2, xi, recs, big_prefix, meta, acc, refit, flags, total;
};

constexpr NoallocLayout noalloc_layout(size_t L, size_t P) {
  NoallocLayout y{};
  y.lf = 0;
  y.minseg2 = y.lf + al256(4 * L);
  y.xi = y.minseg2 + al256(8 * L);
  y.recs = y.xi + al256(8 * (size_t)(lk::kPrepMaxBlocks + 1));
  y.big_prefix = y.recs + al256(3 * sizeof(lk::WorkRec) * P);
  y.meta = y.big_prefix + al256(8 * (P + 1));
  y.acc = y.meta + al256(kMetaBytes);
  y.refit = y.acc + al256(16 * P);
  y.flags = y.refit + al256(8 * P);
  y.total = y.flags + al256(4 * P);
  return y;
}

constexpr size_t kNoallocBytes =
    noalloc_layout((size_t)kNoallocMaxLoops, (size_t)kNoallocMaxPairs).total;

}  // namespace

// The no-allocation entry point's workspace (about 17.6 MiB; each device the
// library runs on holds its own copy until the process ends).  Host code
// never passes this name to a kernel: it stands for a host-side shadow, not
// the device address, which is looked up per device below.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};
bool g_scratch_tried[kMaxDevices] = {};

// With `device` current: look up that device's copy of `scratch`, once.
void scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_tried[device]) return;
  g_scratch_tried[device] = true;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  g_scratch_err[device] = e;
  g_scratch_ptr[device] = e == hipSuccess ? p : nullptr;
}

}  // namespace

extern "C" {

lk_status lk_create(lk_ctx** out, int device) {
  if (!out) return LK_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LK_EDEVICE;
  if (hipSetDevice(device) != hipSuccess) return LK_EDEVICE;
  lk_ctx* ctx = new (std::nothrow) lk_ctx();
  if (!ctx) return LK_ENOMEM;
  ctx->device = device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
    delete ctx;
    return LK_EDEVICE;
  }
  ctx->n_cu = prop.multiProcessorCount;
  memset(&ctx->stats, 0, sizeof(ctx->stats));
  // messages are formatted into at most 512 bytes: with the capacity reserved
  // here, reporting an error later allocates nothing
  ctx->err.reserve(512);
  if (hipEventCreateWithFlags(&ctx->done, hipEventDisableTiming) != hipSuccess) {
    delete ctx;
    return LK_EDEVICE;
  }
  // the no-allocation entry point's device address of `scratch` on this
  // device (a failure is reported by that entry point, not here)
  scratch_setup(device);
  // a generic direction (no coordinate plane or diagonal), exact in FP32
  ctx->view[0] = 0.3671875f;
  ctx->view[1] = -0.6103515625f;
  ctx->view[2] = 1.0f;
  *out = ctx;
  return LK_OK;
}

void lk_destroy(lk_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  // the context's own work must end before its buffers go
  if (ctx->done_pending) (void)hipEventSynchronize(ctx->done);
  for (auto& kv : ctx->graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  DevBuf* bufs[] = {&ctx->loop_flags, &ctx->minseg2, &ctx->xi,      &ctx->recs,
                    &ctx->big_prefix, &ctx->meta,    &ctx->acc,     &ctx->flags,
                    &ctx->refit_list, &ctx->boxes,   &ctx->vcounts, &ctx->vprefix,
                    &ctx->cc_blk,     &ctx->cc_sup,  &ctx->bh_nodes, &ctx->bh_lists,
                    &ctx->bh_counts,  &ctx->bh_adapt, &ctx->pls_grid, &ctx->dz_piece[0], &ctx->dz_piece[1], &ctx->dz_list[0],
                    &ctx->dz_list[1], &ctx->dz_pbox, &ctx->dz_gbox, &ctx->dz_mark,
                    &ctx->dz_pre,     &ctx->dz_pair_pre, &ctx->dz_pair_ab, &ctx->dz_part,
                    &ctx->dz_loops};
  for (DevBuf* b : bufs)
    if (b->p) hipFree(b->p);
  for (auto& e : ctx->ring)
    if (e) hipEventDestroy(e);
  if (ctx->done) hipEventDestroy(ctx->done);
  delete ctx;
}

const char* lk_last_error(const lk_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

lk_status lk_set_option(lk_ctx* ctx, int key, int64_t v) {
  if (!ctx) return LK_EINVAL;
  switch (key) {
    case LK_OPT_REFIT_THRESHOLD_PPM:
      if (v < 0 || v > 500000) return ctx->fail(LK_EINVAL, "refit threshold out of [0, 0.5]");
      ctx->refit_thr = (double)v * 1e-6;
      break;
    case LK_OPT_GRAPH:
      ctx->use_graph = v != 0;
      break;
    case LK_OPT_TIMING: {
      if (v < 0 || v > 4096) return ctx->fail(LK_EINVAL, "timing ring must be in [0, 4096]");
      if (hipSetDevice(ctx->device) != hipSuccess) return ctx->fail(LK_EDEVICE, "hipSetDevice");
      hipDeviceSynchronize();
      for (auto& e : ctx->ring)
        if (e) hipEventDestroy(e);
      ctx->ring.assign(4 * (size_t)v, nullptr);
      for (auto& e : ctx->ring)
        if (hipEventCreate(&e) != hipSuccess) return ctx->fail(LK_EDEVICE, "hipEventCreate");
      ctx->ring_pos = ctx->ring_count = 0;
      ctx->timing = v != 0;
      break;
    }
    case LK_OPT_TILE_A:
      if (v != 0 && (v < 16 || v > lk::kMaxTileF32 || (v & 15)))
        return ctx->fail(LK_EINVAL, "tile must be 0 or a multiple of 16 in [16, %d]",
                         lk::kMaxTileF32);
      ctx->opt_tile = (int)v;
      break;
    case LK_OPT_CHUNK_A:
      if (v != 0 && (v < 16 || v > (1 << 24)))
        return ctx->fail(LK_EINVAL, "chunk must be 0 or in [16, 2^24]");
      ctx->opt_chunk = (int)v;
      break;
    case LK_OPT_WAVES_PER_CU:
      if (v < 0 || v > 64) return ctx->fail(LK_EINVAL, "waves per CU must be in [0, 64]");
      ctx->opt_waves = (int)v;
      break;
    case LK_OPT_ATAN:
      if (v < 0 || v > 2) return ctx->fail(LK_EINVAL, "atan form must be 0, 1 or 2");
      ctx->opt_atan = (int)v;
      break;
    case LK_OPT_SEGS_PER_LANE:
      if (v != 0 && v != 1 && v != 2 && v != 4 && v != 8)
        return ctx->fail(LK_EINVAL, "segments per lane must be 0, 1, 2, 4 or 8");
      ctx->opt_segs = (int)v;
      break;
    case LK_OPT_SMALL_BATCH:
      if (v < 0 || v > 64) return ctx->fail(LK_EINVAL, "small-pair batch must be in [0, 64]");
      ctx->opt_batch = (int)v;
      break;
    case LK_OPT_CROSSING_TOL:
      if (v < 1 || v > (1 << 20))
        return ctx->fail(LK_EINVAL, "crossing tolerance multiplier must be in [1, 2^20]");
      ctx->cc_tol = (int)v;
      break;
    case LK_OPT_CROSSING_CULL:
      if (v != 0 && v != 1) return ctx->fail(LK_EINVAL, "crossing culling must be 0 or 1");
      ctx->cc_cull = v != 0;
      break;
    case LK_OPT_BH_BETA_MILLI:
      if (v < 500 || v > 1000000)
        return ctx->fail(LK_EINVAL, "Barnes-Hut beta (x 1000) must be in [500, 1e6]");
      ctx->bh_beta = (double)v * 1e-3;
      break;
    case LK_OPT_PAIR_SEARCH:
      if (v < 0 || v > 2) return ctx->fail(LK_EINVAL, "pair search must be 0, 1 or 2");
      ctx->pair_search = (int)v;
      return LK_OK;  // no captured graph depends on it
    case LK_OPT_BH_ADAPTIVE:
      if (v != 0 && v != 1) return ctx->fail(LK_EINVAL, "adaptive beta must be 0 or 1");
      ctx->bh_adaptive = v != 0;
      break;
    case LK_OPT_BH_BETA_MAX_MILLI:
      if (v < 500 || v > 1000000)
        return ctx->fail(LK_EINVAL, "Barnes-Hut beta_max (x 1000) must be in [500, 1e6]");
      ctx->bh_beta_max = (double)v * 1e-3;
      break;
    case LK_OPT_BH_TARGET_PPM:
      if (v < 1 || v > 1000000)
        return ctx->fail(LK_EINVAL, "Barnes-Hut error target (ppm) must be in [1, 1e6]");
      ctx->bh_target = (double)v * 1e-6;
      break;
    case LK_OPT_BH_ORDER:
      if (v != 1 && v != 2) return ctx->fail(LK_EINVAL, "Barnes-Hut order must be 1 or 2");
      ctx->bh_order = (int)v;
      break;
    case LK_OPT_DZ_MAX_PASSES:
      if (v < 1 || v > 1000) return ctx->fail(LK_EINVAL, "discretization passes must be in [1, 1000]");
      ctx->dz_max_passes = (int)v;
      return LK_OK;  // no captured graph depends on it
    case LK_OPT_SEGS_PER_LANE_F64:
      if (v != 0 && v != 1 && v != 2)
        return ctx->fail(LK_EINVAL, "FP64 segments per lane must be 0, 1 or 2");
      ctx->opt_segs64 = (int)v;
      break;
    default:
      return ctx->fail(LK_EINVAL, "unknown option %d", key);
  }
  // configuration is baked into captured graphs
  for (auto& kv : ctx->graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  ctx->graphs.clear();
  return LK_OK;
}

lk_status lk_set_view_direction(lk_ctx* ctx, const double* dir) {
  if (!ctx) return LK_EINVAL;
  if (!dir) return ctx->fail(LK_EINVAL, "null direction");
  double m = 0.0;
  for (int q = 0; q < 3; ++q) {
    if (!std::isfinite(dir[q])) return ctx->fail(LK_EINVAL, "non-finite direction");
    m = std::max(m, std::fabs(dir[q]));
  }
  if (!(m > 0.0)) return ctx->fail(LK_EINVAL, "zero direction");
  float v[3];
  for (int q = 0; q < 3; ++q) v[q] = (float)(dir[q] / m);
  // rounding keeps the largest component at magnitude 1 and the others <= 1
  for (int q = 0; q < 3; ++q) ctx->view[q] = v[q];
  for (auto& kv : ctx->graphs)
    if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
  ctx->graphs.clear();
  return LK_OK;
}

lk_status lk_get_view_direction(const lk_ctx* ctx, double* dir) {
  if (!ctx || !dir) return LK_EINVAL;
  for (int q = 0; q < 3; ++q) dir[q] = (double)ctx->view[q];
  return LK_OK;
}

namespace {

lk_status direct_sum_enqueue(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                             int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                             double* lk_real, int32_t* lk_int, uint32_t* flags, void* stream,
                             const Check& ck) {
  if (!ctx) return LK_EINVAL;
  ctx->err.clear();
  if (!check_dtype(dtype)) return ctx->fail(LK_EINVAL, "unknown dtype %d", dtype);
  if (mode != LK_PLAIN_F64 && mode != LK_MIXED && mode != LK_CROSSINGS && mode != LK_BARNES_HUT)
    return ctx->fail(LK_EINVAL, "unknown mode %d", mode);
  if (n_loops < 1) return ctx->fail(LK_EINVAL, "n_loops must be >= 1");
  if (n_pairs < 0) return ctx->fail(LK_EINVAL, "n_pairs must be >= 0");
  if (n_pairs > 0x7fffffffLL) return ctx->fail(LK_EINVAL, "n_pairs exceeds int32 range");
  if (!xyz || !off || (n_pairs > 0 && (!pairs || !lk_real || !lk_int)))
    return ctx->fail(LK_EINVAL, "null pointer argument");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  ctx->stats = lk_stats{};
  if (n_pairs == 0) {
    if (ck.n_mismatch) LK_HIP(lk::launch_zero_i64(ck.n_mismatch, s));
    return LK_OK;
  }

  const bool in_f64 = dtype == LK_F64;
  const bool mixed = mode != LK_PLAIN_F64;
  const Plan P = make_plan(ctx, in_f64, mode, n_pairs);
  if ((st = ensure_workspace(ctx, n_loops, n_pairs)) != LK_OK) return st;
  if (P.crossings || P.bh) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (s && hipStreamIsCapturing(s, &cs) != hipSuccess) cs = hipStreamCaptureStatusNone;
    const bool can_sync = cs == hipStreamCaptureStatusNone;
    if (P.crossings && (st = cc_prepare(ctx, off, n_loops, s, can_sync)) != LK_OK) return st;
    if (P.bh && (st = bh_prepare(ctx, off, n_loops, n_pairs, s, can_sync)) != LK_OK) return st;
  }
  if (!flags) {
    if ((st = ensure(ctx, ctx->flags, 4 * (size_t)n_pairs)) != LK_OK) return st;
    flags = (uint32_t*)ctx->flags.p;
  }

  ctx->stats.tile_a = P.tile;
  ctx->stats.chunk_a = P.chunk;
  ctx->stats.waves_per_cu = (mixed ? P.grid : P.grid64) / (ctx->n_cu > 0 ? ctx->n_cu : 1);
  ctx->stats.atan_form = P.atan_form;
  ctx->stats.segs_per_lane = mixed ? P.segs : P.segs64;
  ctx->last_stream = s;
  ctx->last_mixed = mixed;
  ctx->last_crossings = P.crossings;
  ctx->last_bh = P.bh;
  ctx->last_timed = false;

  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (s) {
    if (hipStreamIsCapturing(s, &cap) != hipSuccess) cap = hipStreamCaptureStatusNone;
  }
  const bool timed = ctx->timing;
  const bool graph_ok = ctx->use_graph && !timed && s != nullptr && cap == hipStreamCaptureStatusNone;
  if (!graph_ok) {
    hipEvent_t* ev = nullptr;
    if (timed) {
      const int slots = (int)(ctx->ring.size() / 4);
      ev = &ctx->ring[4 * (size_t)(ctx->ring_pos % slots)];
    }
    st = enqueue_direct_sum(ctx, ctx_ws(ctx), P, xyz, off, n_loops, pairs, n_pairs, lk_real, lk_int, flags, s,
                            ev, ck);
    if (timed && st == LK_OK) {
      const int slots = (int)(ctx->ring.size() / 4);
      ctx->ring_pos = (ctx->ring_pos + 1) % slots;
      if (ctx->ring_count < slots) ctx->ring_count++;
      ctx->last_timed = true;
    }
    return st;
  }
  GraphKey key{xyz, dtype, off, n_loops, pairs, n_pairs, mode, lk_real, lk_int, flags,
               P.tile, P.chunk, P.grid,
               ctx->opt_batch * 1024 + P.atan_form * 16 + P.segs * 4 + P.segs64,
               (int64_t)(ctx->refit_thr * 1e9), ck.expected, ck.n_mismatch, ck.early_exit};
  auto it = ctx->graphs.find(key);
  if (it != ctx->graphs.end() && it->second.epoch == ctx->ws_epoch && it->second.exec) {
    LK_HIP(hipGraphLaunch(it->second.exec, s));
    ctx->stats.graph_replayed = 1;
    return LK_OK;
  }
  if (it != ctx->graphs.end()) {
    if (it->second.exec) hipGraphExecDestroy(it->second.exec);
    ctx->graphs.erase(it);
  }
  LK_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  st = enqueue_direct_sum(ctx, ctx_ws(ctx), P, xyz, off, n_loops, pairs, n_pairs, lk_real, lk_int, flags, s,
                          nullptr, ck);
  hipGraph_t g = nullptr;
  hipError_t ce = hipStreamEndCapture(s, &g);
  if (st != LK_OK) {
    if (g) hipGraphDestroy(g);
    return st;
  }
  if (ce != hipSuccess || !g) return ctx->fail(LK_EDEVICE, "graph capture failed: %s",
                                               hipGetErrorString(ce));
  hipGraphExec_t ex = nullptr;
  hipError_t ie = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  hipGraphDestroy(g);
  if (ie != hipSuccess) return ctx->fail(LK_EDEVICE, "graph instantiate: %s", hipGetErrorString(ie));
  if (ctx->graphs.size() > 64) {
    for (auto& kv : ctx->graphs)
      if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    ctx->graphs.clear();
  }
  ctx->graphs[key] = {ex, ctx->ws_epoch};
  LK_HIP(hipGraphLaunch(ex, s));
  return LK_OK;
}

lk_status direct_sum_call(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                          int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                          double* lk_real, int32_t* lk_int, uint32_t* flags, void* stream,
                          const Check& ck) {
  const lk_status st = direct_sum_enqueue(ctx, xyz, dtype, off, n_loops, pairs, n_pairs, mode,
                                          lk_real, lk_int, flags, stream, ck);
  if (st == LK_OK) mark_done(ctx, (hipStream_t)stream);
  return st;
}

}  // namespace

lk_status lk_direct_sum(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                        int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                        double* lk_real, int32_t* lk_int, uint32_t* flags, void* stream) {
  return direct_sum_call(ctx, xyz, dtype, off, n_loops, pairs, n_pairs, mode, lk_real, lk_int,
                         flags, stream, Check());
}

lk_status lk_direct_sum_check(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                              int32_t n_loops, const int32_t* pairs, int64_t n_pairs,
                              const int32_t* expected, int early_exit, int mode, double* lk_real,
                              int32_t* lk_int, uint32_t* flags, int64_t* n_mismatch,
                              void* stream) {
  if (!ctx) return LK_EINVAL;
  if (!n_mismatch || (n_pairs > 0 && !expected)) {
    ctx->err.clear();
    return ctx->fail(LK_EINVAL, "null expected or n_mismatch");
  }
  Check ck;
  ck.expected = expected;
  ck.early_exit = early_exit ? 1 : 0;
  ck.n_mismatch = n_mismatch;
  return direct_sum_call(ctx, xyz, dtype, off, n_loops, pairs, n_pairs, mode, lk_real, lk_int,
                         flags, stream, ck);
}

lk_status lk_direct_sum_noalloc(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                                int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                                double* lk_real, int32_t* lk_int, uint32_t* flags, void* stream) {
  if (!ctx) return LK_EINVAL;
  ctx->err.clear();
  if (!check_dtype(dtype)) return ctx->fail(LK_EINVAL, "unknown dtype %d", dtype);
  if (mode != LK_PLAIN_F64 && mode != LK_MIXED)
    return ctx->fail(LK_EINVAL, "mode %d: the no-allocation direct sum runs PLAIN_F64 and MIXED only",
                     mode);
  if (n_loops < 1) return ctx->fail(LK_EINVAL, "n_loops must be >= 1");
  if (n_pairs < 0) return ctx->fail(LK_EINVAL, "n_pairs must be >= 0");
  if (n_loops > kNoallocMaxLoops || n_pairs > kNoallocMaxPairs)
    return ctx->fail(LK_ECAPACITY,
                     "%d loops and %lld pairs exceed the static workspace (at most %d loops and "
                     "%lld pairs)",
                     n_loops, (long long)n_pairs, kNoallocMaxLoops, (long long)kNoallocMaxPairs);
  if (!xyz || !off || (n_pairs > 0 && (!pairs || !lk_real || !lk_int)))
    return ctx->fail(LK_EINVAL, "null pointer argument");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (ctx->device < kMaxDevices) base = (char*)g_scratch_ptr[ctx->device];
    if (!base)
      return ctx->fail(LK_EDEVICE, "static workspace of device %d unavailable: %s", ctx->device,
                       ctx->device < kMaxDevices && g_scratch_tried[ctx->device]
                           ? hipGetErrorString(g_scratch_err[ctx->device])
                           : "not set up");
  }
  hipStream_t s = (hipStream_t)stream;
  // lk_get_stats reports this call's configuration, not its refit count
  ctx->stats = lk_stats{};
  ctx->last_mixed = ctx->last_crossings = ctx->last_bh = ctx->last_timed = false;
  if (n_pairs == 0) return LK_OK;

  const NoallocLayout y = noalloc_layout((size_t)n_loops, (size_t)n_pairs);
  Ws W;
  W.loop_flags = (uint32_t*)(base + y.lf);
  W.minseg2 = (double*)(base + y.minseg2);
  W.xi = (double*)(base + y.xi);
  W.recs = (lk::WorkRec*)(base + y.recs);
  W.big_prefix = (int64_t*)(base + y.big_prefix);
  W.meta = base + y.meta;
  W.acc = (unsigned long long*)(base + y.acc);
  W.refit_list = (int32_t*)(base + y.refit);
  if (!flags) flags = (uint32_t*)(base + y.flags);

  const bool mixed = mode == LK_MIXED;
  const Plan P = make_plan(ctx, dtype == LK_F64, mode, n_pairs);
  ctx->stats.tile_a = P.tile;
  ctx->stats.chunk_a = P.chunk;
  ctx->stats.waves_per_cu = (mixed ? P.grid : P.grid64) / (ctx->n_cu > 0 ? ctx->n_cu : 1);
  ctx->stats.atan_form = P.atan_form;
  ctx->stats.segs_per_lane = mixed ? P.segs : P.segs64;
  // eager launches only: instantiating a graph would allocate
  return enqueue_direct_sum(ctx, W, P, xyz, off, n_loops, pairs, n_pairs, lk_real, lk_int, flags,
                            s, nullptr);
}

lk_status lk_get_stats(lk_ctx* ctx, lk_stats* out) {
  if (!ctx || !out) return LK_EINVAL;
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  if (ctx->last_mixed && ctx->meta.p) {
    LK_HIP(hipStreamSynchronize(ctx->last_stream));
    int32_t rn = 0, rn2 = 0;
    LK_HIP(hipMemcpy(&rn, meta_at<int32_t>(ctx, kMetaRefitN), 4, hipMemcpyDeviceToHost));
    if (ctx->last_crossings)
      LK_HIP(hipMemcpy(&rn2, meta_at<int32_t>(ctx, kMetaRefitN2), 4, hipMemcpyDeviceToHost));
    ctx->stats.refits = rn;
    ctx->stats.refits_direct_sum = rn2;
    if (ctx->last_bh && ctx->bh_counts.p) {
      int32_t c[lk::kBhMaxIters + 3];
      LK_HIP(hipMemcpy(c, ctx->bh_counts.p, sizeof(c), hipMemcpyDeviceToHost));
      int64_t peak = 0;
      for (int k = 0; k <= lk::kBhMaxIters; ++k) peak = std::max<int64_t>(peak, c[k]);
      ctx->stats.bh_list_peak = peak;
      ctx->stats.bh_near_pairs = c[lk::kBhMaxIters + 1];
      ctx->stats.bh_list_cap = ctx->last_bh_list_cap;
      ctx->stats.bh_reruns = ctx->bh_adaptive ? c[lk::kBhMaxIters + 2] : 0;
    }
  }
  if (ctx->timing && ctx->ring_count > 0) {
    LK_HIP(hipStreamSynchronize(ctx->last_stream));
    double sum = 0.0, rsum = 0.0;
    for (int k = 0; k < ctx->ring_count; ++k) {
      float ms = 0.f;
      LK_HIP(hipEventElapsedTime(&ms, ctx->ring[4 * k], ctx->ring[4 * k + 1]));
      sum += ms;
      if (ctx->last_mixed) {
        LK_HIP(hipEventElapsedTime(&ms, ctx->ring[4 * k + 2], ctx->ring[4 * k + 3]));
        rsum += ms;
      }
    }
    ctx->stats.kernel_ms = sum / ctx->ring_count;
    ctx->stats.refit_kernel_ms = rsum / ctx->ring_count;
    ctx->stats.timed_calls = ctx->ring_count;
  }
  *out = ctx->stats;
  return LK_OK;
}

lk_status lk_build_pairs(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                         int32_t n_loops, int32_t* pairs_out, int64_t capacity, int64_t* n_pairs,
                         void* stream) {
  if (!ctx) return LK_EINVAL;
  ctx->err.clear();
  if (!check_dtype(dtype)) return ctx->fail(LK_EINVAL, "unknown dtype %d", dtype);
  if (n_loops < 1) return ctx->fail(LK_EINVAL, "n_loops must be >= 1");
  if (capacity < 0) return ctx->fail(LK_EINVAL, "capacity must be >= 0");
  if (!xyz || !off || !n_pairs || (capacity > 0 && !pairs_out))
    return ctx->fail(LK_EINVAL, "null pointer argument");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ensure(ctx, ctx->boxes, 48 * (size_t)n_loops)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->vcounts, 8 * (size_t)n_loops)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->vprefix, 8 * (size_t)(n_loops + 1))) != LK_OK) return st;
  double* boxes = (double*)ctx->boxes.p;
  int64_t* cnt = (int64_t*)ctx->vcounts.p;
  int64_t* pre = (int64_t*)ctx->vprefix.p;
  // the grid pays off beyond a few thousand loops; both give the same pairs
  const bool grid = ctx->pair_search == 2 || (ctx->pair_search == 0 && n_loops >= 2048);
  lk::GridBufs G{};
  if (grid) {
    const size_t L = (size_t)n_loops;
    G.buckets = 64;  // a power of two of at least 4 buckets per loop
    while (G.buckets < 4 * (int64_t)n_loops) G.buckets *= 2;
    const size_t mc = (size_t)G.buckets;
    const size_t o_cnt = 64, o_start = o_cnt + 8 * mc, o_of = o_start + 8 * (mc + 1);
    const size_t o_cbox = o_of + 8 * L, o_items = o_cbox + 48 * L;
    const size_t o_over = o_items + 4 * L, o_nover = o_over + 4 * L;
    const size_t o_part = o_nover + 64, o_tiles = o_part + 8 * 6 * lk::kGridStatBlocks;
    const size_t n_tiles = (mc + 4095) / 4096;
    if ((st = ensure(ctx, ctx->pls_grid, o_tiles + 8 * 2 * (n_tiles + 2))) != LK_OK) return st;
    char* gb = (char*)ctx->pls_grid.p;
    G.params = (lk::GridParams*)gb;
    G.cell_count = (unsigned long long*)(gb + o_cnt);
    G.cell_start = (int64_t*)(gb + o_start);
    G.cell_of = (int64_t*)(gb + o_of);
    G.cell_items = (int32_t*)(gb + o_items);
    G.cell_box = (double*)(gb + o_cbox);
    G.over = (int32_t*)(gb + o_over);
    G.n_over = (int32_t*)(gb + o_nover);
    G.part = (double*)(gb + o_part);
    G.tiles = (int64_t*)(gb + o_tiles);
    G.row_counts = cnt;
  }
  LK_HIP(lk::launch_boxes(xyz, dtype == LK_F64, off, n_loops, boxes, s));
  if (grid)
    LK_HIP(lk::launch_grid_pairs(boxes, n_loops, G, 0, nullptr, nullptr, s));
  else
    LK_HIP(lk::launch_pair_count(boxes, n_loops, cnt, s));
  LK_HIP(lk::launch_scan(cnt, n_loops, pre, s));
  int64_t total = 0;
  LK_HIP(hipMemcpyAsync(&total, pre + n_loops, 8, hipMemcpyDeviceToHost, s));
  LK_HIP(hipStreamSynchronize(s));
  *n_pairs = total;
  if (total > 0 && total <= capacity) {
    if (grid)
      LK_HIP(lk::launch_grid_pairs(boxes, n_loops, G, 1, pre, pairs_out, s));
    else
      LK_HIP(lk::launch_pair_fill(boxes, n_loops, pre, pairs_out, capacity, s));
    LK_HIP(hipStreamSynchronize(s));
  }
  if (total > capacity)
    return ctx->fail(LK_ECAPACITY, "%lld pairs do not fit capacity %lld", (long long)total,
                     (long long)capacity);
  return LK_OK;
}

lk_status lk_discretize(lk_ctx* ctx, const double* ctrl, const int64_t* ctrl_offsets,
                        int32_t n_loops, int kind, const int32_t* pairs, int64_t n_pairs,
                        double* xyz_out, int64_t capacity, int64_t* offsets_out,
                        uint32_t* loop_flags, int64_t* n_vertices, lk_dz_info* info,
                        void* stream) {
  if (!ctx) return LK_EINVAL;
  ctx->err.clear();
  if (kind != LK_DZ_BSPLINE && kind != LK_DZ_POLYLINE)
    return ctx->fail(LK_EINVAL, "unknown curve kind %d", kind);
  if (n_loops < 1) return ctx->fail(LK_EINVAL, "n_loops must be >= 1");
  if (n_pairs < 0 || capacity < 0) return ctx->fail(LK_EINVAL, "negative size");
  if (!ctrl || !ctrl_offsets || !offsets_out || !n_vertices || (n_pairs > 0 && !pairs) ||
      (capacity > 0 && !xyz_out))
    return ctx->fail(LK_EINVAL, "null pointer argument");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if (s) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return ctx->fail(LK_EBUSY, "lk_discretize synchronises and cannot be captured");
  }
  // the point count sizes every buffer: read it, and whether the offsets
  // ever decrease (one synchronisation)
  const size_t L = (size_t)n_loops;
  const size_t o_lsum = (4 * L + 7) / 8 * 8, o_off = o_lsum + 8 * L;
  const size_t o_tot = o_off + 4 * 8 * (L + 1), o_lim = o_tot + 32;
  if ((st = ensure(ctx, ctx->dz_loops, o_lim + 8)) != LK_OK) return st;
  int32_t* bad_d = (int32_t*)((char*)ctx->dz_loops.p + o_tot);  // the totals slot, free until the passes
  int64_t ends[2] = {0, 0};
  int32_t bad = 0;
  LK_HIP(hipMemsetAsync(bad_d, 0, 4, s));
  LK_HIP(lk::launch_dz_check(ctrl_offsets, n_loops, bad_d, s));
  LK_HIP(hipMemcpyAsync(&bad, bad_d, 4, hipMemcpyDeviceToHost, s));
  LK_HIP(hipMemcpyAsync(&ends[0], ctrl_offsets, 8, hipMemcpyDeviceToHost, s));
  LK_HIP(hipMemcpyAsync(&ends[1], ctrl_offsets + n_loops, 8, hipMemcpyDeviceToHost, s));
  LK_HIP(hipStreamSynchronize(s));
  const int64_t N = ends[1] - ends[0];
  if (bad || N < 0) return ctx->fail(LK_EINVAL, "offsets decrease");
  // piece indices are int32 and the split packs two 32-bit counts
  const int64_t kMaxPieces = (int64_t)1 << 30;
  if (N > kMaxPieces) return ctx->fail(LK_EINVAL, "more than 2^30 input spans");
  // per-loop block (sized above): lflags [L] u32 | lsum [L] f64 | 4 offset
  // arrays [L+1] i64 | totals [4] u64 | lim2 f64
  if ((st = ensure(ctx, ctx->dz_pair_pre, 8 * (size_t)(n_pairs + 1))) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->dz_pair_ab, 8 * (size_t)(n_pairs + 1))) != LK_OK) return st;
  auto piece_cap = [](const DevBuf& b) { return (int64_t)(b.bytes / lk::kDzBytesPerPiece); };
  auto open_cap = [](const DevBuf& b) { return (int64_t)(b.bytes / lk::kDzBytesPerOpen); };
  auto pieces_of = [&](const DevBuf& b) {
    lk::DzPieces P;
    P.cap = piece_cap(b);
    P.start = (double*)b.p;
    P.loop = (int32_t*)((char*)b.p + 24 * (size_t)P.cap);
    P.state = (uint32_t*)((char*)b.p + 28 * (size_t)P.cap);
    return P;
  };
  // sizes the buffers of a pass over n pieces of which nu are unprocessed
  // (the current arrays already hold them; the next ones are written whole)
  auto size_pass = [&](int64_t n, int64_t nu, int cur) -> lk_status {
    lk_status r;
    const size_t want = (size_t)(n + nu > 0 ? n + nu : 1);
    if ((size_t)piece_cap(ctx->dz_piece[cur ^ 1]) < want &&
        (r = ensure(ctx, ctx->dz_piece[cur ^ 1], lk::kDzBytesPerPiece * want)) != LK_OK)
      return r;
    if ((size_t)open_cap(ctx->dz_list[cur ^ 1]) < (size_t)(2 * nu + 1) &&
        (r = ensure(ctx, ctx->dz_list[cur ^ 1], lk::kDzBytesPerOpen * (size_t)(2 * nu + 1))) !=
            LK_OK)
      return r;
    if ((r = ensure(ctx, ctx->dz_pbox, 48 * (size_t)(nu + 1))) != LK_OK) return r;
    if ((r = ensure(ctx, ctx->dz_gbox, 48 * (size_t)(nu / lk::kDzGroup + L + 1))) != LK_OK)
      return r;
    if ((r = ensure(ctx, ctx->dz_mark, 4 * (size_t)(nu + 1))) != LK_OK) return r;
    if ((r = ensure(ctx, ctx->dz_pre, 8 * (size_t)(n + 1))) != LK_OK) return r;
    const int64_t nb = (std::max(n, n_pairs) + lk::kDzScanBlock - 1) / lk::kDzScanBlock + 1;
    return ensure(ctx, ctx->dz_part, 8 * (size_t)nb);
  };
  int cur = 0;
  if ((size_t)piece_cap(ctx->dz_piece[0]) < (size_t)(N > 0 ? N : 1) &&
      (st = ensure(ctx, ctx->dz_piece[0], lk::kDzBytesPerPiece * (size_t)(N > 0 ? N : 1))) != LK_OK)
    return st;
  if ((size_t)open_cap(ctx->dz_list[0]) < (size_t)(N + 1) &&
      (st = ensure(ctx, ctx->dz_list[0], lk::kDzBytesPerOpen * (size_t)(N + 1))) != LK_OK)
    return st;
  if ((st = size_pass(N, N, cur)) != LK_OK) return st;
  // every buffer is final for this pass; the pointers are taken after sizing
  auto args = [&](int c, int64_t n, int64_t nu) {
    lk::DzArgs a;
    memset(&a, 0, sizeof(a));
    a.ctrl = ctrl;
    a.cp_off = ctrl_offsets;
    a.n_loops = n_loops;
    a.kind = kind;
    a.pairs = pairs;
    a.n_pairs = n_pairs;
    a.eps = 2.220446049250313e-16;  // FP64 machine epsilon (2^-52)
    a.cur = pieces_of(ctx->dz_piece[c]);
    a.nxt = pieces_of(ctx->dz_piece[c ^ 1]);
    a.ubz_cur = (double*)ctx->dz_list[c].p;
    a.ubz_nxt = (double*)ctx->dz_list[c ^ 1].p;
    a.cap_o = open_cap(ctx->dz_list[c]);
    a.cap_on = open_cap(ctx->dz_list[c ^ 1]);
    char* lb = (char*)ctx->dz_loops.p;
    a.lflags = (uint32_t*)lb;
    a.lsum = (double*)(lb + o_lsum);
    int64_t* offs = (int64_t*)(lb + o_off);
    a.aoff_cur = offs + (c ? 2 : 0) * (L + 1);
    a.aoff_nxt = offs + (c ? 0 : 2) * (L + 1);
    a.uoff_cur = offs + (c ? 3 : 1) * (L + 1);
    a.uoff_nxt = offs + (c ? 1 : 3) * (L + 1);
    a.totals = (uint64_t*)(lb + o_tot);
    a.lim2 = (double*)(lb + o_lim);
    a.cap_u = (int64_t)(ctx->dz_pbox.bytes / 48);
    a.pbox = (double*)ctx->dz_pbox.p;
    a.cap_g = (int64_t)(ctx->dz_gbox.bytes / 48);
    a.gbox = (double*)ctx->dz_gbox.p;
    a.mark = (uint32_t*)ctx->dz_mark.p;
    a.pre = (uint64_t*)ctx->dz_pre.p;
    a.pair_pre = (int64_t*)ctx->dz_pair_pre.p;
    a.pair_ab = (int32_t*)ctx->dz_pair_ab.p;
    a.part = (uint64_t*)ctx->dz_part.p;
    a.n = n;
    a.n_u = nu;
    return a;
  };
  LK_HIP(lk::launch_dz_setup(args(cur, N, N), N, s));
  int64_t n = N, nu = N;
  int passes = 0;
  int64_t splits = 0;
  while (nu > 0 && passes < ctx->dz_max_passes) {
    if ((st = size_pass(n, nu, cur)) != LK_OK) return st;
    lk::DzArgs a = args(cur, n, nu);
    LK_HIP(lk::launch_dz_pass(a, ctx->n_cu, s));
    uint64_t tot = 0;
    LK_HIP(hipMemcpyAsync(&tot, a.totals, 8, hipMemcpyDeviceToHost, s));
    LK_HIP(hipStreamSynchronize(s));
    const int64_t n2 = (int64_t)(tot >> 32), nu2 = (int64_t)(tot & 0xffffffffull);
    splits += n2 - n;
    n = n2;
    nu = nu2;
    cur ^= 1;
    ++passes;
    if (n > kMaxPieces)
      return ctx->fail(LK_ENOMEM, "refinement exceeds 2^30 pieces (curves nearly touch?)");
  }
  *n_vertices = n;
  lk::DzArgs a = args(cur, n, nu);
  LK_HIP(lk::launch_dz_finish(a, xyz_out, capacity, offsets_out, loop_flags, s));
  mark_done(ctx, s);
  if (info) {
    memset(info, 0, sizeof(*info));
    info->passes = passes;
    info->input_spans = N;
    info->vertices = n;
    info->splits = splits;
    info->unfinished = nu;
  }
  if (n > capacity) {
    LK_HIP(hipStreamSynchronize(s));
    return ctx->fail(LK_ECAPACITY, "%lld vertices do not fit capacity %lld", (long long)n,
                     (long long)capacity);
  }
  return LK_OK;
}

lk_status lk_verify(lk_ctx* ctx, const int32_t* pairs, const int32_t* lk, int64_t n,
                    const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp, int early_exit,
                    int64_t* n_mismatch, int32_t* mismatches, int64_t cap, void* stream) {
  if (!ctx) return LK_EINVAL;
  ctx->err.clear();
  if (n < 0 || n_exp < 0 || cap < 0) return ctx->fail(LK_EINVAL, "negative size");
  if (!n_mismatch || (n > 0 && (!pairs || !lk)) || (n_exp > 0 && (!exp_pairs || !exp_lk)) ||
      (cap > 0 && !mismatches))
    return ctx->fail(LK_EINVAL, "null pointer argument");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  *n_mismatch = 0;
  const int64_t m = n + n_exp;
  if (m == 0) return LK_OK;
  if ((st = ensure(ctx, ctx->vcounts, 8 * (size_t)m)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->vprefix, 8 * (size_t)(m + 1))) != LK_OK) return st;
  int64_t* flag = (int64_t*)ctx->vcounts.p;
  int64_t* pre = (int64_t*)ctx->vprefix.p;
  LK_HIP(lk::launch_verify(pairs, lk, n, exp_pairs, exp_lk, n_exp, flag, s));
  LK_HIP(lk::launch_scan(flag, m, pre, s));
  int64_t total = 0;
  LK_HIP(hipMemcpyAsync(&total, pre + m, 8, hipMemcpyDeviceToHost, s));
  LK_HIP(hipStreamSynchronize(s));
  int64_t c = cap;
  if (early_exit) {
    total = total > 0 ? 1 : 0;
    c = cap < 1 ? cap : 1;
  }
  *n_mismatch = total;
  if (total > 0 && c > 0) {
    LK_HIP(lk::launch_verify_scatter(pairs, lk, n, exp_pairs, exp_lk, n_exp, pre, mismatches, c, s));
    LK_HIP(hipStreamSynchronize(s));
  }
  return LK_OK;
}

lk_status lk_reserve(lk_ctx* ctx, int32_t max_loops, int64_t max_pairs, int64_t max_verify) {
  if (!ctx) return LK_EINVAL;
  if (max_loops < 1 || max_pairs < 1 || max_verify < 0)
    return ctx->fail(LK_EINVAL, "bad reservation sizes");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  if ((st = ensure_workspace(ctx, max_loops, max_pairs)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->flags, 4 * (size_t)max_pairs)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->boxes, 48 * (size_t)max_loops)) != LK_OK) return st;
  const int64_t nv = max_verify > max_loops ? max_verify : max_loops;
  if ((st = ensure(ctx, ctx->vcounts, 8 * (size_t)nv)) != LK_OK) return st;
  if ((st = ensure(ctx, ctx->vprefix, 8 * (size_t)(nv + 1))) != LK_OK) return st;
  return LK_OK;
}

lk_status lk_autotune(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* off,
                      int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                      double* lk_real, int32_t* lk_int, uint32_t* flags, const char* cache_path,
                      lk_tuning* out, void* stream) {
  if (!ctx) return LK_EINVAL;
  ctx->err.clear();
  if (!out) return ctx->fail(LK_EINVAL, "null output");
  if (!check_dtype(dtype)) return ctx->fail(LK_EINVAL, "unknown dtype %d", dtype);
  if (mode != LK_PLAIN_F64 && mode != LK_MIXED && mode != LK_CROSSINGS)
    return ctx->fail(LK_EINVAL, "unknown mode %d", mode);
  if (n_loops < 1 || n_pairs < 1 || n_pairs > 0x7fffffffLL)
    return ctx->fail(LK_EINVAL, "need n_loops >= 1 and 1 <= n_pairs < 2^31");
  if (!xyz || !off || !pairs || !lk_real || !lk_int)
    return ctx->fail(LK_EINVAL, "null pointer argument");
  lk_status st = set_device(ctx);
  if (st != LK_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  const bool in_f64 = dtype == LK_F64;
  const bool mixed = mode != LK_PLAIN_F64;
  const bool crossings = mode == LK_CROSSINGS;
  *out = lk_tuning{};

  // workload profile, read once from the device
  std::vector<int64_t> ho((size_t)n_loops + 1);
  std::vector<int32_t> hp(2 * (size_t)n_pairs);
  LK_HIP(hipStreamSynchronize(s));
  LK_HIP(hipMemcpy(ho.data(), off, 8 * ho.size(), hipMemcpyDeviceToHost));
  LK_HIP(hipMemcpy(hp.data(), pairs, 4 * hp.size(), hipMemcpyDeviceToHost));
  double terms = 0.0, max_terms = 0.0;
  int64_t n_small = 0, n_big = 0;
  for (int64_t q = 0; q < n_pairs; ++q) {
    const int32_t i = hp[2 * q], j = hp[2 * q + 1];
    if (i < 0 || j < 0 || i >= n_loops || j >= n_loops || i == j) continue;
    const double na = (double)(ho[i + 1] - ho[i]), nb = (double)(ho[j + 1] - ho[j]);
    terms += na * nb;
    max_terms = std::max(max_terms, na * nb);
    if (na < lk::kSmallA && nb <= 256) ++n_small; else ++n_big;
  }
  hipDeviceProp_t prop;
  LK_HIP(hipGetDeviceProperties(&prop, ctx->device));
  char key[512];
  snprintf(key, sizeof(key), "%s|mode%d|dtype%d|L%d|P%lld|V%lld|T%.3e|max%.3e|small%lld",
           prop.gcnArchName, mode, dtype, n_loops, (long long)n_pairs,
           (long long)(ho[n_loops] - ho[0]), terms, max_terms, (long long)n_small);

  auto apply = [&](const lk_tuning& t) {
    ctx->opt_segs = t.segs_per_lane;
    ctx->opt_segs64 = t.segs_per_lane_f64;
    ctx->opt_tile = t.tile_a;
    ctx->opt_chunk = t.chunk_a;
    ctx->opt_batch = t.small_batch;
    ctx->opt_waves = t.waves_per_cu;
    ctx->opt_atan = t.atan_form;
    for (auto& kv : ctx->graphs)
      if (kv.second.exec) hipGraphExecDestroy(kv.second.exec);
    ctx->graphs.clear();
  };

  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      lk_tuning t{};
      if (ls >> k >> t.segs_per_lane >> t.segs_per_lane_f64 >> t.tile_a >> t.chunk_a >>
          t.small_batch >> t.waves_per_cu >> t.best_ms >> t.start_ms >> t.atan_form) {
        if (k == key && t.atan_form >= 0 && t.atan_form <= 2) {
          t.from_cache = 1;
          apply(t);
          *out = t;
          return LK_OK;
        }
      }
    }
  }

  if ((st = ensure_workspace(ctx, n_loops, n_pairs)) != LK_OK) return st;
  if (crossings && (st = cc_prepare(ctx, off, n_loops, s, true)) != LK_OK) return st;
  if (!flags) {
    if ((st = ensure(ctx, ctx->flags, 4 * (size_t)n_pairs)) != LK_OK) return st;
    flags = (uint32_t*)ctx->flags.p;
  }
  hipEvent_t ev[4];
  for (auto& e : ev) LK_HIP(hipEventCreate(&e));
  struct Guard {
    hipEvent_t* e;
    ~Guard() {
      for (int k = 0; k < 4; ++k) hipEventDestroy(e[k]);
    }
  } guard{ev};

  // start from the current options, filled with the defaults
  lk_tuning cur{};
  cur.segs_per_lane = ctx->opt_segs ? ctx->opt_segs : kDefaultSegs32;
  cur.segs_per_lane_f64 = ctx->opt_segs64 ? ctx->opt_segs64 : kDefaultSegs64;
  cur.tile_a = ctx->opt_tile ? ctx->opt_tile : default_tile(!mixed);
  cur.chunk_a = ctx->opt_chunk ? ctx->opt_chunk : default_chunk(!mixed);
  cur.small_batch = ctx->opt_batch ? ctx->opt_batch : kDefaultBatch;
  cur.waves_per_cu = ctx->opt_waves;
  cur.atan_form = ctx->opt_atan;
  int evaluated = 0;
  auto measure = [&](const lk_tuning& t, double* ms) -> lk_status {
    apply(t);
    const Plan P = make_plan(ctx, in_f64, mode, n_pairs);
    double best = 1e30;
    int reps = 3;
    for (int r = 0; r <= reps; ++r) {
      lk_status e = enqueue_direct_sum(ctx, ctx_ws(ctx), P, xyz, off, n_loops, pairs, n_pairs, lk_real, lk_int,
                                       flags, s, ev);
      if (e != LK_OK) return e;
      LK_HIP(hipStreamSynchronize(s));
      float k = 0.f;
      LK_HIP(hipEventElapsedTime(&k, ev[0], ev[1]));
      if (r == 0) {
        if (k > 50.f) reps = 1;  // long calls: one timed repetition after the warm-up
        continue;
      }
      best = std::min(best, (double)k);
    }
    ++evaluated;
    *ms = best;
    return LK_OK;
  };
  double cur_ms = 0.0;
  if ((st = measure(cur, &cur_ms)) != LK_OK) return st;
  const double start_ms = cur_ms;

  auto sweep = [&](int32_t lk_tuning::*field, std::initializer_list<int32_t> values) -> lk_status {
    for (int32_t v : values) {
      if (cur.*field == v) continue;
      lk_tuning t = cur;
      t.*field = v;
      double ms = 0.0;
      lk_status e = measure(t, &ms);
      if (e != LK_OK) return e;
      if (ms < cur_ms * 0.99) {  // keep a change only for a clear gain
        cur = t;
        cur_ms = ms;
      }
    }
    return LK_OK;
  };
  if (crossings) {
    if ((st = sweep(&lk_tuning::segs_per_lane, {2, 4, 8})) != LK_OK) return st;
  } else if (mixed) {
    // segments per lane and the arctangent's instruction order interact (the
    // compiler schedules each variant differently): sweep one, the other, and
    // the first again
    if ((st = sweep(&lk_tuning::segs_per_lane, {1, 2, 4})) != LK_OK) return st;
    if ((st = sweep(&lk_tuning::atan_form, {0, 2})) != LK_OK) return st;
    if ((st = sweep(&lk_tuning::segs_per_lane, {1, 2, 4})) != LK_OK) return st;
  } else {
    // FP64: at two segments per lane a batch of one small pair is slow while
    // one segment per lane barely depends on it, so a start from batch 1
    // (left by an FP32 tuning) would settle on one segment: sweep the batch
    // first
    if (n_small > 0 && (st = sweep(&lk_tuning::small_batch, {1, 2, 4, 8})) != LK_OK) return st;
    if ((st = sweep(&lk_tuning::segs_per_lane_f64, {1, 2})) != LK_OK) return st;
  }
  if (n_small > 0 && (st = sweep(&lk_tuning::small_batch, {1, 2, 4, 8, 16, 32})) != LK_OK) return st;
  if (n_big > 0) {
    if (mixed) {
      if ((st = sweep(&lk_tuning::tile_a, {256, 512, 1024})) != LK_OK) return st;
    } else {
      if ((st = sweep(&lk_tuning::tile_a, {128, 256, 512})) != LK_OK) return st;
    }
    if (crossings) {
      // culling makes an item's cost its overlapping blocks, not its size
      if ((st = sweep(&lk_tuning::chunk_a, {4096, 16384, 65536, 262144, 1048576})) != LK_OK)
        return st;
    } else if ((st = sweep(&lk_tuning::chunk_a, {1024, 2048, 4096, 8192, 16384})) != LK_OK) {
      return st;
    }
    if (mixed && !crossings) {
      // the arctangent form was chosen at the starting chunk; the best form
      // can change with the chunk (big pairs walk longer per item), so it is
      // swept again, and the chunk with it when the form changes
      const int32_t form = cur.atan_form;
      if ((st = sweep(&lk_tuning::atan_form, {0, 2})) != LK_OK) return st;
      if (cur.atan_form != form &&
          (st = sweep(&lk_tuning::chunk_a, {1024, 2048, 4096, 8192, 16384})) != LK_OK)
        return st;
    }
  }
  if ((st = sweep(&lk_tuning::waves_per_cu, {0, 8, 12})) != LK_OK) return st;

  cur.best_ms = cur_ms;
  cur.start_ms = start_ms;
  cur.evaluated = evaluated;
  apply(cur);
  // leave the outputs as a valid result of the chosen configuration
  {
    const Plan P = make_plan(ctx, in_f64, mode, n_pairs);
    if ((st = enqueue_direct_sum(ctx, ctx_ws(ctx), P, xyz, off, n_loops, pairs, n_pairs, lk_real, lk_int,
                                 flags, s, nullptr)) != LK_OK)
      return st;
    LK_HIP(hipStreamSynchronize(s));
  }
  if (cache_path) {
    std::ofstream o(cache_path, std::ios::app);
    o << key << " " << cur.segs_per_lane << " " << cur.segs_per_lane_f64 << " " << cur.tile_a
      << " " << cur.chunk_a << " " << cur.small_batch << " " << cur.waves_per_cu << " "
      << cur.best_ms << " " << cur.start_ms << " " << cur.atan_form << "\n";
  }
  *out = cur;
  return LK_OK;
}

}  // extern "C"


// ------------------------------------------- runtime internals for the server
namespace lk {

int64_t ctx_workspace_bytes(const lk_ctx* ctx) {
  const DevBuf* bufs[] = {&ctx->loop_flags, &ctx->minseg2, &ctx->xi,       &ctx->recs,
                          &ctx->big_prefix, &ctx->meta,    &ctx->acc,      &ctx->flags,
                          &ctx->refit_list, &ctx->boxes,   &ctx->vcounts,  &ctx->vprefix,
                          &ctx->cc_blk,     &ctx->cc_sup,  &ctx->bh_nodes, &ctx->bh_lists,
                          &ctx->bh_counts,  &ctx->bh_adapt, &ctx->pls_grid};
  int64_t b = 0;
  for (const DevBuf* d : bufs) b += (int64_t)d->bytes;
  return b;
}

int64_t ctx_workspace_need(int mode, int32_t n_loops, int64_t n_pairs, int64_t n_vertices,
                           int64_t n_verify) {
  const double L = (double)n_loops, P = (double)n_pairs, V = (double)n_vertices;
  // the direct sum's own arrays (ensure_workspace) and its flags
  double b = 12.0 * L + 8.0 * (kPrepMaxBlocks + 1) + 3.0 * sizeof(WorkRec) * P + 8.0 * (P + 1) +
             (double)kMetaBytes + 16.0 * P + 8.0 * P + 4.0 * P;
  // the pair search: boxes, counts, prefix, and the grid (buckets <= 8 L)
  b += 48.0 * L + 8.0 * L + 8.0 * (L + 1) + (n_loops >= 2048 ? 192.0 * L + 4096.0 : 0.0);
  // verification's flags and prefix over current + expected pairs
  b += 16.0 * (double)(n_verify + 1);
  if (mode == LK_CROSSINGS)
    b += 16.0 * (V / kCcBlock + L + 1) + 16.0 * (V / kCcSuper + L + 1);
  if (mode == LK_BARNES_HUT) {
    const BhLayout Y = bh_layout(n_vertices, n_loops, n_pairs);
    b += (double)sizeof(BhNode) * (double)Y.nodes +
         (double)sizeof(BhPair) * (double)(2 * Y.list_cap + Y.near_cap) + 24.0 * (P + 1) +
         4.0 * (kBhMaxIters + 3);
  }
  return (int64_t)(1.25 * b);  // ensure() allocates a quarter more than asked
}

void ctx_forget_offsets(lk_ctx* ctx) {
  ctx->cc_off_key = nullptr;
  ctx->cc_loops_key = -1;
  ctx->cc_vertices = 0;
}

}  // namespace lk
