// lk_internal.h -- declarations shared by the HIP translation units of liblk.so.
// Kernels live in lk_ds.hip (the direct-sum and crossing-count hot loop, and
// the Barnes-Hut leaf pairs), lk_aux.hip (planning, scheduling, validation,
// reduction, pair search, verification), lk_bh.hip (Barnes-Hut trees and
// traversal) and lk_dz.hip (discretization, declared in lk_dz.h);
// lk_runtime.hip holds the C ABI and lk_server.hip the verification server.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace lk {

constexpr int kWave = 64;            // CDNA wavefront width; one wave per work item
constexpr int kMaxTileF32 = 1024;    // largest FP32 LDS tile of loop A (vertices)
constexpr int kMaxTileF64 = 512;     // largest FP64 LDS tile
constexpr int kSmallA = 128;         // small pairs: loop A has fewer segments than this
constexpr double kInvTwoPi = 0.15915494309189533577;

// One loop pair as the direct-sum kernel sees it: resolved offsets and sizes
// plus its number of work items (chunks of A x blocks of 64 R segments of B,
// R = segments per lane).
struct WorkRec {
  int64_t oa, ob;  // first vertex of loop A (gamma_1) and loop B (gamma_2)
  int32_t na, nb;  // vertex (= segment) counts
  int32_t p;       // index into the caller's pair arrays
  int32_t items;   // work items of this pair
};

// Device-side schedule of one pass.  Pairs with one work item and loop A
// shorter than kSmallA go to `small` in any order; all others go to `big`,
// sorted by item count, largest first (longest-processing-time order), with
// an exclusive prefix of items.  Work index w < big_total is item w of the big
// pairs; w >= big_total is the batch of `batch` small pairs starting at
// (w - big_total) * batch.  All counts are device values.
struct Sched {
  WorkRec* small;               // [cap]
  WorkRec* big_in;              // [cap] unsorted (filled by plan)
  WorkRec* big;                 // [cap] sorted (filled by sched)
  int64_t* big_prefix;          // [cap + 1]
  int32_t* counts;              // [0] = n_small, [1] = n_big
  int64_t* big_total;           // items of all big pairs
  unsigned long long* counter;  // work counter
};

// Where a pass writes its per-pair results (finalisation happens in the
// planning kernel for pairs without work, in the direct-sum kernel for pairs
// of one work item and in a short kernel after it for pairs of several).
struct Outs {
  double* lk_real;             // [n_pairs]
  int32_t* lk_int;             // [n_pairs]
  uint32_t* flags;             // [n_pairs]
  int32_t* refit_list;         // main MIXED pass: pairs queued for the FP64 refit (else NULL)
  int32_t* refit_n;            // its length
  double thr;                  // |v - round(v)| above this queues (main) or flags AMBIGUOUS
  int32_t refit_pass;          // 1: the pass over the refit list (sets LK_FLAG_REFIT)
  // fused check (NULL expected: none): final integers are compared with
  // expected[p]; mismatches are counted, and with early_exit the first one
  // sets *stop, which the kernels poll before taking new work
  const int32_t* expected;
  unsigned long long* n_mismatch;
  int32_t* stop;
  int32_t early_exit;
};

// Culling of the crossing count (Alg. 4 bounds its search with a BVH over
// projected segments; here the hierarchy is implicit in the vertex order).
// Loop i's vertex block k holds vertices kCcBlock k .. kCcBlock k + m
// (m = min(kCcBlock, n - kCcBlock k), cyclic: the last vertex closes the
// block's last segment); its projected box sits at slot
// (off[i] - off[0]) / kCcBlock + i + k.  Superblock s covers blocks
// kCcSuper / kCcBlock s .. + (kCcSuper / kCcBlock - 1) at slot
// (off[i] - off[0]) / kCcSuper + i + s.  A box is {min, max} of x . e1 then
// {min, max} of x . e2, e1 and e2 spanning the plane orthogonal to the view
// direction; two disjoint boxes hold no crossing.
constexpr int kCcBlock = 64;
constexpr int kCcSuper = 64 * 64;

__device__ __forceinline__ bool boxes_disjoint(const float4& a, const float4& b) {
  // NaN compares false: such boxes never cull
  return a.y < b.x || b.y < a.x || a.w < b.z || b.w < a.z;
}

// Per-loop validation results of the preparation kernel.
struct LoopInfo {
  const uint32_t* lf;          // NONFINITE / BADLOOP bits known without xi [n_loops]
  const double* minseg2;       // shortest squared segment length [n_loops]
  const double* part;          // partial sums of |coordinate| [n_part]
  int32_t n_part;
  double eps;                  // machine epsilon of the input dtype
};

// Inputs of the planning step.
struct PlanArgs {
  const int64_t* off;          // loop offsets [n_loops + 1]
  const int32_t* pairs;        // [n_pairs][2]
  const int32_t* list;         // optional: pair index per list position (NULL = identity)
  const int32_t* n_list_dev;   // optional: list length on the device (NULL = n_list)
  int64_t n_list;              // list length (upper bound when n_list_dev is set)
  unsigned long long* acc;     // per-pair 128-bit fixed-point sums [n_pairs][2]
  int32_t chunk;               // vertices of loop A per work item
  int32_t bblock;              // segments of loop B per work item (64 x segments per lane)
  const float4* cc_sup;        // crossing count: superblock boxes (NULL: no pair culling)
  int64_t cc_nsup;             // their slots (a slot beyond never culls)
  Outs out;
};

// Inputs of one direct-sum pass.
struct DsArgs {
  const void* xyz;             // vertices, float or double, [V][3]
  Sched s;
  unsigned long long* acc;     // per-pair 128-bit fixed-point sums [n_pairs][2]
  int32_t tile;                // LDS tile of loop A, vertices
  int32_t chunk;               // vertices of loop A per work item (multiple of tile)
  int32_t batch;               // small pairs per work index
  // crossing count only: view direction (|n|_inf = 1) and the certainty
  // factors of the side predicates and of the crossing sign
  float view[3];
  float cc_tau, cc_tau_p;
  const float4* cc_blk;        // block and superblock boxes (NULL: no culling)
  const float4* cc_sup;
  int64_t cc_nblk, cc_nsup;    // their slots (a slot beyond never culls)
  const int32_t* pairs;        // the call's pair list (loop indices for the box slots)
  const int64_t* off;          // loop offsets (off[0] anchors the box slots)
  Outs out;
};

constexpr uint32_t kFlagRefit = 1u, kFlagAmbiguous = 2u, kFlagNonfinite = 4u, kFlagBadpair = 8u,
                   kFlagBadloop = 16u, kFlagSkipped = 32u;
constexpr uint32_t kFlagUncertified = kFlagNonfinite | kFlagAmbiguous | kFlagBadpair | kFlagBadloop;

// Fused check of one final pair (see Outs).
__device__ __forceinline__ void check_pair(const Outs& o, int32_t p, int32_t value, uint32_t f) {
  if (!o.expected) return;
  if ((f & kFlagUncertified) || value != o.expected[p]) {
    atomicAdd(o.n_mismatch, 1ull);
    if (o.early_exit) atomicExch(o.stop, 1);
  }
}
constexpr int32_t kIntInvalid = INT32_MIN;

// Rounds and flags one pair's value and writes its outputs (a6 of the path):
// round half away from zero; a value farther than `thr` from its integer, or a
// non-finite one, goes to the refit list in the main MIXED pass and is flagged
// AMBIGUOUS (or NONFINITE) otherwise.  Called by one lane per pair.
__device__ __forceinline__ void finalize_pair(const Outs& o, int32_t p, double v, uint32_t f) {
  bool requeue = false;
  f &= ~kFlagSkipped;
  if (o.refit_pass) f |= kFlagRefit;
  double real;
  int32_t ival;
  const bool bad = (f & kFlagNonfinite) || !isfinite(v) || fabs(v) > 2.0e9;
  if (bad) {
    f |= kFlagNonfinite;
    real = __builtin_nan("");
    ival = kIntInvalid;
    requeue = o.refit_list != nullptr;
  } else {
    const double r = round(v);  // half away from zero
    real = v;
    ival = (int32_t)r;
    if (fabs(v - r) > o.thr) {
      if (o.refit_list)
        requeue = true;
      else
        f |= kFlagAmbiguous;
    }
  }
  if (requeue && o.expected) {
    // a fused check leaves the pair undecided (SKIPPED, no value) until the
    // FP64 refit finalises it
    real = __builtin_nan("");
    ival = kIntInvalid;
    f |= kFlagSkipped;
  }
  o.lk_real[p] = real;
  o.lk_int[p] = ival;
  o.flags[p] = f;
  if (requeue)
    o.refit_list[atomicAdd(o.refit_n, 1)] = p;
  else
    check_pair(o, p, ival, f);
}

// 128-bit two's-complement fixed point with 64 fraction bits, accumulated with
// 64-bit integer atomics: integer addition is associative, so the pair sum is
// the same whatever order the work items finish in.  The conversion is exact
// except for bits below 2^-64, which are dropped by an arithmetic shift (always
// towards -infinity, so deterministically).  |v| < 2^50 is required.
__device__ __forceinline__ void to_fixed(double v, unsigned long long& lo, unsigned long long& hi) {
  lo = 0ull;
  hi = 0ull;
  if (v == 0.0) return;
  int e = 0;
  const double f = frexp(v, &e);                   // v = f 2^e, 0.5 <= |f| < 1
  const long long m = (long long)ldexp(f, 53);     // exact: |m| < 2^53
  const int s = e + 11;                            // v 2^64 = m 2^s
  if (s > 0) {
    lo = (unsigned long long)m << s;
    hi = (unsigned long long)(m >> (64 - s));
  } else if (s == 0) {
    lo = (unsigned long long)m;
    hi = m < 0 ? ~0ull : 0ull;
  } else if (s > -64) {
    const long long t = m >> (-s);
    lo = (unsigned long long)t;
    hi = t < 0 ? ~0ull : 0ull;
  } else {
    lo = m < 0 ? ~0ull : 0ull;
    hi = lo;
  }
}

__device__ __forceinline__ void fixed_add(unsigned long long* acc, double v) {
  unsigned long long lo, hi;
  to_fixed(v, lo, hi);
  if (lo == 0ull && hi == 0ull) return;
  const unsigned long long old = atomicAdd(&acc[0], lo);
  const unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
  atomicAdd(&acc[1], hi + carry);
}

// 128-bit two's complement -> sign and magnitude -> double (one rounding of
// the fraction word, one of the sum).
__device__ __forceinline__ double from_fixed(unsigned long long lo, unsigned long long hi) {
  const bool neg = (long long)hi < 0;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  const double mag = (double)hi + (double)lo * 5.421010862427522170e-20;  // 2^-64
  return neg ? -mag : mag;
}

// --- Barnes-Hut (Sec. 3.4.4, Alg. 6): lk_bh.hip, and the leaf pairs in lk_ds.hip
// Trees over consecutive segments: a leaf holds kBhLeaf segments of a loop, a
// node of level h holds kBhLeaf * kBhArity^h (the last one of a level fewer)
// and its children are the level h - 1 nodes inside it; a loop's root is its
// lowest level with a single node.  Node k of level h of loop i sits at slot
// level_base[h] + (off[i] - off[0]) / span_h + i + k (span_h = kBhLeaf *
// kBhArity^h), which leaves room for every loop without a prefix sum.
constexpr int kBhLeaf = 64;
constexpr int kBhArity = 8;
constexpr int kBhMaxLevels = 10;
constexpr int kBhMaxIters = 2 * kBhMaxLevels;

// Box centre and half extents (R = |e|, half the box diagonal), and the
// moments about the centre: c_M, C_D[p][b], C_Q[p][b][c] (row-major).
struct BhNode {
  double c[3], e[3];
  double M[3], D[9], Q[27];
};

// One pair of tree nodes of one loop pair: node ka of level ha of loop A
// (gamma_1) against node kb of level hb of loop B.
struct BhPair {
  int32_t p, ka, kb, lev;  // lev = ha | hb << 8
};

struct BhArgs {
  const void* xyz;
  const int64_t* off;
  const int32_t* pairs;
  int32_t n_loops;
  BhNode* nodes;
  int64_t level_base[kBhMaxLevels];  // first slot of each level
  int64_t level_cap[kBhMaxLevels];   // slots of each level (a slot beyond fails the pair)
  int32_t levels;                    // levels built
  BhPair* list[2];                   // ping-pong node-pair lists
  BhPair* near;                      // leaf pairs for the direct sum
  int64_t list_cap, near_cap;
  int32_t* counts;                   // [kBhMaxIters + 3]: list entries per iteration, near
                                     // pairs, pairs evaluated again at a larger beta
  unsigned long long* acc;           // per-pair fixed point [n_pairs][2]
  // adaptive beta (Sec. 3.4.4): the first traversal sums each pair's
  // next-order error estimate into est (fixed point [n_pairs][2]); the second
  // traverses only the pairs with beta_p[p] > 0, at that beta.  Both NULL for
  // a fixed beta.
  unsigned long long* est;
  double* beta_p;
  uint32_t* lf;                      // per-loop validation, folded in by the leaf kernel
  double* minseg2;                   //   (the preparation kernel only initialises it)
  double beta;
  int32_t order;
  Outs out;
};

__device__ __forceinline__ int64_t bh_span(int h) {
  int64_t s = kBhLeaf;
  for (int q = 0; q < h; ++q) s *= kBhArity;
  return s;
}
__device__ __forceinline__ int64_t bh_count(int64_t n, int h) {
  const int64_t s = bh_span(h);
  return (n + s - 1) / s;
}

// Tree build (one launch for the leaves, one per level above).
hipError_t launch_bh_leaves(const BhArgs& a, bool in_f64, hipStream_t s);
hipError_t launch_bh_level(const BhArgs& a, int level, hipStream_t s);
// After the planning kernel (validation, flags, zeroed accumulators): push
// the root pair of every pair that has work.
hipError_t launch_bh_roots(const BhArgs& a, int64_t n_pairs, hipStream_t s);
// One breadth-first step: node pairs of list iteration `it`.
hipError_t launch_bh_expand(const BhArgs& a, int it, hipStream_t s);
// Eq. 4 over every leaf pair of the near list (FP32 terms, FP64 sums).
hipError_t launch_bh_near(const BhArgs& a, bool in_f64, hipStream_t s);
// Round and flag every pair that has work (refit list as in the mixed mode).
hipError_t launch_bh_finalize(const BhArgs& a, int64_t n_pairs, hipStream_t s);
// Adaptive beta, between the two traversals: beta_t = (E / target)^(1/4) beta
// per pair; pairs with beta_t > beta get beta_p = min(beta_t, beta_max) and a
// cleared accumulator, the others beta_p = 0; the lists start empty again.
hipError_t launch_bh_adapt(const BhArgs& a, int64_t n_pairs, double target, double beta_max,
                           hipStream_t s);

// --- lk_ds.hip
// in_f64: input dtype; compute_f64: arithmetic (true = plain FP64 / refit);
// form (FP32 only): 0 / 2 = own minimax arctangent (phased / inline), 1 = HIP
// atan2f, 3 = crossing count instead of the Eq. 4 sum; segs: segments of loop
// B per lane (register blocking; rounded down to a built variant).
// unpacked: every small pair on a whole wave (the layout for calls with few
// pairs; the crossing count and R = 1 ignore it).
hipError_t launch_direct_sum(const DsArgs& a, bool in_f64, bool compute_f64, int atan_form,
                             int segs, int grid, hipStream_t s, bool unpacked = false);
// Largest co-resident grid for the persistent kernel on this device.
int direct_sum_grid(bool in_f64, bool compute_f64, int atan_form, int segs, int tile, int n_cu,
                    int waves_per_cu, bool unpacked = false);
// Segments per lane of the variant that `segs` selects (the crossing count
// also has 8).
int segs_supported(bool compute_f64, int segs, bool crossings = false);

// --- lk_aux.hip
constexpr int kXiBlocks = 256;        // least workgroups of the preparation kernel
constexpr int kPrepMaxBlocks = 4096;  // most workgroups (xi partials buffer size)
// Workgroups of the preparation kernel for n_loops loops (= xi partials).
int prep_blocks(int32_t n_loops, int64_t n_vertices = 0);
// xi partial sums (one per workgroup) and, one wavefront per loop, the loop's
// NONFINITE / <3-vertex bits and shortest squared segment; zeroes the main
// pass's two schedule counts and (when given) the fused check's mismatch
// count and stop flag.
// Crossing count: block and superblock boxes of every loop (see kCcBlock)
// for the slots below n_blk / n_sup (the rest are not written), and the
// per-loop validation of the preparation kernel (lf, minseg2, which a
// preparation launched without its loop scan has initialised).
struct CcProj {
  float e1[3], e2[3];  // directions spanning the plane orthogonal to the view
};
hipError_t launch_cc_boxes(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                           const CcProj& pr, float4* blk, int64_t n_blk, float4* sup,
                           int64_t n_sup, uint32_t* lf, double* minseg2, hipStream_t s);
hipError_t launch_prep(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                       double* xi_partials /*[prep_blocks]*/, uint32_t* lf, double* minseg2,
                       int32_t* zero_counts, unsigned long long* zero_mismatch,
                       int32_t* zero_stop, bool scan_loops, int n_blocks /*prep_blocks*/,
                       hipStream_t s);
// Per list position: validate the pair, apply the zero-length test (xi from
// the partials), zero its accumulator, count its work items and append its
// record to the small or big list; pairs without work are finalised here.
// refit = true: REFIT-pass semantics (keeps flags, clears NONFINITE).
hipError_t launch_plan(const PlanArgs& a, int32_t n_loops, const LoopInfo& li, const Sched& s,
                       bool refit, hipStream_t st);
// After the direct-sum kernel: finalise the pairs of the big list that were
// split over several work items (128-bit fixed point -> FP64, round, flag).
hipError_t launch_finalize_split(const Sched& s, const unsigned long long* acc, const Outs& o,
                                 int64_t n_pairs, hipStream_t st);
// Sort the big list (largest first), scan its items, set big_total, zero the
// work counter and (optionally) three int32 of the next pass: its two
// schedule counts and the refit count that follows them in memory.
hipError_t launch_sched(const Sched& s, int32_t* zero_counts_next, hipStream_t st);
// prep, plan (main pass) and sched as one single-workgroup launch, for calls
// with few pairs; the per-loop scan runs on 16 wavefronts.
hipError_t launch_prep_plan(const void* xyz, bool in_f64, const PlanArgs& a, int32_t n_loops,
                            const LoopInfo& li, uint32_t* lf, double* minseg2, const Sched& sc,
                            unsigned long long* zero_mismatch, int32_t* zero_stop,
                            int32_t* zero_counts_next, hipStream_t st);
// finalize_split of one pass, then the plan (refit semantics, list and its
// length on the device) and the schedule of the next, as one single-workgroup
// launch.
hipError_t launch_finalize_replan(const Sched& s, const unsigned long long* acc, const Outs& o,
                                  const PlanArgs& r, int32_t n_loops, const LoopInfo& li,
                                  const Sched& sr, int32_t* zero_counts_next, hipStream_t st);
// *p = 0 with a kernel (safe inside a captured sequence).
hipError_t launch_zero_i64(int64_t* p, hipStream_t s);
// Exclusive scan of counts[0..n) into prefix[0..n] (single workgroup).
hipError_t launch_scan(const int64_t* counts, int64_t n, int64_t* prefix, hipStream_t s);
// Potential link search.
hipError_t launch_boxes(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                        double* boxes /*[n_loops][6]*/, hipStream_t s);
hipError_t launch_pair_count(const double* boxes, int32_t n_loops, int64_t* counts,
                             hipStream_t s);
hipError_t launch_pair_fill(const double* boxes, int32_t n_loops, const int64_t* row_start,
                            int32_t* pairs_out, int64_t capacity, hipStream_t s);

// Potential link search on a hashed grid of the boxes' min corners (see
// grid_stats_k): the same pairs as launch_pair_count / launch_pair_fill in
// about L x (boxes in 27 buckets) tests instead of L^2 / 2.
struct GridParams {
  double h;         // cell size; boxes with every side at most h / 2 are binned
  double lo[3];     // grid origin
  int64_t buckets;  // hash table size (a power of two)
};
struct GridBufs {
  GridParams* params;
  unsigned long long* cell_count;  // [buckets] (int64 counts)
  int64_t* cell_start;             // [buckets + 1]
  int64_t* cell_of;                // [L] bucket, -1 for a box tested against all
  int32_t* cell_items;             // [L]
  double* cell_box;                // [L][6] the boxes in bucket order
  int32_t* over;                   // [L]
  int32_t* n_over;
  int64_t* row_counts;             // [L]
  double* part;                    // [kGridStatBlocks][6] per-workgroup partials
  int64_t* tiles;                  // [2 (buckets / 4096 + 2)] tile sums and offsets
  int64_t buckets;
};
constexpr int kGridStatBlocks = 64;
// pass 0: grid, binning, per-row counts into row_counts; pass 1 (after the
// caller's scan of the counts into row_start): fill and sort the rows.
hipError_t launch_grid_pairs(const double* boxes, int32_t n_loops, const GridBufs& b, int pass,
                             const int64_t* row_start, int32_t* pairs_out, hipStream_t s);

// Verification: per merged position, mismatch flags, then a scan and a scatter.
hipError_t launch_verify(const int32_t* pairs, const int32_t* lk, int64_t n,
                         const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                         int64_t* mism_counts /*[n + n_exp]*/, hipStream_t s);
hipError_t launch_verify_scatter(const int32_t* pairs, const int32_t* lk, int64_t n,
                                 const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                                 const int64_t* mism_prefix, int32_t* out, int64_t cap,
                                 hipStream_t s);

}  // namespace lk

// Runtime internals the verification server uses (lk_runtime.hip).
struct lk_ctx;
namespace lk {
// Device bytes the context's workspace holds now.
int64_t ctx_workspace_bytes(const lk_ctx* ctx);
// Device bytes a context's workspace may grow to for one request in `mode`
// (pair search, direct sum and verification of n_verify entries).
int64_t ctx_workspace_need(int mode, int32_t n_loops, int64_t n_pairs, int64_t n_vertices,
                           int64_t n_verify);
// Drop the cached vertex count of the last offsets array (the next CROSSINGS
// or BARNES_HUT call reads and validates it again).
void ctx_forget_offsets(lk_ctx* ctx);
}  // namespace lk
