// lk_internal.h -- declarations shared by the HIP translation units of liblk.so.
// Kernels live in lk_ds.hip (the direct-sum hot loop) and lk_aux.hip (planning,
// scheduling, validation, reduction, pair search, verification);
// lk_runtime.hip holds the C ABI.
#pragma once
#include <hip/hip_runtime.h>
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

// Inputs of the planning step.
struct PlanArgs {
  const int64_t* off;          // loop offsets [n_loops + 1]
  const int32_t* pairs;        // [n_pairs][2]
  const int32_t* list;         // optional: pair index per list position (NULL = identity)
  const int32_t* n_list_dev;   // optional: list length on the device (NULL = n_list)
  int64_t n_list;              // list length (upper bound when n_list_dev is set)
  unsigned long long* acc;     // per-pair 128-bit fixed-point sums [n_pairs][2]
  uint32_t* flags;             // per-pair flags [n_pairs]
  int32_t chunk;               // vertices of loop A per work item
  int32_t bblock;              // segments of loop B per work item (64 x segments per lane)
};

// Inputs of one direct-sum pass.
struct DsArgs {
  const void* xyz;             // vertices, float or double, [V][3]
  Sched s;
  unsigned long long* acc;     // per-pair 128-bit fixed-point sums [n_pairs][2]
  uint32_t* flags;             // per-pair flags [n_pairs]
  int32_t tile;                // LDS tile of loop A, vertices
  int32_t chunk;               // vertices of loop A per work item (multiple of tile)
  int32_t batch;               // small pairs per work index
};

// --- lk_ds.hip
// in_f64: input dtype; compute_f64: arithmetic (true = plain FP64 / refit);
// atan_form: 0 = own minimax FP32 arctangent, 1 = HIP atan2f; segs: segments of
// loop B per lane (register blocking; rounded down to a built variant).
hipError_t launch_direct_sum(const DsArgs& a, bool in_f64, bool compute_f64, int atan_form,
                             int segs, int grid, hipStream_t s);
// Largest co-resident grid for the persistent kernel on this device.
int direct_sum_grid(bool in_f64, bool compute_f64, int atan_form, int segs, int tile, int n_cu,
                    int waves_per_cu);
// Segments per lane of the variant that `segs` selects.
int segs_supported(bool compute_f64, int segs);

// --- lk_aux.hip
constexpr int kXiBlocks = 256;
// xi = mean |coordinate| over vertices [off[0], off[n_loops]); writes loop flags.
// Also zeroes the given schedule counts (start of a call).
hipError_t launch_loop_flags(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                             double* xi_partials /*[kXiBlocks]*/, double* xi,
                             uint32_t* loop_flags, int32_t* zero_counts, hipStream_t s);

// Per list position: validate the pair, merge loop flags, zero its accumulator,
// count its work items and append its record to the small or big list.
// refit = true: REFIT-pass semantics (keeps flags, clears NONFINITE).
hipError_t launch_plan(const PlanArgs& a, int32_t n_loops, const uint32_t* loop_flags,
                       const Sched& s, bool refit, hipStream_t s_);
// Sort the big list (largest first), scan its items, set big_total, zero the
// work counter and (optionally) three int32 of the next pass: its two
// schedule counts and the refit count that follows them in memory.
hipError_t launch_sched(const Sched& s, int32_t* zero_counts_next, hipStream_t st);

// Convert sums to outputs.  refit_list/refit_n: if non-NULL (main MIXED pass),
// pairs with |frac| > thr or a non-finite value are appended.  refit_pass: the
// list being finalised is the refit list (sets LK_FLAG_REFIT).
hipError_t launch_finalize(const PlanArgs& a, double thr, double* lk_real, int32_t* lk_int,
                           int32_t* refit_list, int32_t* refit_n, bool refit_pass,
                           hipStream_t s);

// Exclusive scan of counts[0..n) into prefix[0..n] (single workgroup).
hipError_t launch_scan(const int64_t* counts, int64_t n, int64_t* prefix, hipStream_t s);

// Potential link search.
hipError_t launch_boxes(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                        double* boxes /*[n_loops][6]*/, hipStream_t s);
hipError_t launch_pair_count(const double* boxes, int32_t n_loops, int64_t* counts,
                             hipStream_t s);
hipError_t launch_pair_fill(const double* boxes, int32_t n_loops, const int64_t* row_start,
                            int32_t* pairs_out, int64_t capacity, hipStream_t s);

// Verification: per merged position, mismatch flags, then a scan and a scatter.
hipError_t launch_verify(const int32_t* pairs, const int32_t* lk, int64_t n,
                         const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                         int64_t* mism_counts /*[n + n_exp]*/, hipStream_t s);
hipError_t launch_verify_scatter(const int32_t* pairs, const int32_t* lk, int64_t n,
                                 const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                                 const int64_t* mism_prefix, int32_t* out, int64_t cap,
                                 hipStream_t s);

}  // namespace lk
