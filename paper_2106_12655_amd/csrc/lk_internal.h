// lk_internal.h -- declarations shared by the HIP translation units of liblk.so.
// Kernels live in lk_ds.hip (the direct-sum hot loop) and lk_aux.hip (planning,
// validation, reduction, pair search, verification); lk_runtime.hip holds the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lk {

constexpr int kWave = 64;            // CDNA wavefront width; one wave per work item
constexpr int kBlockB = 64;          // B segments per work item (one per lane)
constexpr int kMaxTileF32 = 1024;    // largest FP32 LDS tile of loop A (vertices)
constexpr int kMaxTileF64 = 512;     // largest FP64 LDS tile
constexpr double kInvTwoPi = 0.15915494309189533577;

// Parameters of one direct-sum pass over a list of pairs.
struct DsArgs {
  const void* xyz;             // vertices, float or double, [V][3]
  const int64_t* off;          // loop offsets [n_loops + 1]
  const int32_t* pairs;        // [n_pairs][2]
  const int32_t* list;         // optional: pair index per list position (NULL = identity)
  const int32_t* n_list_dev;   // optional: list length on the device (NULL = n_list)
  int64_t n_list;              // list length (upper bound when n_list_dev is set)
  const int64_t* prefix;       // work items before each list position [n_list + 1]
  unsigned long long* counter; // work counter (zeroed by the scan kernel)
  unsigned long long* acc;     // per-pair 128-bit fixed-point sums [n_pairs][2]
  uint32_t* flags;             // per-pair flags [n_pairs]
  int32_t tile;                // LDS tile of loop A, vertices
  int32_t chunk;               // vertices of loop A per work item (multiple of tile)
};

// --- lk_ds.hip
// in_f64: input dtype; compute_f64: arithmetic (true = plain FP64 / refit);
// atan_form: 0 = own minimax FP32 arctangent, 1 = HIP atan2f.
hipError_t launch_direct_sum(const DsArgs& a, bool in_f64, bool compute_f64, int atan_form,
                             int grid, hipStream_t s);
// Largest co-resident grid for the persistent kernel on this device.
int direct_sum_grid(bool in_f64, bool compute_f64, int atan_form, int tile, int n_cu,
                    int waves_per_cu);

// --- lk_aux.hip
// xi = mean |coordinate| over vertices [off[0], off[n_loops]); writes loop flags.
hipError_t launch_loop_flags(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                             double* xi_partials /*[kXiBlocks]*/, double* xi,
                             uint32_t* loop_flags, hipStream_t s);
constexpr int kXiBlocks = 256;

// Per list position: validate the pair, merge loop flags, zero its accumulator,
// count its work items (tile/chunk rule).  refit = true keeps REFIT-pass
// semantics (clears NONFINITE, reads the list length from n_list_dev).
hipError_t launch_plan(const DsArgs& a, int32_t n_loops, const uint32_t* loop_flags,
                       int64_t* counts, bool refit, hipStream_t s);
// Exclusive scan of counts[0..n) into prefix[0..n] and zero the work counter.
hipError_t launch_scan(const int64_t* counts, const int32_t* n_dev, int64_t n, int64_t* prefix,
                       unsigned long long* counter, hipStream_t s);
// Same, and also zeroes *zero_i32 (the refit count of the following finalize).
hipError_t launch_scan_zero(const int64_t* counts, const int32_t* n_dev, int64_t n,
                            int64_t* prefix, unsigned long long* counter, int32_t* zero_i32,
                            hipStream_t s);
// Convert sums to outputs.  refit_list/refit_n: if non-NULL (main MIXED pass),
// pairs with |frac| > thr or a non-finite value are appended.  refit_pass: the
// list being finalised is the refit list (sets LK_FLAG_REFIT).
hipError_t launch_finalize(const DsArgs& a, double thr, double* lk_real, int32_t* lk_int,
                           int32_t* refit_list, int32_t* refit_n, bool refit_pass,
                           hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n, hipStream_t s);

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
