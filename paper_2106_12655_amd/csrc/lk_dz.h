// lk_dz.h -- declarations of the discretization (Sec. 3.3, Alg. 3) shared by
// lk_dz.hip (kernels) and lk_runtime.hip (the pass loop of lk_discretize).
#pragma once
#include "lk_internal.h"

namespace lk {

// Pieces are cubic Bezier curves kept in each loop's parameter order.  The
// ordered array holds what every piece needs: its start point (3 planes of
// FP64), owning loop and state (kDzFinal, or the piece's position in the
// unprocessed list).  The unprocessed list holds the four control points of
// each unprocessed piece (12 planes: point k, coordinate q in plane 3k + q).
// Every plane of an array is `cap` entries long.
constexpr int kDzGroup = 64;           // unprocessed pieces per group box (one wavefront)
constexpr int kDzScanBlock = 256;      // elements per block of the device scans
constexpr uint32_t kFlagIntersect = 64u;
constexpr uint32_t kDzFinal = 0xffffffffu;
constexpr int kDzBytesPerPiece = 3 * 8 + 4 + 4;
constexpr int kDzBytesPerOpen = 12 * 8;

struct DzPieces {
  double* start;    // [3][cap]
  int32_t* loop;    // [cap]
  uint32_t* state;  // [cap]
  int64_t cap;
};

struct DzArgs {
  const double* ctrl;      // input points [N][3]
  const int64_t* cp_off;   // [L+1]
  int32_t n_loops;
  int32_t kind;            // 0: uniform cubic B-spline control points, 1: polyline vertices
  const int32_t* pairs;    // [P][2]
  int64_t n_pairs;
  double eps;
  DzPieces cur, nxt;
  double* ubz_cur;         // [12][cap_o] control points of the unprocessed pieces
  double* ubz_nxt;
  int64_t cap_o, cap_on;   // plane lengths of ubz_cur and ubz_nxt
  int64_t *aoff_cur, *aoff_nxt;  // [L+1] piece offsets per loop
  int64_t *uoff_cur, *uoff_nxt;  // [L+1] offsets into the unprocessed list
  double* pbox;            // [6][cap_u] boxes of the unprocessed pieces (lo xyz, hi xyz)
  int64_t cap_u;
  double* gbox;            // [6][cap_g] group boxes by slot
  int64_t cap_g;
  uint32_t* mark;          // [n_u] under-refined marks, by list position
  uint64_t* pre;           // [cur.cap] packed exclusive prefix of the split
  int64_t* pair_pre;       // [P+1] exclusive prefix of work items per pair
  int32_t* pair_ab;        // [P][2] the pair as (a, b), a the side of more groups
  uint64_t* part;          // scan partials, one per block
  uint64_t* totals;        // [0] packed (pieces << 32 | unprocessed) after the split
  uint32_t* lflags;        // [L]
  double* lsum;            // [L] sums of |coordinate| per loop
  double* lim2;            // [1] (eps * xi)^2
  int64_t n, n_u;          // pieces and unprocessed pieces of cur (host copies)
};

// *bad (device int32, set to 0 by the caller) becomes 1 if the offsets decrease.
hipError_t launch_dz_check(const int64_t* off, int32_t n_loops, int32_t* bad, hipStream_t s);
hipError_t launch_dz_setup(const DzArgs& a, int64_t n_points, hipStream_t s);
hipError_t launch_dz_pass(const DzArgs& a, int n_cu, hipStream_t s);
hipError_t launch_dz_finish(const DzArgs& a, double* xyz_out, int64_t capacity,
                            int64_t* off_out, uint32_t* flags_out, hipStream_t s);

}  // namespace lk
