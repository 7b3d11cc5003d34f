// lk_dz.hip -- adaptive discretization of closed curves (Sec. 3.3, Alg. 3).
//
// Every input span (a uniform cubic B-spline span, or a polyline segment) is
// a cubic Bezier piece.  Pieces stay in each loop's parameter order in one
// array, so the output polyline is the pieces' start points and no sort is
// needed.  One pass of Alg. 3 is a fixed sequence of launches:
//   boxes   one wavefront per group of 64 consecutive unprocessed pieces of a
//           loop: the pieces' control-point boxes (the curve lies in their
//           convex hull) and the group's box; clears the pieces' marks;
//   items   a device scan over the candidate pairs of the number of groups on
//           the side with more groups: work item = (pair, group);
//   test    one wavefront per item: its 64 pieces against every group of the
//           other loop whose box overlaps; overlapping piece boxes mark both
//           pieces under-refined (plain stores of 1, so order is irrelevant);
//   split   a device scan over all pieces of (pieces out, unprocessed out):
//           final pieces are copied, unmarked unprocessed pieces become
//           final, marked pieces are replaced by their two de Casteljau
//           halves at t = 1/2, which form the next unprocessed list.  The
//           ordered array carries only start points, loops and states; the
//           control points live in the compact unprocessed list, so a final
//           piece costs 32 bytes per pass instead of 104;
//   offsets the per-loop offsets of the new array and list.
// The host reads the new counts after each pass (one synchronisation) and
// sizes the next launches from them.  Arithmetic is FP64 without fused
// multiply-adds, so every piece is bitwise the one the plain definition gives.
#include "lk_dz.h"

#pragma clang fp contract(off)

namespace lk {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int o) {
  const uint32_t lo = (uint32_t)__shfl_up((int)(uint32_t)v, o);
  const uint32_t hi = (uint32_t)__shfl_up((int)(uint32_t)(v >> 32), o);
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int o) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, o);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), o);
  return ((uint64_t)hi << 32) | lo;
}

// Exclusive scan over the block (blockDim.x a multiple of 64, at most 1024);
// *total receives the block's sum.
__device__ uint64_t block_excl_scan(uint64_t v, uint64_t* total) {
  __shared__ uint64_t wsum[16];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = shfl_up_u64(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint64_t off = 0, tot = 0;
  for (int k = 0; k < nw; ++k) {
    if (k < w) off += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();  // wsum is reused by the next call
  *total = tot;
  return off + x - v;
}

__device__ uint64_t block_sum(uint64_t v) {
  uint64_t t;
  block_excl_scan(v, &t);
  return t;
}

// Exclusive scan of part[0, nb) in place (one block of 1024 threads); the sum
// goes to *total.
__global__ __launch_bounds__(1024) void dz_scan_part_k(uint64_t* part, int64_t nb,
                                                       uint64_t* total, int64_t* total_i64) {
  uint64_t carry = 0;
  for (int64_t base = 0; base < nb; base += blockDim.x) {
    const int64_t i = base + threadIdx.x;
    const uint64_t v = i < nb ? part[i] : 0;
    uint64_t t;
    const uint64_t e = block_excl_scan(v, &t);
    if (i < nb) part[i] = carry + e;
    carry += t;
  }
  if (threadIdx.x == 0) {
    if (total) *total = carry;
    if (total_i64) *total_i64 = (int64_t)carry;
  }
}

__device__ __forceinline__ int64_t dz_groups(int64_t n) { return (n + kDzGroup - 1) / kDzGroup; }

// Slot of group g of loop i: (uoff[i] / 64) + i + g never collides with the
// next loop's slots and needs no prefix sum.
__device__ __forceinline__ int64_t dz_slot(const int64_t* uoff, int32_t i, int64_t g) {
  return uoff[i] / kDzGroup + i + g;
}

// Largest i in [0, n) with key(i) <= x, for a non-decreasing key with
// key(0) <= x and a wave-uniform x: the wavefront probes 64 evenly spaced
// keys per step (the lanes that pass form a prefix), so a search over n
// entries takes log64(n) dependent loads instead of log2(n).
template <typename Key>
__device__ __forceinline__ int64_t wave_search(int64_t n, int64_t x, Key key) {
  const int lane = threadIdx.x & 63;
  int64_t lo = 0, hi = n;
  while (hi - lo > 1) {
    const int64_t step = (hi - lo + 63) / 64;
    const int64_t idx = lo + lane * step;
    const uint64_t m = __ballot(idx < hi && key(idx) <= x);
    lo += (int64_t)(63 - __builtin_clzll(m)) * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  return lo;
}

// Largest loop i with uoff[i] / 64 + i <= slot.
__device__ __forceinline__ int32_t dz_slot_loop(const int64_t* uoff, int32_t L, int64_t slot) {
  return (int32_t)wave_search(L, slot, [&](int64_t i) { return uoff[i] / kDzGroup + i; });
}

// Squared diagonal of the box of four points (min/max in point order, then
// dx*dx + dy*dy + dz*dz).
__device__ __forceinline__ double diag2(const double (&b)[4][3]) {
  double d[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    double lo = b[0][q], hi = b[0][q];
#pragma unroll
    for (int k = 1; k < 4; ++k) {
      lo = b[k][q] < lo ? b[k][q] : lo;
      hi = b[k][q] > hi ? b[k][q] : hi;
    }
    d[q] = hi - lo;
  }
  return d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
}

// Control points of unprocessed piece u.
__device__ __forceinline__ void load_open(const double* ubz, int64_t cap, int64_t u,
                                          double (&b)[4][3]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int q = 0; q < 3; ++q) b[k][q] = ubz[(3 * k + q) * cap + u];
}

__device__ __forceinline__ void store_open(double* ubz, int64_t cap, int64_t u,
                                           const double (&b)[4][3]) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int q = 0; q < 3; ++q) ubz[(3 * k + q) * cap + u] = b[k][q];
}

// Entry i of the ordered array: start point, loop, state.
__device__ __forceinline__ void store_piece(const DzPieces& P, int64_t i, const double* x0,
                                            int32_t loop, uint32_t state) {
#pragma unroll
  for (int q = 0; q < 3; ++q) P.start[q * P.cap + i] = x0[q];
  P.loop[i] = loop;
  P.state[i] = state;
}

// Halves of the parameter domain: de Casteljau at t = 1/2, or the midpoint
// of a linear piece (points 0 = 1 and 2 = 3).
__device__ __forceinline__ void split_half(const double (&x)[4][3], bool linear, double (&l)[4][3],
                                           double (&r)[4][3]) {
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    if (linear) {
      const double m = 0.5 * (x[0][q] + x[3][q]);
      l[0][q] = x[0][q];
      l[1][q] = x[0][q];
      l[2][q] = m;
      l[3][q] = m;
      r[0][q] = m;
      r[1][q] = m;
      r[2][q] = x[3][q];
      r[3][q] = x[3][q];
      continue;
    }
    const double m01 = 0.5 * (x[0][q] + x[1][q]);
    const double m12 = 0.5 * (x[1][q] + x[2][q]);
    const double m23 = 0.5 * (x[2][q] + x[3][q]);
    const double m012 = 0.5 * (m01 + m12);
    const double m123 = 0.5 * (m12 + m23);
    const double m = 0.5 * (m012 + m123);
    l[0][q] = x[0][q];
    l[1][q] = m01;
    l[2][q] = m012;
    l[3][q] = m;
    r[0][q] = m;
    r[1][q] = m123;
    r[2][q] = m23;
    r[3][q] = x[3][q];
  }
}

struct Box {
  double lo[3], hi[3];
};

__device__ __forceinline__ Box empty_box() {
  Box b;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    b.lo[q] = INFINITY;
    b.hi[q] = -INFINITY;
  }
  return b;
}

__device__ __forceinline__ Box load_box(const double* B, int64_t cap, int64_t i) {
  Box b;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    b.lo[q] = B[q * cap + i];
    b.hi[q] = B[(3 + q) * cap + i];
  }
  return b;
}

// Closed intervals on all three axes.
__device__ __forceinline__ bool overlap(const Box& a, const Box& b) {
  return a.lo[0] <= b.hi[0] && b.lo[0] <= a.hi[0] && a.lo[1] <= b.hi[1] && b.lo[1] <= a.hi[1] &&
         a.lo[2] <= b.hi[2] && b.lo[2] <= a.hi[2];
}

__device__ __forceinline__ Box shfl_box(const Box& b, int src) {
  Box r;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    r.lo[q] = __shfl(b.lo[q], src);
    r.hi[q] = __shfl(b.hi[q], src);
  }
  return r;
}

// ---------------------------------------------------------------- set-up
// One wavefront per loop: sum of |coordinate| (for xi), fewer than 3 points
// or a non-finite coordinate (invalid loop), and the loop's piece offsets.
__global__ __launch_bounds__(kThreads) void dz_loops_k(DzArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kThreads) >> 6;
  const int64_t o0 = A.cp_off[0];
  for (int64_t i = wave; i < A.n_loops; i += nwaves) {
    const int64_t o = A.cp_off[i], m = A.cp_off[i + 1] - o;
    double s = 0.0;
    int bad = 0;
    for (int64_t c = lane; c < 3 * m; c += 64) {
      const double x = A.ctrl[3 * o + c];
      s += fabs(x);
      bad |= !isfinite(x);
    }
#pragma unroll
    for (int w = 32; w > 0; w >>= 1) {
      s += __shfl_xor(s, w);
      bad |= __shfl_xor(bad, w);
    }
    if (lane == 0) {
      A.lsum[i] = s;
      A.lflags[i] = (m < 3 || bad) ? kFlagBadloop : 0u;
      A.aoff_cur[i] = o - o0;
      A.uoff_cur[i] = o - o0;
      if (i == A.n_loops - 1) {
        A.aoff_cur[i + 1] = A.cp_off[i + 1] - o0;
        A.uoff_cur[i + 1] = A.cp_off[i + 1] - o0;
      }
    }
  }
}

// Offsets that decrease anywhere: *bad = 1 (the host rejects the call
// before any kernel indexes with them).
__global__ __launch_bounds__(kThreads) void dz_check_offsets_k(const int64_t* off, int32_t L,
                                                               int32_t* bad) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < L;
       i += (int64_t)gridDim.x * kThreads)
    if (off[i + 1] < off[i]) *bad = 1;
}

// xi = mean over the points of (|x| + |y| + |z|) / 3; lim2 = (eps * xi)^2.
__global__ __launch_bounds__(1024) void dz_xi_k(DzArgs A) {
  __shared__ double red[1024];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < A.n_loops; i += blockDim.x) s += A.lsum[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x >> 1; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t n = A.cp_off[A.n_loops] - A.cp_off[0];
    const double xi = n > 0 ? red[0] / (3.0 * (double)n) : 0.0;
    const double lim = A.eps * xi;
    A.lim2[0] = lim * lim;
  }
}

// One thread per input span: its Bezier piece, the zero-length test of
// Alg. 3, and the first unprocessed list (every piece).
__global__ __launch_bounds__(kThreads) void dz_init_k(DzArgs A, int64_t n_points) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q >= n_points) return;
  const int64_t o0 = A.cp_off[0];
  int32_t lo = 0, hi = A.n_loops;  // largest loop with cp_off[i] - o0 <= q
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (A.cp_off[mid] - o0 <= q)
      lo = mid;
    else
      hi = mid;
  }
  const int32_t i = lo;
  const int64_t o = A.cp_off[i] - o0, m = A.cp_off[i + 1] - A.cp_off[i];
  const int64_t s = q - o;
  const double* q1 = A.ctrl + 3 * (o0 + o + s);
  const double* q2 = A.ctrl + 3 * (o0 + o + (s + 1) % m);
  double b[4][3];
  if (A.kind == 1) {
    for (int c = 0; c < 3; ++c) {
      b[0][c] = q1[c];
      b[1][c] = q1[c];
      b[2][c] = q2[c];
      b[3][c] = q2[c];
    }
  } else {
    const double* q0 = A.ctrl + 3 * (o0 + o + (s + m - 1) % m);
    const double* q3 = A.ctrl + 3 * (o0 + o + (s + 2) % m);
    for (int c = 0; c < 3; ++c) {
      b[0][c] = (q0[c] + 4.0 * q1[c] + q2[c]) / 6.0;
      b[1][c] = (2.0 * q1[c] + q2[c]) / 3.0;
      b[2][c] = (q1[c] + 2.0 * q2[c]) / 3.0;
      b[3][c] = (q1[c] + 4.0 * q2[c] + q3[c]) / 6.0;
    }
  }
  store_piece(A.cur, q, b[0], i, (uint32_t)q);
  store_open(A.ubz_cur, A.cap_o, q, b);
  if (diag2(b) < A.lim2[0]) atomicOr(&A.lflags[i], kFlagBadloop);
}

// ------------------------------------------------------------------ pass
// One wavefront per group slot: boxes of its unprocessed pieces (stored in
// list order) and of the group; clears the pieces' marks.
__global__ __launch_bounds__(kThreads) void dz_boxes_k(DzArgs A, int64_t n_slots) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kThreads) >> 6;
  for (int64_t slot = wave; slot < n_slots; slot += nwaves) {
    const int32_t i = dz_slot_loop(A.uoff_cur, A.n_loops, slot);
    const int64_t u0 = A.uoff_cur[i], nu = A.uoff_cur[i + 1] - u0;
    const int64_t g = slot - (u0 / kDzGroup + i);
    Box bx = empty_box();
    if (g < dz_groups(nu)) {
      const int64_t u = u0 + g * kDzGroup + lane;
      if (u < u0 + nu) {
        double b[4][3];
        load_open(A.ubz_cur, A.cap_o, u, b);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          double lo = b[0][q], hi = b[0][q];
#pragma unroll
          for (int k = 1; k < 4; ++k) {
            lo = b[k][q] < lo ? b[k][q] : lo;
            hi = b[k][q] > hi ? b[k][q] : hi;
          }
          bx.lo[q] = lo;
          bx.hi[q] = hi;
          A.pbox[q * A.cap_u + u] = lo;
          A.pbox[(3 + q) * A.cap_u + u] = hi;
        }
        A.mark[u] = 0u;
      }
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
      for (int w = 32; w > 0; w >>= 1) {
        bx.lo[q] = fmin(bx.lo[q], __shfl_xor(bx.lo[q], w));
        bx.hi[q] = fmax(bx.hi[q], __shfl_xor(bx.hi[q], w));
      }
    if (lane == 0) {
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        A.gbox[q * A.cap_g + slot] = bx.lo[q];
        A.gbox[(3 + q) * A.cap_g + slot] = bx.hi[q];
      }
    }
  }
}

// Pair p as (a, b) with a the loop of more groups; 0 items if the pair is
// invalid, names an invalid loop, or a side has no unprocessed piece.
__device__ __forceinline__ int64_t pair_items(const DzArgs& A, int64_t p, int32_t* pa,
                                              int32_t* pb) {
  int32_t i = A.pairs[2 * p], j = A.pairs[2 * p + 1];
  if (i < 0 || j < 0 || i >= A.n_loops || j >= A.n_loops || i == j) return 0;
  if ((A.lflags[i] | A.lflags[j]) & kFlagBadloop) return 0;
  const int64_t gi = dz_groups(A.uoff_cur[i + 1] - A.uoff_cur[i]);
  const int64_t gj = dz_groups(A.uoff_cur[j + 1] - A.uoff_cur[j]);
  if (gi == 0 || gj == 0) return 0;
  if (gj > gi) {
    const int32_t t = i;
    i = j;
    j = t;
  }
  *pa = i;
  *pb = j;
  return gj > gi ? gj : gi;
}

__global__ __launch_bounds__(kThreads) void dz_items_reduce_k(DzArgs A) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int32_t a, b;
  const uint64_t v = p < A.n_pairs ? (uint64_t)pair_items(A, p, &a, &b) : 0;
  const uint64_t t = block_sum(v);
  if (threadIdx.x == 0) A.part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void dz_items_apply_k(DzArgs A) {
  const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  int32_t a = 0, b = 0;
  const uint64_t v = p < A.n_pairs ? (uint64_t)pair_items(A, p, &a, &b) : 0;
  uint64_t t;
  const uint64_t e = block_excl_scan(v, &t) + A.part[blockIdx.x];
  if (p < A.n_pairs) {
    A.pair_pre[p] = (int64_t)e;
    A.pair_ab[2 * p] = a;
    A.pair_ab[2 * p + 1] = b;
  }
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const int64_t v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(v & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ Box readlane_box(const Box& b, int l) {
  Box r;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    r.lo[q] = readlane_d(b.lo[q], l);
    r.hi[q] = readlane_d(b.hi[q], l);
  }
  return r;
}

// One wavefront per (pair, group of a): lane t holds piece t of the group;
// the groups of b whose boxes overlap the group's box are visited in turn,
// and inside them only the pieces of b whose boxes overlap it, each broadcast
// from its lane.  A wavefront takes a contiguous run of items, so it finds
// its first pair by one search and then steps through the prefix.
__global__ __launch_bounds__(kThreads) void dz_test_k(DzArgs A) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * kThreads) >> 6;
  const int64_t P = A.n_pairs;
  const int64_t total = P > 0 ? A.pair_pre[P] : 0;
  const int64_t chunk = (total + nwaves - 1) / nwaves;
  const int64_t w0 = wave * chunk;
  const int64_t w1 = w0 + chunk < total ? w0 + chunk : total;
  if (w0 >= w1) return;
  int64_t p = wave_search(P, w0, [&](int64_t i) { return A.pair_pre[i]; });
  for (int64_t w = w0; w < w1; ++w) {
    while (A.pair_pre[p + 1] <= w) ++p;  // pair_pre[P] = total > w
    const int32_t a = A.pair_ab[2 * p], b = A.pair_ab[2 * p + 1];
    const int64_t ga = w - A.pair_pre[p];
    const int64_t ua0 = A.uoff_cur[a] + ga * kDzGroup;
    const int64_t ua_end = A.uoff_cur[a + 1];
    const bool has_a = ua0 + lane < ua_end;
    const Box pa = has_a ? load_box(A.pbox, A.cap_u, ua0 + lane) : empty_box();
    const Box gA = load_box(A.gbox, A.cap_g, dz_slot(A.uoff_cur, a, ga));
    const int64_t ub_begin = A.uoff_cur[b], ub_end = A.uoff_cur[b + 1];
    const int64_t ngb = dz_groups(ub_end - ub_begin);
    const int64_t sb0 = dz_slot(A.uoff_cur, b, 0);
    bool ma = false;
    for (int64_t c0 = 0; c0 < ngb; c0 += 64) {
      const int64_t gb = c0 + lane;
      const bool gok = gb < ngb && overlap(load_box(A.gbox, A.cap_g, sb0 + gb), gA);
      uint64_t gm = __ballot(gok);
      while (gm) {
        const int k = __builtin_ctzll(gm);
        gm &= gm - 1;
        const int64_t ub0 = ub_begin + (c0 + k) * kDzGroup;
        const bool has_b = ub0 + lane < ub_end;
        const Box pb = has_b ? load_box(A.pbox, A.cap_u, ub0 + lane) : empty_box();
        uint64_t bm = __ballot(has_b && overlap(pb, gA));
        uint64_t hit = 0;  // b pieces that some a piece overlaps
        while (bm) {
          const int kk = __builtin_ctzll(bm);
          bm &= bm - 1;
          const Box bk = readlane_box(pb, kk);
          const bool ov = has_a && overlap(pa, bk);
          ma |= ov;
          if (__ballot(ov) != 0) hit |= 1ull << kk;
        }
        if ((hit >> lane) & 1ull) A.mark[ub0 + lane] = 1u;
      }
    }
    if (ma) A.mark[ua0 + lane] = 1u;
  }
}

// (pieces out << 32) | (unprocessed out) of piece q; the halves of a marked
// piece are computed here and again when written (same arithmetic).
__device__ __forceinline__ uint64_t split_value(const DzArgs& A, int64_t q, bool* marked,
                                                bool* flagged, double (&l)[4][3],
                                                double (&r)[4][3]) {
  *marked = false;
  *flagged = false;
  if (q >= A.n) return 0;
  const uint32_t st = A.cur.state[q];
  if (st == kDzFinal || A.mark[st] == 0u) return 1ull << 32;
  *marked = true;
  double x[4][3];
  load_open(A.ubz_cur, A.cap_o, st, x);
  split_half(x, A.kind == 1, l, r);
  const double lim2 = A.lim2[0];
  *flagged = diag2(l) < lim2 || diag2(r) < lim2;
  return (2ull << 32) | (*flagged ? 0ull : 2ull);
}

__global__ __launch_bounds__(kThreads) void dz_split_reduce_k(DzArgs A) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  bool mk, fl;
  double l[4][3], r[4][3];
  const uint64_t v = split_value(A, q, &mk, &fl, l, r);
  const uint64_t t = block_sum(v);
  if (threadIdx.x == 0) A.part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void dz_split_apply_k(DzArgs A) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  bool mk, fl;
  double l[4][3], r[4][3];
  const uint64_t v = split_value(A, q, &mk, &fl, l, r);
  uint64_t t;
  const uint64_t e = block_excl_scan(v, &t) + A.part[blockIdx.x];
  if (q >= A.n) return;
  A.pre[q] = e;
  const int64_t np = (int64_t)(e >> 32), nu = (int64_t)(e & 0xffffffffull);
  const int32_t loop = A.cur.loop[q];
  if (!mk) {
    double x0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) x0[c] = A.cur.start[c * A.cur.cap + q];
    store_piece(A.nxt, np, x0, loop, kDzFinal);
    return;
  }
  store_piece(A.nxt, np, l[0], loop, fl ? kDzFinal : (uint32_t)nu);
  store_piece(A.nxt, np + 1, r[0], loop, fl ? kDzFinal : (uint32_t)(nu + 1));
  if (fl) {
    atomicOr(&A.lflags[loop], kFlagIntersect);
  } else {
    store_open(A.ubz_nxt, A.cap_on, nu, l);
    store_open(A.ubz_nxt, A.cap_on, nu + 1, r);
  }
}

__global__ __launch_bounds__(kThreads) void dz_offsets_k(DzArgs A) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i > A.n_loops) return;
  const int64_t q = A.aoff_cur[i];
  const uint64_t e = q < A.n ? A.pre[q] : A.totals[0];
  A.aoff_nxt[i] = (int64_t)(e >> 32);
  A.uoff_nxt[i] = (int64_t)(e & 0xffffffffull);
}

// ---------------------------------------------------------------- finish
__global__ __launch_bounds__(kThreads) void dz_leftover_k(DzArgs A) {
  const int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (q < A.n && A.cur.state[q] != kDzFinal) atomicOr(&A.lflags[A.cur.loop[q]], kFlagIntersect);
}

__global__ __launch_bounds__(kThreads) void dz_output_k(DzArgs A, double* xyz, int64_t capacity,
                                                        int64_t* off, uint32_t* flags) {
  const int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (v < A.n && A.n <= capacity) {
#pragma unroll
    for (int q = 0; q < 3; ++q) xyz[3 * v + q] = A.cur.start[q * A.cur.cap + v];
  }
  if (v <= A.n_loops) off[v] = A.aoff_cur[v];
  if (flags && v < A.n_loops) flags[v] = A.lflags[v];
}

int64_t blocks_for(int64_t n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

hipError_t launch_dz_check(const int64_t* off, int32_t n_loops, int32_t* bad, hipStream_t s) {
  const int64_t b = blocks_for(n_loops);
  dz_check_offsets_k<<<(unsigned)(b < 4096 ? b : 4096), kThreads, 0, s>>>(off, n_loops, bad);
  return hipGetLastError();
}

hipError_t launch_dz_setup(const DzArgs& a, int64_t n_points, hipStream_t s) {
  const int64_t lb = (a.n_loops + 3) / 4;
  dz_loops_k<<<(unsigned)(lb < 4096 ? lb : 4096), kThreads, 0, s>>>(a);
  dz_xi_k<<<1, 1024, 0, s>>>(a);
  if (n_points > 0) dz_init_k<<<(unsigned)blocks_for(n_points), kThreads, 0, s>>>(a, n_points);
  return hipGetLastError();
}

hipError_t launch_dz_pass(const DzArgs& a, int n_cu, hipStream_t s) {
  const int64_t n_slots = a.n_u / kDzGroup + a.n_loops + 1;
  const int64_t bb = (n_slots + 3) / 4;
  dz_boxes_k<<<(unsigned)(bb < 8192 ? bb : 8192), kThreads, 0, s>>>(a, n_slots);
  const int64_t pb = blocks_for(a.n_pairs);
  if (pb > 0) {
    dz_items_reduce_k<<<(unsigned)pb, kThreads, 0, s>>>(a);
    dz_scan_part_k<<<1, 1024, 0, s>>>(a.part, pb, nullptr, a.pair_pre + a.n_pairs);
    dz_items_apply_k<<<(unsigned)pb, kThreads, 0, s>>>(a);
    dz_test_k<<<(unsigned)(32 * n_cu), kThreads, 0, s>>>(a);
  }
  const int64_t qb = blocks_for(a.n);
  dz_split_reduce_k<<<(unsigned)qb, kThreads, 0, s>>>(a);
  dz_scan_part_k<<<1, 1024, 0, s>>>(a.part, qb, a.totals, nullptr);
  dz_split_apply_k<<<(unsigned)qb, kThreads, 0, s>>>(a);
  dz_offsets_k<<<(unsigned)blocks_for(a.n_loops + 1), kThreads, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_dz_finish(const DzArgs& a, double* xyz_out, int64_t capacity, int64_t* off_out,
                            uint32_t* flags_out, hipStream_t s) {
  if (a.n_u > 0) dz_leftover_k<<<(unsigned)blocks_for(a.n), kThreads, 0, s>>>(a);
  const int64_t m = (a.n > a.n_loops + 1 ? a.n : a.n_loops + 1);
  dz_output_k<<<(unsigned)blocks_for(m), kThreads, 0, s>>>(a, xyz_out, capacity, off_out,
                                                            flags_out);
  return hipGetLastError();
}

}  // namespace lk
