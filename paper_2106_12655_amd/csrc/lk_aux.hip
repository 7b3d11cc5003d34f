// lk_aux.hip -- everything around the direct-sum hot loop: input validation,
// work planning with its device-side schedule, the potential link search
// (Alg. 2) and the verification merge (Sec. 3.1, "Fast Verification").
//
// All sizes that depend on the data (work item totals, the refit count) stay in
// device memory, so every launch here has a host-known shape and the whole
// sequence can be captured in a HIP graph.  No kernel uses float atomics: all
// reductions have a fixed order, and results are bitwise reproducible.
#include <float.h>
#include <math.h>

#include "lk_internal.h"

namespace lk {
namespace {

inline int blocks_for(int64_t n, int threads, int cap = 65535 * 8) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// ------------------------------------------------------------- validation
// Sum of one value per thread of a 256-thread workgroup (a fixed-order tree),
// stored at part[blockIdx.x].
__device__ __forceinline__ void block_sum_to(double v, double* red, double* part) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One wavefront per loop: the per-loop bits that do not depend on xi (fewer
// than 3 vertices, non-finite coordinates), each loop's shortest squared
// segment, and one xi partial sum of |coordinate| per workgroup over the
// vertices of its loops.  The zero-length test of Alg. 3 (segment shorter
// than eps * xi) is applied by the plan, which reduces the partials to xi
// itself.  When the crossing count's box kernel does the per-loop scan, this
// kernel sums xi over a flat grid stride and only initialises the per-loop
// entries.  Block 0 also zeroes the main pass's schedule counts.
// One wavefront's scan of loop l: its flags that do not depend on xi (fewer
// than 3 vertices, non-finite coordinates) and its shortest squared segment,
// written by lane 0; returns the lane's sum of |x| + |y| + |z| over the
// vertices it read.
// W: lanes per loop (a power of two up to 64, aligned within the wavefront;
// every lane of the group calls it).
template <typename Tin, int W = 64>
__device__ double scan_loop(const Tin* X, const int64_t* off, int64_t l, int lane, uint32_t* lf,
                            double* minseg2) {
  double s = 0.0;
  const int64_t o = off[l], n = off[l + 1] - o;
  uint32_t f = (n < 3) ? kFlagBadloop : 0u;
  double mn = INFINITY;
  for (int64_t q = lane; q < n; q += W) {
    const int64_t t = (q + 1 == n) ? 0 : q + 1;
    const double x0 = (double)X[3 * (o + q)], y0 = (double)X[3 * (o + q) + 1],
                 z0 = (double)X[3 * (o + q) + 2];
    const double x1 = (double)X[3 * (o + t)], y1 = (double)X[3 * (o + t) + 1],
                 z1 = (double)X[3 * (o + t) + 2];
    if (!isfinite(x0) || !isfinite(y0) || !isfinite(z0)) f |= kFlagNonfinite | kFlagBadloop;
    s += fabs(x0) + fabs(y0) + fabs(z0);
    const double dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
    mn = fmin(mn, dx * dx + dy * dy + dz * dz);
  }
  for (int o2 = W / 2; o2 > 0; o2 >>= 1) {
    f |= (uint32_t)__shfl_xor((int)f, o2);
    mn = fmin(mn, __shfl_xor(mn, o2));
  }
  if (lane == 0) {
    lf[l] = f;
    minseg2[l] = mn;
  }
  return s;
}

template <typename Tin>
__global__ __launch_bounds__(256) void prep_k(const Tin* X, const int64_t* off, int32_t L,
                                              double* part, uint32_t* lf, double* minseg2,
                                              int32_t* zero_counts,
                                              unsigned long long* zero_mismatch,
                                              int32_t* zero_stop, int scan_loops) {
  __shared__ double red[256];
  if (blockIdx.x == 0 && threadIdx.x < 2) zero_counts[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0 && zero_mismatch) {
    *zero_mismatch = 0ull;
    *zero_stop = 0;
  }
  double s = 0.0;
  if (!scan_loops) {
    const int64_t v0 = off[0], v1 = off[L];
    const int64_t n3 = 3 * (v1 - v0);
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n3;
         k += (int64_t)gridDim.x * 256)
      s += fabs((double)X[3 * v0 + k]);
    block_sum_to(s, red, part);
    // the crossing count's box kernel scans the vertices (in parallel over
    // blocks of long loops) and folds its results into these with atomics
    for (int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x; l < L; l += (int64_t)gridDim.x * 256) {
      lf[l] = off[l + 1] - off[l] < 3 ? kFlagBadloop : 0u;
      minseg2[l] = INFINITY;
    }
    return;
  }
  // one pass over the loops: each vertex adds |x| + |y| + |z| to the xi
  // partial of the workgroup that scans its loop
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t l = wave; l < L; l += nwaves) s += scan_loop(X, off, l, lane, lf, minseg2);
  block_sum_to(s, red, part);
}

// ------------------------------------------------- crossing-count boxes
// One wavefront per superblock slot: the loop that owns the slot comes from a
// binary search over the slot bases, and the wave boxes the superblock's
// blocks one after another (lane t holds vertex 64k + t; lane 0 also the
// vertex that closes the block).  Coordinates are FP32 on the vertices as the
// crossing kernel sees them (FP64 input rounded first).  Each box is widened
// by 8 u (u = 2^-24) times the largest |x|_1 of its vertices, which covers the
// rounding of the two projections and the FP32 directions' deviation from
// exact orthogonality to the view direction.  The slot count comes from the
// device offsets, so every vertex is scanned whatever the buffers hold; boxes
// beyond the buffers are not written.
//
// The same scan does the per-loop validation of the preparation kernel (which
// then only initialises it): non-finite coordinates and the shortest squared
// segment, folded into the loop's entries with atomics (a minimum of
// non-negative doubles is a minimum of their bit patterns).
__device__ __forceinline__ float4 box_join(const float4& a, const float4& b) {
  return float4{fminf(a.x, b.x), fmaxf(a.y, b.y), fminf(a.z, b.z), fmaxf(a.w, b.w)};
}

template <typename Tin>
__global__ __launch_bounds__(256) void cc_boxes_k(const Tin* X, const int64_t* off, int32_t L,
                                                  CcProj pr, float4* blk, int64_t n_blk,
                                                  float4* sup, int64_t n_sup, uint32_t* lf,
                                                  double* minseg2) {
  const int lane = threadIdx.x & 63;
  const int64_t o0 = off[0];
  const int64_t n_slots = (off[L] - o0) / kCcSuper + L + 1;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t slot = wave; slot < n_slots; slot += nwaves) {
    // largest loop i with (off[i] - off[0]) / kCcSuper + i <= slot
    int32_t lo = 0, hi = L;
    while (hi - lo > 1) {
      const int32_t mid = (lo + hi) >> 1;
      if ((off[mid] - o0) / kCcSuper + mid <= slot)
        lo = mid;
      else
        hi = mid;
    }
    const int64_t oi = off[lo], n = off[lo + 1] - oi;
    const int64_t s = slot - ((oi - o0) / kCcSuper + lo);
    const int64_t nblk = n > 0 ? (n + kCcBlock - 1) / kCcBlock : 0;
    constexpr int64_t kPer = kCcSuper / kCcBlock;
    // slot not used by the loop, or offsets that decrease (uniform over the wave)
    if (n <= 0 || s < 0 || s * kPer >= nblk) continue;
    const int64_t bbase = (oi - o0) / kCcBlock + lo;
    float4 acc = float4{INFINITY, -INFINITY, INFINITY, -INFINITY};
    uint32_t f = 0u;
    double mn = INFINITY;
    const int64_t kend = (s + 1) * kPer < nblk ? (s + 1) * kPer : nblk;
    for (int64_t k = s * kPer; k < kend; ++k) {
      const int64_t v0 = k * kCcBlock;
      const int64_t m = (n - v0) < kCcBlock ? (n - v0) : kCcBlock;
      float a0 = INFINITY, a1 = -INFINITY, b0 = INFINITY, b1 = -INFINITY, mag = 0.0f;
      for (int t = lane; t <= m; t += 64) {  // m + 1 vertices: the last closes the block
        int64_t v = v0 + t;
        if (v >= n) v -= n;
        const Tin* p = X + 3 * (oi + v);
        const double x = (double)p[0], y = (double)p[1], z = (double)p[2];
        if (t < m) {
          // the loop's validation: vertex v and its segment to v + 1
          int64_t w = v + 1;
          if (w >= n) w -= n;
          const Tin* q = X + 3 * (oi + w);
          if (!isfinite(x) || !isfinite(y) || !isfinite(z)) f |= kFlagNonfinite | kFlagBadloop;
          const double dx = (double)q[0] - x, dy = (double)q[1] - y, dz = (double)q[2] - z;
          mn = fmin(mn, dx * dx + dy * dy + dz * dz);
        }
        const float xf = (float)x, yf = (float)y, zf = (float)z;
        const float a = fmaf(xf, pr.e1[0], fmaf(yf, pr.e1[1], zf * pr.e1[2]));
        const float b = fmaf(xf, pr.e2[0], fmaf(yf, pr.e2[1], zf * pr.e2[2]));
        a0 = fminf(a0, a);
        a1 = fmaxf(a1, a);
        b0 = fminf(b0, b);
        b1 = fmaxf(b1, b);
        mag = fmaxf(mag, fabsf(xf) + fabsf(yf) + fabsf(zf));
      }
      for (int o = 32; o > 0; o >>= 1) {
        a0 = fminf(a0, __shfl_xor(a0, o));
        a1 = fmaxf(a1, __shfl_xor(a1, o));
        b0 = fminf(b0, __shfl_xor(b0, o));
        b1 = fmaxf(b1, __shfl_xor(b1, o));
        mag = fmaxf(mag, __shfl_xor(mag, o));
      }
      const float pad = 4.76837158203125e-7f * mag;  // 8 * 2^-24
      const float4 box = float4{a0 - pad, a1 + pad, b0 - pad, b1 + pad};
      if (lane == 0 && (uint64_t)(bbase + k) < (uint64_t)n_blk) blk[bbase + k] = box;
      acc = box_join(acc, box);
    }
    for (int o = 32; o > 0; o >>= 1) {
      f |= (uint32_t)__shfl_xor((int)f, o);
      mn = fmin(mn, __shfl_xor(mn, o));
    }
    if (lane == 0) {
      if (slot < n_sup) sup[slot] = acc;
      if (f) atomicOr(&lf[lo], f);
      // the entry only decreases, so a plain read that is not above mn
      // makes the atomic unnecessary (thousands of blocks share one loop)
      if (mn < INFINITY && mn < minseg2[lo])
        atomicMin(reinterpret_cast<unsigned long long*>(&minseg2[lo]),
                  (unsigned long long)__double_as_longlong(mn));
    }
  }
}

// --------------------------------------------------------------- planning
// Workgroup-collective append to two lists at once: one atomic per list per
// workgroup (instead of one per wavefront), so the plan of tens of thousands
// of pairs does not queue thousands of atomics on two counters.  Every
// thread of the workgroup must call it; *pos0 / *pos1 receive the thread's
// slot in list 0 / 1 when it appends there.
__device__ __forceinline__ void block_append2(int32_t* count0, bool pred0, int32_t* pos0,
                                              int32_t* count1, bool pred1, int32_t* pos1) {
  __shared__ int32_t wn[2][16], base[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const unsigned long long m0 = __ballot(pred0), m1 = __ballot(pred1);
  if (lane == 0) {
    wn[0][w] = (int32_t)__popcll(m0);
    wn[1][w] = (int32_t)__popcll(m1);
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int k = threadIdx.x;
    int32_t t = 0;
    for (int q = 0; q < nw; ++q) t += wn[k][q];
    base[k] = t ? atomicAdd(k ? count1 : count0, t) : 0;
  }
  __syncthreads();
  int32_t b0 = base[0], b1 = base[1];
  for (int q = 0; q < w; ++q) {
    b0 += wn[0][q];
    b1 += wn[1][q];
  }
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  *pos0 = b0 + (int32_t)__popcll(m0 & below);
  *pos1 = b1 + (int32_t)__popcll(m1 & below);
  __syncthreads();  // wn and base are reused by the next call
}

// Exclusive scan of one value per thread over a 1024-thread workgroup
// (wavefront shuffles, then the 16 wave totals).  *total receives the sum.
__device__ int64_t block_excl_scan(int64_t v, int64_t* wsum, int64_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int64_t sw = lane < 16 ? wsum[lane] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int64_t y = __shfl_up(sw, o);
      if (lane >= o) sw += y;
    }
    if (lane < 16) wsum[lane] = sw;
  }
  __syncthreads();
  const int64_t before = wave ? wsum[wave - 1] : 0;
  *total = wsum[15];
  __syncthreads();
  return before + x - v;
}

// In-place-capable exclusive scan of src[0..n) into dst[0..n], dst[n] = total;
// 4 consecutive elements per thread per round, so loads are coalesced.
__device__ int64_t block_scan_array(const int64_t* src, int64_t n, int64_t* dst, int64_t* wsum) {
  const int t = threadIdx.x;
  int64_t carry = 0;
  for (int64_t base = 0; base < n; base += 4096) {
    const int64_t k0 = base + 4 * (int64_t)t;
    int64_t v[4];
    int64_t sum = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      v[i] = (k0 + i < n) ? src[k0 + i] : 0;
      sum += v[i];
    }
    int64_t tot = 0;
    int64_t run = carry + block_excl_scan(sum, wsum, &tot);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      if (k0 + i < n) dst[k0 + i] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (t == 0) dst[n] = carry;
  return carry;
}

__device__ __forceinline__ int cost_bucket(int32_t items) { return 31 - __clz(items); }

// One workgroup (1024 threads): bucket the big pairs by log2(items), largest
// bucket first (an LPT order up to a factor of two), then scan their items.
__device__ void schedule(const Sched& S, int32_t* zero_next) {
  __shared__ int hist[32];
  __shared__ int cur[32];
  __shared__ int64_t wsum[16];
  const int t = threadIdx.x;
  // a device-scope load: in the fused launch below the count was built by
  // atomics of the same kernel
  const int nb = __hip_atomic_load(&S.counts[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (t < 32) hist[t] = 0;
  __syncthreads();
  for (int k = t; k < nb; k += 1024) atomicAdd(&hist[cost_bucket(S.big_in[k].items)], 1);
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int b = 31; b >= 0; --b) {
      cur[b] = run;
      run += hist[b];
    }
  }
  __syncthreads();
  for (int k = t; k < nb; k += 1024) {
    const WorkRec r = S.big_in[k];
    const int pos = atomicAdd(&cur[cost_bucket(r.items)], 1);
    S.big[pos] = r;
    S.big_prefix[pos] = r.items;
  }
  __syncthreads();
  const int64_t total = block_scan_array(S.big_prefix, nb, S.big_prefix, wsum);
  if (t == 0) {
    *S.big_total = total;
    *S.counter = 0ull;
    if (zero_next) {
      zero_next[0] = 0;
      zero_next[1] = 0;
      zero_next[2] = 0;
    }
  }
}

// The plan's work over list positions base = first, first + stride, ...
// below n, one thread per position (every thread of the workgroup takes part:
// the appends are workgroup-collective, so n and the loop bounds must be the
// same in every thread).
__device__ void plan_positions(const PlanArgs& A, int32_t L, const LoopInfo& li, const Sched& S,
                               int refit, double xi, int64_t n, int64_t first, int64_t stride) {
  for (int64_t base = first; base < n; base += stride) {
    const int64_t q = base + threadIdx.x;
    bool small = false, big = false;
    WorkRec r{};
    if (q < n) {
      const int32_t p = A.list ? A.list[q] : (int32_t)q;
      const int32_t i = A.pairs[2 * p], j = A.pairs[2 * p + 1];
      const bool valid = i >= 0 && j >= 0 && i < L && j < L && i != j;
      int64_t items = 0;
      if (valid) {
        r.oa = A.off[i];
        r.ob = A.off[j];
        const int64_t na = A.off[i + 1] - r.oa, nb = A.off[j + 1] - r.ob;
        r.na = (int32_t)na;
        r.nb = (int32_t)nb;
        if (na >= 1 && nb >= 1)
          items = ((nb + A.bblock - 1) / A.bblock) * ((na + A.chunk - 1) / A.chunk);
      }
      // loops beyond 2^31 vertices or pairs beyond 2^31 work items are not handled
      const bool too_big = valid && (A.off[i + 1] - A.off[i] > 0x7fffffffLL ||
                                     A.off[j + 1] - A.off[j] > 0x7fffffffLL ||
                                     items > 0x7fffffffLL);
      if (too_big) items = 0;
      // crossing count: two loops of one superblock each whose projected
      // boxes are disjoint have no crossing, so the pair is 0 without work
      if (A.cc_sup && valid && !too_big && items > 0 && r.na <= kCcSuper && r.nb <= kCcSuper) {
        const int64_t o0 = A.off[0];
        const int64_t si = (r.oa - o0) / kCcSuper + i, sj = (r.ob - o0) / kCcSuper + j;
        if ((uint64_t)si < (uint64_t)A.cc_nsup && (uint64_t)sj < (uint64_t)A.cc_nsup &&
            boxes_disjoint(A.cc_sup[si], A.cc_sup[sj]))
          items = 0;
      }
      uint32_t f;
      if (refit) {
        // a non-finite value of the previous pass may become finite in FP64;
        // non-finite coordinates stay non-finite
        const uint32_t coords = valid ? (li.lf[i] | li.lf[j]) & kFlagNonfinite : 0u;
        f = (A.out.flags[p] & ~kFlagNonfinite) | coords | (too_big ? kFlagNonfinite : 0u);
      } else if (valid) {
        // Alg. 3's zero-length test: a segment shorter than eps * xi
        const double lim = li.eps * xi;
        const double lim2 = lim * lim;
        const uint32_t fi = li.lf[i] | (li.minseg2[i] < lim2 ? kFlagBadloop : 0u);
        const uint32_t fj = li.lf[j] | (li.minseg2[j] < lim2 ? kFlagBadloop : 0u);
        f = fi | fj | (too_big ? kFlagBadloop | kFlagNonfinite : 0u);
      } else {
        f = kFlagBadpair;
      }
      A.acc[2 * (int64_t)p] = 0ull;
      A.acc[2 * (int64_t)p + 1] = 0ull;
      r.p = p;
      r.items = (int32_t)items;
      small = items == 1 && r.na < kSmallA;
      big = items > 0 && !small;
      if (!valid) {
        A.out.flags[p] = f;
        A.out.lk_real[p] = __builtin_nan("");
        A.out.lk_int[p] = kIntInvalid;
        check_pair(A.out, p, kIntInvalid, f);
      } else if (items == 0) {
        // nothing to sum (an empty loop, or beyond the supported sizes)
        Outs o = A.out;
        o.refit_list = nullptr;
        finalize_pair(o, p, 0.0, f);
      } else {
        if (A.out.expected && !refit) {
          // a fused check marks every pair SKIPPED until it is finalised
          f |= kFlagSkipped;
          A.out.lk_real[p] = __builtin_nan("");
          A.out.lk_int[p] = kIntInvalid;
        }
        A.out.flags[p] = f;
      }
    }
    int32_t ps, pb;
    block_append2(&S.counts[0], small, &ps, &S.counts[1], big, &pb);
    if (small) S.small[ps] = r;
    if (big) S.big_in[pb] = r;
  }
}

// One thread per list position, 1024-thread workgroups.  The schedule is a
// separate single-workgroup launch: handing it to the plan's last workgroup
// (a fence and a ticket in every workgroup) measured slower on MI355X, where
// a device-scope fence writes back the XCD's L2.
__global__ __launch_bounds__(1024) void plan_k(PlanArgs A, int32_t L, LoopInfo li, Sched S,
                                               int refit) {
  // xi = mean |coordinate|: every block reduces the preparation kernel's
  // partials in the same fixed order (cheaper than another launch); a refit
  // pass validates nothing and skips it
  __shared__ double red[1024];
  double xi = 0.0;
  if (!refit) {
    double part = 0.0;
    for (int k = threadIdx.x; k < li.n_part; k += 1024) part += li.part[k];
    red[threadIdx.x] = part;
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    const int64_t nv = A.off[L] - A.off[0];
    xi = nv > 0 ? red[0] / (3.0 * (double)nv) : 0.0;
  }
  int64_t n = A.n_list;
  if (A.n_list_dev) {
    const int64_t nd = __hip_atomic_load(A.n_list_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    n = nd < n ? nd : n;
  }
  // grid stride over the list's length on the device (the same in every
  // thread), so an empty refit list costs each workgroup one load
  plan_positions(A, L, li, S, refit, xi, n, (int64_t)blockIdx.x * 1024, (int64_t)gridDim.x * 1024);
}

// Finalises the big-list pairs that were split over several work items,
// positions first, first + stride, ...
__device__ void finalize_split_range(const Sched& S, const unsigned long long* acc, const Outs& o,
                                     int32_t first, int32_t stride) {
  if (o.stop && *o.stop) return;  // a fused check stopped early: sums may be partial
  const int32_t nb = S.counts[1];
  for (int32_t k = first; k < nb; k += stride) {
    const WorkRec r = S.big[k];
    if (r.items < 2) continue;  // single-item pairs were finalised by their wave
    const int32_t p = r.p;
    finalize_pair(o, p, from_fixed(acc[2 * (int64_t)p], acc[2 * (int64_t)p + 1]), o.flags[p]);
  }
}

__global__ __launch_bounds__(256) void finalize_split_k(Sched S, const unsigned long long* acc,
                                                        Outs o) {
  finalize_split_range(S, acc, o, blockIdx.x * 256 + threadIdx.x, gridDim.x * 256);
}

// The end of one pass and the start of the next in one launch of a single
// workgroup: the pass's split pairs are finalised (queuing their refits), then
// the refit list is planned and scheduled.  Every write that a later step
// reads comes from the same workgroup, so barriers order the three steps and
// no grid-wide synchronisation is needed.  This saves two kernel boundaries
// per call (each a few microseconds on MI355X); the steps are short (a refit
// list is usually empty, and the split pairs number a few thousand at most).
__global__ __launch_bounds__(1024) void finalize_replan_k(Sched S, const unsigned long long* acc,
                                                          Outs o, PlanArgs R, int32_t L,
                                                          LoopInfo li, Sched SR,
                                                          int32_t* zero_next) {
  finalize_split_range(S, acc, o, threadIdx.x, 1024);
  __syncthreads();
  int64_t n = R.n_list;
  const int64_t nd = __hip_atomic_load(R.n_list_dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  n = nd < n ? nd : n;
  plan_positions(R, L, li, SR, 1, 0.0, n, 0, 1024);
  __syncthreads();
  schedule(SR, zero_next);
}

__global__ __launch_bounds__(1024) void sched_k(Sched S, int32_t* zero_next) {
  schedule(S, zero_next);
}

// General single-workgroup exclusive scan (pair search, verification).
__global__ __launch_bounds__(1024) void scan_k(const int64_t* counts, int64_t n, int64_t* prefix) {
  __shared__ int64_t wsum[16];
  block_scan_array(counts, n, prefix, wsum);
}

// ------------------------------------------------------ potential link search
template <typename Tin>
__global__ __launch_bounds__(256) void boxes_k(const Tin* X, const int64_t* off, int32_t L,
                                               double* box) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t l = wave; l < L; l += nwaves) {
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t v = off[l] + lane; v < off[l + 1]; v += 64)
      for (int q = 0; q < 3; ++q) {
        const double x = (double)X[3 * v + q];
        lo[q] = fmin(lo[q], x);
        hi[q] = fmax(hi[q], x);
      }
    for (int o = 32; o > 0; o >>= 1)
      for (int q = 0; q < 3; ++q) {
        lo[q] = fmin(lo[q], __shfl_xor(lo[q], o));
        hi[q] = fmax(hi[q], __shfl_xor(hi[q], o));
      }
    if (lane == 0)
      for (int q = 0; q < 3; ++q) {
        box[6 * l + q] = lo[q];
        box[6 * l + 3 + q] = hi[q];
      }
  }
}

__device__ __forceinline__ bool overlap(const double* P, const double* Q) {
  return !(P[0] > Q[3] || Q[0] > P[3] || P[1] > Q[4] || Q[1] > P[4] || P[2] > Q[5] || Q[2] > P[5]);
}

// Thread i scans j > i through LDS tiles of boxes; write = 0 counts, 1 fills.
template <int WRITE>
__global__ __launch_bounds__(256) void pair_scan_k(const double* box, int32_t L, int64_t* counts,
                                                   const int64_t* row_start, int32_t* out,
                                                   int64_t cap) {
  __shared__ double tile[256 * 6];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double me[6];
  if (i < L)
    for (int q = 0; q < 6; ++q) me[q] = box[6 * i + q];
  int64_t cnt = 0;
  int64_t pos = (WRITE && i < L) ? row_start[i] : 0;
  for (int64_t t0 = (int64_t)blockIdx.x * 256; t0 < L; t0 += 256) {
    __syncthreads();
    for (int k = threadIdx.x; k < 256 * 6; k += 256) {
      const int64_t g = t0 * 6 + k;
      tile[k] = (g < (int64_t)L * 6) ? box[g] : 0.0;
    }
    __syncthreads();
    if (i < L) {
      const int kend = (L - t0) < 256 ? (int)(L - t0) : 256;
      for (int k = 0; k < kend; ++k) {
        const int64_t j = t0 + k;
        if (j <= i) continue;
        if (overlap(me, &tile[6 * k])) {
          if (WRITE) {
            if (pos < cap) {
              out[2 * pos] = (int32_t)i;
              out[2 * pos + 1] = (int32_t)j;
            }
            ++pos;
          } else {
            ++cnt;
          }
        }
      }
    }
  }
  if (!WRITE && i < L) counts[i] = cnt;
}

// ------------------------------------- potential link search on a hashed grid
// A box is "regular" when it is finite and no side is longer than half the
// cell size h; regular boxes are binned by the cell of their min corner.  Two
// overlapping regular boxes have min corners at most h/2 apart on every
// axis, so their cells differ by at most one: a regular box only meets the
// regular boxes of the 27 cells around its own.  Cells are hashed into a
// table of buckets, so the scene's extent does not matter; boxes of other
// cells that share a bucket are candidates the box test rejects.  Every
// other box (large, empty or non-finite) is tested against all boxes with
// the same predicate as the brute-force scan, so both give exactly the same
// pairs.  Each pair is found once, from its smaller index; a row's pairs are
// sorted by j afterwards, so the output is lexicographic.
__device__ __forceinline__ bool box_regular(const double* b, double h) {
  bool ok = true;
  for (int q = 0; q < 3; ++q) {
    const double e = b[3 + q] - b[q];
    ok = ok && isfinite(b[q]) && isfinite(b[3 + q]) && e >= 0.0 && e <= 0.5 * h;
  }
  return ok;
}

__device__ __forceinline__ int64_t grid_coord(const GridParams& g, const double* b, int q) {
  // far beyond any real scene the coordinate saturates (a shared cell only
  // adds candidates; boxes that far apart do not overlap a nearer one)
  const double c = floor((b[q] - g.lo[q]) / g.h);
  return c < 4.0e18 ? (int64_t)c : (int64_t)4000000000000000000ll;
}

// buckets is a power of two, so the hash is masked rather than divided
__device__ __forceinline__ int64_t grid_bucket(const GridParams& g, int64_t x, int64_t y,
                                               int64_t z) {
  const uint64_t k = ((uint64_t)x * 73856093ull) ^ ((uint64_t)y * 19349663ull) ^
                     ((uint64_t)z * 83492791ull);
  return (int64_t)((k ^ (k >> 29)) & (uint64_t)(g.buckets - 1));
}

// The grid parameters in three passes over the boxes; grid_bin_k finishes
// them from the partials.  Every reduction runs in a fixed order (64 workgroup
// partials, each a tree in LDS), so the cell size does not depend on
// scheduling.  Pass 0 sums the box sizes (the largest side per box) and
// clears the bucket counts; pass 1 takes the largest size not above 4 x their
// mean; pass 2 takes the least min corner of the boxes regular at h = 2 x that
// largest size.  A box's size and regularity use the same tests everywhere.
__device__ __forceinline__ double grid_box_size(const double* b) {
  double e = -1.0;
  for (int q = 0; q < 3; ++q) e = fmax(e, b[3 + q] - b[q]);
  return e;
}

// every thread of every workgroup reduces the partials the same way
__device__ __forceinline__ double grid_size_cap(const double* part) {
  double s = 0.0, c = 0.0;
  for (int k = 0; k < kGridStatBlocks; ++k) {
    s += part[k];
    c += part[kGridStatBlocks + k];
  }
  return 4.0 * (c > 0.0 ? s / c : 0.0);
}
__device__ __forceinline__ double grid_cell_size(const double* part) {
  double em = 0.0;
  for (int k = 0; k < kGridStatBlocks; ++k) em = fmax(em, part[2 * kGridStatBlocks + k]);
  return em > 0.0 ? 2.0 * em : 1.0;
}

template <int PASS>
__global__ __launch_bounds__(256) void grid_stats_k(const double* box, int32_t L,
                                                    int64_t buckets, double* part,
                                                    unsigned long long* cell_count,
                                                    int32_t* n_over) {
  __shared__ double red[3][256];
  const int t = threadIdx.x;
  const double cap = PASS == 1 ? grid_size_cap(part) : 0.0;
  const double h = PASS == 2 ? grid_cell_size(part) : 0.0;
  double v[3] = {0.0, 0.0, 0.0};
  if (PASS == 2) v[0] = v[1] = v[2] = INFINITY;
  for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < L; i += kGridStatBlocks * 256) {
    const double* b = box + 6 * i;
    if (PASS == 0) {
      const double e = grid_box_size(b);
      if (isfinite(e) && e >= 0.0) {
        v[0] += e;
        v[1] += 1.0;
      }
    } else if (PASS == 1) {
      const double e = grid_box_size(b);
      if (isfinite(e) && e <= cap) v[0] = fmax(v[0], e);
    } else if (box_regular(b, h)) {
      for (int q = 0; q < 3; ++q) v[q] = fmin(v[q], b[q]);
    }
  }
  if (PASS == 0) {
    for (int64_t k = (int64_t)blockIdx.x * 256 + t; k < buckets; k += kGridStatBlocks * 256)
      cell_count[k] = 0ull;
    if (blockIdx.x == 0 && t == 0) *n_over = 0;
  }
  for (int q = 0; q < 3; ++q) red[q][t] = v[q];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) {
      if (PASS == 0) {
        red[0][t] += red[0][t + w];
        red[1][t] += red[1][t + w];
      } else if (PASS == 1) {
        red[0][t] = fmax(red[0][t], red[0][t + w]);
      } else {
        for (int q = 0; q < 3; ++q) red[q][t] = fmin(red[q][t], red[q][t + w]);
      }
    }
    __syncthreads();
  }
  if (t == 0) {
    if (PASS == 0) {
      part[blockIdx.x] = red[0][0];
      part[kGridStatBlocks + blockIdx.x] = red[1][0];
    } else if (PASS == 1) {
      part[2 * kGridStatBlocks + blockIdx.x] = red[0][0];
    } else {
      for (int q = 0; q < 3; ++q) part[(3 + q) * kGridStatBlocks + blockIdx.x] = red[q][0];
    }
  }
}

__device__ GridParams grid_params_of(const double* part, int64_t buckets) {
  GridParams g;
  g.h = grid_cell_size(part);
  for (int q = 0; q < 3; ++q) {
    double m = INFINITY;
    for (int k = 0; k < kGridStatBlocks; ++k) m = fmin(m, part[(3 + q) * kGridStatBlocks + k]);
    g.lo[q] = isfinite(m) ? m : 0.0;
  }
  g.buckets = buckets;
  return g;
}

// Exclusive scan across workgroups of 4096 entries: the tiles' totals, a
// single-workgroup scan of those into tile offsets (whose last entry is the
// grand total), then each tile's scan from its offset.
__global__ __launch_bounds__(1024) void tile_sums_k(const int64_t* counts, int64_t n,
                                                    int64_t* tile_sum) {
  __shared__ int64_t wsum[16];
  const int64_t k0 = (int64_t)blockIdx.x * 4096 + 4 * (int64_t)threadIdx.x;
  int64_t v = 0;
  for (int i = 0; i < 4; ++i) v += (k0 + i < n) ? counts[k0 + i] : 0;
  int64_t tot = 0;
  block_excl_scan(v, wsum, &tot);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ __launch_bounds__(1024) void tile_scan_k(const int64_t* counts, int64_t n,
                                                    const int64_t* tile_off, int64_t* prefix) {
  __shared__ int64_t wsum[16];
  const int64_t k0 = (int64_t)blockIdx.x * 4096 + 4 * (int64_t)threadIdx.x;
  int64_t v[4], sum = 0;
  for (int i = 0; i < 4; ++i) {
    v[i] = (k0 + i < n) ? counts[k0 + i] : 0;
    sum += v[i];
  }
  int64_t tot = 0;
  int64_t run = tile_off[blockIdx.x] + block_excl_scan(sum, wsum, &tot);
  for (int i = 0; i < 4; ++i) {
    if (k0 + i < n) prefix[k0 + i] = run;
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) prefix[n] = tile_off[gridDim.x];
}

// Each workgroup finishes the grid parameters from the partials (the same
// fixed order everywhere); the first one stores them for the later kernels.
__global__ __launch_bounds__(256) void grid_bin_k(const double* box, int32_t L,
                                                  const double* part, int64_t buckets,
                                                  GridParams* gp,
                                                  unsigned long long* cell_count,
                                                  int64_t* cell_of, int32_t* over,
                                                  int32_t* n_over) {
  __shared__ GridParams gs;
  if (threadIdx.x == 0) {
    gs = grid_params_of(part, buckets);
    if (blockIdx.x == 0) *gp = gs;
  }
  __syncthreads();
  const GridParams g = gs;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < L; i += (int64_t)gridDim.x * 256) {
    const double* b = box + 6 * i;
    if (box_regular(b, g.h)) {
      const int64_t c =
          grid_bucket(g, grid_coord(g, b, 0), grid_coord(g, b, 1), grid_coord(g, b, 2));
      cell_of[i] = c;
      atomicAdd(&cell_count[c], 1ull);
    } else {
      cell_of[i] = -1;
      over[atomicAdd(n_over, 1)] = (int32_t)i;
    }
  }
}

// cell_count still holds the counts: each box takes a slot by counting down;
// a copy of the box goes with it, so a bucket's boxes are read contiguously.
__global__ __launch_bounds__(256) void grid_scatter_k(const double* box, int32_t L,
                                                      const int64_t* cell_of,
                                                      const int64_t* cell_start,
                                                      unsigned long long* cell_count,
                                                      int32_t* cell_items, double* cell_box) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < L; i += (int64_t)gridDim.x * 256) {
    const int64_t c = cell_of[i];
    if (c < 0) continue;
    const unsigned long long k = atomicAdd(&cell_count[c], ~0ull);  // - 1
    const int64_t pos = cell_start[c] + (int64_t)k - 1;
    cell_items[pos] = (int32_t)i;
    for (int q = 0; q < 6; ++q) cell_box[6 * pos + q] = box[6 * i + q];
  }
}

// Row i: the pairs (i, j > i), one wavefront per row, the lanes testing
// candidates side by side.  WRITE = 0 counts, 1 fills (in bucket order for a
// regular box; ascending j for the others, since each chunk of 64 is emitted
// in lane order).
template <int WRITE>
__global__ __launch_bounds__(256) void grid_rows_k(const double* box, int32_t L,
                                                   const GridParams* gp, const int64_t* cell_of,
                                                   const int64_t* cell_start,
                                                   const int32_t* cell_items,
                                                   const double* cell_box, const int32_t* over,
                                                   const int32_t* n_over, int64_t* counts,
                                                   const int64_t* row_start, int32_t* out) {
  const GridParams g = *gp;
  const int32_t no = *n_over;
  const int lane = threadIdx.x & 63;
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  for (int64_t i = wave; i < L; i += nwaves) {
    double me[6];
    for (int q = 0; q < 6; ++q) me[q] = box[6 * i + q];
    int64_t pos = WRITE ? row_start[i] : 0;  // uniform over the wave
    // all lanes call it; lane with `hit` writes (i, j) in lane order
    auto emit = [&](bool hit, int64_t j) {
      const unsigned long long m = __ballot(hit);
      if (WRITE && hit) {
        const int64_t at = pos + __popcll(m & below);
        out[2 * at] = (int32_t)i;
        out[2 * at + 1] = (int32_t)j;
      }
      pos += __popcll(m);
    };
    if (cell_of[i] >= 0) {
      const int64_t c0 = grid_coord(g, me, 0), c1 = grid_coord(g, me, 1), c2 = grid_coord(g, me, 2);
      // lane t < 27 hashes neighbour cell t; a bucket reached by two
      // neighbour cells is visited once (at its first lane)
      const int tl = lane < 27 ? lane : 0;
      const int64_t mine = grid_bucket(g, c0 + tl % 3 - 1, c1 + (tl / 3) % 3 - 1, c2 + tl / 9 - 1);
      bool dup = false;
      for (int u = 0; u < 27; ++u) {
        const int64_t bu = __shfl(mine, u);
        dup = dup || (u < lane && bu == mine);
      }
      const unsigned long long visit = __ballot(lane < 27 && !dup);
      for (int t = 0; t < 27; ++t) {
        if (!((visit >> t) & 1ull)) continue;
        const int64_t c = __shfl(mine, t);
        for (int64_t k0 = cell_start[c]; k0 < cell_start[c + 1]; k0 += 64) {
          const int64_t k = k0 + lane;
          const bool in = k < cell_start[c + 1];
          const int32_t j = in ? cell_items[k] : -1;
          emit(in && j > i && overlap(me, cell_box + 6 * k), j);
        }
      }
      for (int32_t k0 = 0; k0 < no; k0 += 64) {
        const int32_t k = k0 + lane;
        const int32_t j = k < no ? over[k] : -1;
        emit(k < no && j > i && overlap(me, box + 6 * (int64_t)j), j);
      }
    } else {
      for (int64_t j0 = i + 1; j0 < L; j0 += 64) {
        const int64_t j = j0 + lane;
        emit(j < L && overlap(me, box + 6 * (j < L ? j : 0)), j);
      }
    }
    if (!WRITE && lane == 0) counts[i] = pos;
  }
}

// Rows of regular boxes were filled in cell order: sort each by j.
__global__ __launch_bounds__(256) void grid_sort_rows_k(int32_t L, const int64_t* cell_of,
                                                        const int64_t* row_start, int32_t* out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < L; i += (int64_t)gridDim.x * 256) {
    if (cell_of[i] < 0) continue;
    const int64_t a = row_start[i], b = row_start[i + 1];
    for (int64_t k = a + 1; k < b; ++k) {
      const int32_t v = out[2 * k + 1];
      int64_t m = k - 1;
      while (m >= a && out[2 * m + 1] > v) {
        out[2 * (m + 1) + 1] = out[2 * m + 1];
        --m;
      }
      out[2 * (m + 1) + 1] = v;
    }
  }
}

// ------------------------------------------------------------ verification
__device__ __forceinline__ long long key_of(const int32_t* pr, int64_t k) {
  return ((long long)pr[2 * k] << 32) | (unsigned int)pr[2 * k + 1];
}
// first index in [0, n) whose key is >= x
__device__ __forceinline__ int64_t lower_bound_key(const int32_t* pr, int64_t n, long long x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (key_of(pr, mid) < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Mismatch indicator per position of the concatenation [current | expected]:
// current c mismatches when lk[c] differs from the expected value (0 if the
// pair is not expected); expected e counts when it is absent from the current
// list and non-zero.
__global__ __launch_bounds__(256) void verify_flag_k(const int32_t* pr, const int32_t* lk,
                                                     int64_t n, const int32_t* ep,
                                                     const int32_t* elk, int64_t ne,
                                                     int64_t* m) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k < n) {
    const long long x = key_of(pr, k);
    const int64_t e = lower_bound_key(ep, ne, x);
    const int32_t want = (e < ne && key_of(ep, e) == x) ? elk[e] : 0;
    m[k] = (lk[k] != want) ? 1 : 0;
  } else if (k < n + ne) {
    const int64_t e = k - n;
    const long long x = key_of(ep, e);
    const int64_t c = lower_bound_key(pr, n, x);
    const bool present = c < n && key_of(pr, c) == x;
    m[k] = (!present && elk[e] != 0) ? 1 : 0;
  }
}

// Scatter mismatch records in pair order.  The rank of a mismatch in pair
// order is (mismatches of the other list with a smaller key) + (its rank
// within its own list); keys of the two lists never tie for counted records
// (a key in both lists is counted once, from the current list).
__global__ __launch_bounds__(256) void verify_scatter_k(const int32_t* pr, const int32_t* lk,
                                                        int64_t n, const int32_t* ep,
                                                        const int32_t* elk, int64_t ne,
                                                        const int64_t* mp, int32_t* out,
                                                        int64_t cap) {
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= n + ne) return;
  if (mp[k + 1] == mp[k]) return;  // not a mismatch
  const int64_t base_c = 0, base_e = mp[n];
  long long x;
  int64_t rank;
  int32_t got, want;
  if (k < n) {
    x = key_of(pr, k);
    const int64_t e = lower_bound_key(ep, ne, x);
    want = (e < ne && key_of(ep, e) == x) ? elk[e] : 0;
    got = lk[k];
    rank = (mp[k] - base_c) + (mp[n + e] - base_e);
  } else {
    const int64_t e = k - n;
    x = key_of(ep, e);
    const int64_t c = lower_bound_key(pr, n, x);
    want = elk[e];
    got = 0;
    rank = (mp[k] - base_e) + (mp[c] - base_c);
  }
  if (rank < cap) {
    out[4 * rank] = (int32_t)(x >> 32);
    out[4 * rank + 1] = (int32_t)(x & 0xffffffffll);
    out[4 * rank + 2] = got;
    out[4 * rank + 3] = want;
  }
}

// Preparation, plan and schedule of a call with few pairs in one launch of a
// single workgroup: the per-loop scan of prep_k (16 lanes per loop, so 64
// loops are scanned at once and their loads overlap), xi as this workgroup's
// fixed-order sum, then the plan and the schedule.  Each step reads only
// what the workgroup wrote before a barrier.  Used where the pairs are at
// most two per compute unit: there three launches cost more than their work
// (a call with few but very long loops scans them with one workgroup only,
// which its direct sum dwarfs).
template <typename Tin>
__global__ __launch_bounds__(1024) void prep_plan_k(const Tin* X, PlanArgs A, int32_t L,
                                                    LoopInfo li, uint32_t* lf, double* minseg2,
                                                    Sched S, unsigned long long* zero_mismatch,
                                                    int32_t* zero_stop, int32_t* zero_next) {
  __shared__ double red[1024];
  if (threadIdx.x < 2) S.counts[threadIdx.x] = 0;
  if (threadIdx.x == 0 && zero_mismatch) {
    *zero_mismatch = 0ull;
    *zero_stop = 0;
  }
  const int sub = threadIdx.x & 15, group = threadIdx.x >> 4;
  double s = 0.0;
  for (int64_t l = group; l < L; l += 64) s += scan_loop<Tin, 16>(X, A.off, l, sub, lf, minseg2);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const int64_t nv = A.off[L] - A.off[0];
  const double xi = nv > 0 ? red[0] / (3.0 * (double)nv) : 0.0;
  plan_positions(A, L, li, S, 0, xi, A.n_list, 0, 1024);
  __syncthreads();
  schedule(S, zero_next);
}

}  // namespace

// ---------------------------------------------------------------- launchers
int prep_blocks(int32_t n_loops, int64_t n_vertices) {
  // one wavefront per loop up to kPrepMaxBlocks * 4 loops, and (when the
  // vertex count is known) enough workgroups to stream the coordinates
  int64_t g = ((int64_t)n_loops + 3) / 4;
  const int64_t gv = n_vertices / 8192;
  if (gv > g) g = gv;
  if (g < kXiBlocks) g = kXiBlocks;
  if (g > kPrepMaxBlocks) g = kPrepMaxBlocks;
  return (int)g;
}

hipError_t launch_prep(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                       double* xi_partials, uint32_t* lf, double* minseg2, int32_t* zero_counts,
                       unsigned long long* zero_mismatch, int32_t* zero_stop, bool scan_loops,
                       int n_blocks, hipStream_t s) {
  const int g = n_blocks;
  const int sl = scan_loops ? 1 : 0;
  if (in_f64)
    prep_k<double><<<g, 256, 0, s>>>((const double*)xyz, off, n_loops, xi_partials, lf, minseg2,
                                     zero_counts, zero_mismatch, zero_stop, sl);
  else
    prep_k<float><<<g, 256, 0, s>>>((const float*)xyz, off, n_loops, xi_partials, lf, minseg2,
                                    zero_counts, zero_mismatch, zero_stop, sl);
  return hipGetLastError();
}

hipError_t launch_cc_boxes(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                           const CcProj& pr, float4* blk, int64_t n_blk, float4* sup,
                           int64_t n_sup, uint32_t* lf, double* minseg2, hipStream_t s) {
  // four slots (waves) per workgroup; the grid strides over the device's count
  const int g = blocks_for(n_sup, 4, 16384);
  if (in_f64)
    cc_boxes_k<double><<<g, 256, 0, s>>>((const double*)xyz, off, n_loops, pr, blk, n_blk, sup,
                                         n_sup, lf, minseg2);
  else
    cc_boxes_k<float><<<g, 256, 0, s>>>((const float*)xyz, off, n_loops, pr, blk, n_blk, sup, n_sup,
                                        lf, minseg2);
  return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs& a, int32_t n_loops, const LoopInfo& li, const Sched& sc,
                       bool refit, hipStream_t s) {
  // a refit list is short (pairs far from an integer): a few workgroups
  plan_k<<<blocks_for(a.n_list, 1024, refit ? 16 : 8192), 1024, 0, s>>>(a, n_loops, li, sc,
                                                                       refit ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_finalize_split(const Sched& sc, const unsigned long long* acc, const Outs& o,
                                 int64_t n_pairs, hipStream_t s) {
  // only multi-item pairs remain, at most a few thousand: grid stride
  finalize_split_k<<<blocks_for(n_pairs, 256, 64), 256, 0, s>>>(sc, acc, o);
  return hipGetLastError();
}

hipError_t launch_sched(const Sched& sc, int32_t* zero_next, hipStream_t s) {
  sched_k<<<1, 1024, 0, s>>>(sc, zero_next);
  return hipGetLastError();
}

hipError_t launch_prep_plan(const void* xyz, bool in_f64, const PlanArgs& a, int32_t n_loops,
                            const LoopInfo& li, uint32_t* lf, double* minseg2, const Sched& sc,
                            unsigned long long* zero_mismatch, int32_t* zero_stop,
                            int32_t* zero_next, hipStream_t s) {
  if (a.list || a.n_list_dev) return hipErrorInvalidValue;  // the main pass only
  if (in_f64)
    prep_plan_k<double><<<1, 1024, 0, s>>>((const double*)xyz, a, n_loops, li, lf, minseg2, sc,
                                          zero_mismatch, zero_stop, zero_next);
  else
    prep_plan_k<float><<<1, 1024, 0, s>>>((const float*)xyz, a, n_loops, li, lf, minseg2, sc,
                                         zero_mismatch, zero_stop, zero_next);
  return hipGetLastError();
}

hipError_t launch_finalize_replan(const Sched& sc, const unsigned long long* acc, const Outs& o,
                                  const PlanArgs& r, int32_t n_loops, const LoopInfo& li,
                                  const Sched& sr, int32_t* zero_next, hipStream_t s) {
  if (!r.n_list_dev) return hipErrorInvalidValue;
  finalize_replan_k<<<1, 1024, 0, s>>>(sc, acc, o, r, n_loops, li, sr, zero_next);
  return hipGetLastError();
}

__global__ void zero_i64_k(int64_t* p) { *p = 0; }

hipError_t launch_zero_i64(int64_t* p, hipStream_t s) {
  zero_i64_k<<<1, 1, 0, s>>>(p);
  return hipGetLastError();
}

hipError_t launch_scan(const int64_t* counts, int64_t n, int64_t* prefix, hipStream_t s) {
  scan_k<<<1, 1024, 0, s>>>(counts, n, prefix);
  return hipGetLastError();
}

hipError_t launch_boxes(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                        double* boxes, hipStream_t s) {
  const int lb = blocks_for((int64_t)n_loops * 64, 256, 8192);
  if (in_f64)
    boxes_k<double><<<lb, 256, 0, s>>>((const double*)xyz, off, n_loops, boxes);
  else
    boxes_k<float><<<lb, 256, 0, s>>>((const float*)xyz, off, n_loops, boxes);
  return hipGetLastError();
}

hipError_t launch_pair_count(const double* boxes, int32_t n_loops, int64_t* counts,
                             hipStream_t s) {
  pair_scan_k<0><<<blocks_for(n_loops, 256), 256, 0, s>>>(boxes, n_loops, counts, nullptr, nullptr,
                                                          0);
  return hipGetLastError();
}

hipError_t launch_pair_fill(const double* boxes, int32_t n_loops, const int64_t* row_start,
                            int32_t* pairs_out, int64_t capacity, hipStream_t s) {
  pair_scan_k<1><<<blocks_for(n_loops, 256), 256, 0, s>>>(boxes, n_loops, nullptr, row_start,
                                                          pairs_out, capacity);
  return hipGetLastError();
}

hipError_t launch_grid_pairs(const double* boxes, int32_t n_loops, const GridBufs& b, int pass,
                             const int64_t* row_start, int32_t* pairs_out, hipStream_t s) {
  const int g = blocks_for(n_loops, 256, 4096);
  const int gw = blocks_for((int64_t)n_loops * 64, 256, 16384);  // one wavefront per row
  switch (pass) {
    case 0: {  // grid, binning and the per-cell scan
      grid_stats_k<0><<<kGridStatBlocks, 256, 0, s>>>(boxes, n_loops, b.buckets, b.part,
                                                      b.cell_count, b.n_over);
      grid_stats_k<1><<<kGridStatBlocks, 256, 0, s>>>(boxes, n_loops, b.buckets, b.part,
                                                      nullptr, nullptr);
      grid_stats_k<2><<<kGridStatBlocks, 256, 0, s>>>(boxes, n_loops, b.buckets, b.part,
                                                      nullptr, nullptr);
      grid_bin_k<<<g, 256, 0, s>>>(boxes, n_loops, b.part, b.buckets, b.params, b.cell_count,
                                   b.cell_of, b.over, b.n_over);
      const int64_t nt = (b.buckets + 4095) / 4096;
      const int64_t* counts = reinterpret_cast<const int64_t*>(b.cell_count);
      tile_sums_k<<<(unsigned)nt, 1024, 0, s>>>(counts, b.buckets, b.tiles);
      scan_k<<<1, 1024, 0, s>>>(b.tiles, nt, b.tiles + nt + 1);
      tile_scan_k<<<(unsigned)nt, 1024, 0, s>>>(counts, b.buckets, b.tiles + nt + 1,
                                                b.cell_start);
      grid_scatter_k<<<g, 256, 0, s>>>(boxes, n_loops, b.cell_of, b.cell_start, b.cell_count,
                                       b.cell_items, b.cell_box);
      grid_rows_k<0><<<gw, 256, 0, s>>>(boxes, n_loops, b.params, b.cell_of, b.cell_start,
                                       b.cell_items, b.cell_box, b.over, b.n_over, b.row_counts,
                                       nullptr, nullptr);
      break;
    }
    default:  // fill and sort the rows
      grid_rows_k<1><<<gw, 256, 0, s>>>(boxes, n_loops, b.params, b.cell_of, b.cell_start,
                                       b.cell_items, b.cell_box, b.over, b.n_over, nullptr,
                                       row_start, pairs_out);
      grid_sort_rows_k<<<g, 256, 0, s>>>(n_loops, b.cell_of, row_start, pairs_out);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_verify(const int32_t* pairs, const int32_t* lk, int64_t n,
                         const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                         int64_t* mism_counts, hipStream_t s) {
  verify_flag_k<<<blocks_for(n + n_exp, 256), 256, 0, s>>>(pairs, lk, n, exp_pairs, exp_lk, n_exp,
                                                           mism_counts);
  return hipGetLastError();
}

hipError_t launch_verify_scatter(const int32_t* pairs, const int32_t* lk, int64_t n,
                                 const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                                 const int64_t* mism_prefix, int32_t* out, int64_t cap,
                                 hipStream_t s) {
  verify_scatter_k<<<blocks_for(n + n_exp, 256), 256, 0, s>>>(pairs, lk, n, exp_pairs, exp_lk,
                                                              n_exp, mism_prefix, out, cap);
  return hipGetLastError();
}

}  // namespace lk
