// lk_aux.hip -- everything around the direct-sum hot loop: input validation,
// work planning, the device-side scan, conversion of the fixed-point sums to
// outputs (round + flag + refit list), the potential link search (Alg. 2) and
// the verification merge (Sec. 3.1, "Fast Verification").
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

constexpr uint32_t kFlagRefit = 1u, kFlagAmbiguous = 2u, kFlagNonfinite = 4u, kFlagBadpair = 8u,
                   kFlagBadloop = 16u;
constexpr int32_t kIntInvalid = INT32_MIN;

inline int blocks_for(int64_t n, int threads, int cap = 65535 * 8) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

// ------------------------------------------------------------- validation
template <typename Tin>
__global__ __launch_bounds__(256) void xi_partial(const Tin* X, const int64_t* off, int32_t L,
                                                  double* part) {
  __shared__ double red[256];
  const int64_t v0 = off[0], v1 = off[L];
  const int64_t n = 3 * (v1 - v0);
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < n; k += (int64_t)gridDim.x * 256)
    s += fabs((double)X[3 * v0 + k]);
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void xi_final(const double* part, const int64_t* off, int32_t L,
                                                double* xi, int32_t* zero_counts) {
  __shared__ double red[256];
  red[threadIdx.x] = part[threadIdx.x];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int64_t nv = off[L] - off[0];
    *xi = nv > 0 ? red[0] / (3.0 * (double)nv) : 0.0;
    if (zero_counts) {
      zero_counts[0] = 0;
      zero_counts[1] = 0;
    }
  }
}

// One wavefront per loop: <3 vertices, non-finite coordinates and segments
// shorter than eps * xi (the zero-length test of Alg. 3).
template <typename Tin>
__global__ __launch_bounds__(256) void loop_flags_k(const Tin* X, const int64_t* off, int32_t L,
                                                    const double* xi, double eps, uint32_t* lf) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * 256) >> 6;
  const double lim = eps * (*xi);
  const double lim2 = lim * lim;
  for (int64_t l = wave; l < L; l += nwaves) {
    const int64_t o = off[l], n = off[l + 1] - o;
    uint32_t f = (n < 3) ? kFlagBadloop : 0u;
    for (int64_t s = lane; s < n; s += 64) {
      const int64_t t = (s + 1 == n) ? 0 : s + 1;
      const double x0 = (double)X[3 * (o + s)], y0 = (double)X[3 * (o + s) + 1],
                   z0 = (double)X[3 * (o + s) + 2];
      const double x1 = (double)X[3 * (o + t)], y1 = (double)X[3 * (o + t) + 1],
                   z1 = (double)X[3 * (o + t) + 2];
      if (!isfinite(x0) || !isfinite(y0) || !isfinite(z0)) f |= kFlagNonfinite | kFlagBadloop;
      const double dx = x1 - x0, dy = y1 - y0, dz = z1 - z0;
      if (dx * dx + dy * dy + dz * dz < lim2) f |= kFlagBadloop;
    }
    for (int o2 = 32; o2 > 0; o2 >>= 1) f |= (uint32_t)__shfl_xor((int)f, o2);
    if (lane == 0) lf[l] = f;
  }
}

// --------------------------------------------------------------- planning
// Append to a device list from a wavefront: one atomic per wave, then each
// lane with `pred` gets base + (number of lower lanes with pred).  All active
// lanes must call it.
__device__ __forceinline__ int32_t wave_append(int32_t* count, bool pred) {
  const unsigned long long m = __ballot(pred);
  const unsigned long long act = __ballot(1);
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)act) - 1;
  int32_t base = 0;
  if (lane == leader && m) base = atomicAdd(count, (int32_t)__popcll(m));
  base = __shfl(base, leader);
  const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
  return base + (int32_t)__popcll(m & below);
}

__global__ __launch_bounds__(256) void plan_k(PlanArgs A, int32_t L, const uint32_t* lf, Sched S,
                                              int refit) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t n = A.n_list;
  if (A.n_list_dev) {
    const int64_t nd = *A.n_list_dev;
    n = nd < n ? nd : n;
  }
  if (q >= n) return;
  const int32_t p = A.list ? A.list[q] : (int32_t)q;
  const int32_t i = A.pairs[2 * p], j = A.pairs[2 * p + 1];
  const bool valid = i >= 0 && j >= 0 && i < L && j < L && i != j;
  int64_t items = 0;
  WorkRec r{};
  if (valid) {
    r.oa = A.off[i];
    r.ob = A.off[j];
    const int64_t na = A.off[i + 1] - r.oa, nb = A.off[j + 1] - r.ob;
    r.na = (int32_t)na;
    r.nb = (int32_t)nb;
    if (na >= 1 && nb >= 1) items = ((nb + A.bblock - 1) / A.bblock) * ((na + A.chunk - 1) / A.chunk);
  }
  // loops beyond 2^31 vertices or pairs beyond 2^31 work items are not handled
  const bool too_big = valid && (A.off[i + 1] - A.off[i] > 0x7fffffffLL ||
                                 A.off[j + 1] - A.off[j] > 0x7fffffffLL || items > 0x7fffffffLL);
  if (too_big) items = 0;
  if (refit)
    A.flags[p] = (A.flags[p] & ~kFlagNonfinite) | (too_big ? kFlagNonfinite : 0u);
  else
    A.flags[p] = valid ? (lf[i] | lf[j] | (too_big ? kFlagBadloop | kFlagNonfinite : 0u))
                       : kFlagBadpair;
  A.acc[2 * (int64_t)p] = 0ull;
  A.acc[2 * (int64_t)p + 1] = 0ull;
  r.p = p;
  r.items = (int32_t)items;
  const bool small = items == 1 && r.na < kSmallA;
  const bool big = items > 0 && !small;
  const int32_t ps = wave_append(&S.counts[0], small);
  const int32_t pb = wave_append(&S.counts[1], big);
  if (small) S.small[ps] = r;
  if (big) S.big_in[pb] = r;
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

// One workgroup: bucket the big pairs by log2(items), largest bucket first
// (an LPT order up to a factor of two), then scan their items.
__global__ __launch_bounds__(1024) void sched_k(Sched S, int32_t* zero_next) {
  __shared__ int hist[32];
  __shared__ int cur[32];
  __shared__ int64_t wsum[16];
  const int t = threadIdx.x;
  const int nb = S.counts[1];
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

// General single-workgroup exclusive scan (pair search, verification).
__global__ __launch_bounds__(1024) void scan_k(const int64_t* counts, int64_t n, int64_t* prefix) {
  __shared__ int64_t wsum[16];
  block_scan_array(counts, n, prefix, wsum);
}

__global__ __launch_bounds__(256) void finalize_k(PlanArgs A, double thr, double* lk_real,
                                                  int32_t* lk_int, int32_t* refit_list,
                                                  int32_t* refit_n, int refit_pass) {
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t n = A.n_list;
  if (A.n_list_dev) {
    const int64_t nd = *A.n_list_dev;
    n = nd < n ? nd : n;
  }
  if (q >= n) return;
  const int32_t p = A.list ? A.list[q] : (int32_t)q;
  uint32_t f = A.flags[p];
  unsigned long long lo = A.acc[2 * (int64_t)p], hi = A.acc[2 * (int64_t)p + 1];
  // 128-bit two's complement -> sign and magnitude -> double (one rounding of
  // the fraction word, one of the sum)
  const bool neg = (long long)hi < 0;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  const double mag = (double)hi + (double)lo * 5.421010862427522170e-20;  // 2^-64
  const double v = neg ? -mag : mag;
  bool requeue = false;
  if (f & kFlagBadpair) {
    lk_real[p] = __builtin_nan("");
    lk_int[p] = kIntInvalid;
  } else {
    if (refit_pass) f |= kFlagRefit;
    const bool bad = (f & kFlagNonfinite) || !isfinite(v) || fabs(v) > 2.0e9;
    if (bad) {
      f |= kFlagNonfinite;
      lk_real[p] = __builtin_nan("");
      lk_int[p] = kIntInvalid;
      requeue = refit_list != nullptr;
    } else {
      const double r = round(v);  // half away from zero
      const double frac = fabs(v - r);
      lk_real[p] = v;
      lk_int[p] = (int32_t)r;
      if (frac > thr) {
        if (refit_list)
          requeue = true;
        else
          f |= kFlagAmbiguous;
      }
    }
    A.flags[p] = f;
  }
  if (refit_list) {
    const int32_t pos = wave_append(refit_n, requeue);
    if (requeue) refit_list[pos] = p;
  }
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

}  // namespace

// ---------------------------------------------------------------- launchers
hipError_t launch_loop_flags(const void* xyz, bool in_f64, const int64_t* off, int32_t n_loops,
                             double* xi_partials, double* xi, uint32_t* lf, int32_t* zero_counts,
                             hipStream_t s) {
  const int lb = blocks_for((int64_t)n_loops * 64, 256, 8192);
  if (in_f64) {
    xi_partial<double><<<kXiBlocks, 256, 0, s>>>((const double*)xyz, off, n_loops, xi_partials);
    xi_final<<<1, 256, 0, s>>>(xi_partials, off, n_loops, xi, zero_counts);
    loop_flags_k<double><<<lb, 256, 0, s>>>((const double*)xyz, off, n_loops, xi, DBL_EPSILON, lf);
  } else {
    xi_partial<float><<<kXiBlocks, 256, 0, s>>>((const float*)xyz, off, n_loops, xi_partials);
    xi_final<<<1, 256, 0, s>>>(xi_partials, off, n_loops, xi, zero_counts);
    loop_flags_k<float><<<lb, 256, 0, s>>>((const float*)xyz, off, n_loops, xi,
                                           (double)FLT_EPSILON, lf);
  }
  return hipGetLastError();
}

hipError_t launch_plan(const PlanArgs& a, int32_t n_loops, const uint32_t* lf, const Sched& sc,
                       bool refit, hipStream_t s) {
  plan_k<<<blocks_for(a.n_list, 256), 256, 0, s>>>(a, n_loops, lf, sc, refit ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_sched(const Sched& sc, int32_t* zero_next, hipStream_t s) {
  sched_k<<<1, 1024, 0, s>>>(sc, zero_next);
  return hipGetLastError();
}

hipError_t launch_scan(const int64_t* counts, int64_t n, int64_t* prefix, hipStream_t s) {
  scan_k<<<1, 1024, 0, s>>>(counts, n, prefix);
  return hipGetLastError();
}

hipError_t launch_finalize(const PlanArgs& a, double thr, double* lk_real, int32_t* lk_int,
                           int32_t* refit_list, int32_t* refit_n, bool refit_pass,
                           hipStream_t s) {
  finalize_k<<<blocks_for(a.n_list, 256), 256, 0, s>>>(a, thr, lk_real, lk_int, refit_list,
                                                       refit_n, refit_pass ? 1 : 0);
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
