// lk_ds.hip -- the direct-summation hot loop for CDNA4 (gfx950).
//
// Computes, for every work item (pair p, a block of 64 segments of loop B, a
// chunk of segments of loop A), the partial sum of the Eq. 4 segment-pair term
// and adds it into the pair's 128-bit fixed-point accumulator.
//
// Layout of the work (one 64-lane wavefront = one workgroup = one item):
//   * each lane owns one segment (k_i, k_{i+1}) of loop B in registers;
//   * the item's vertices of loop A are staged through LDS in tiles and every
//     lane walks them in order (a broadcast read: all lanes read the same
//     vertex at the same step);
//   * when loop B has fewer than 64 segments left, the lanes split loop A's
//     range into groups instead (both loops parallel, as the paper does for
//     small pairs).
// The kernel is persistent: a fixed grid of waves pulls items from a device
// counter until the device-side item total is reached, so the launch shape
// does not depend on the data and the whole pass can live in a HIP graph.
//
// Per term (Eq. 4, Sec. 2.1): a = l_j - k_i, b = l_j - k_{i+1},
// c = l_{j+1} - k_{i+1}, d = l_{j+1} - k_i.  Walking j in order, a and b of
// segment j+1 are d and c of segment j, so each step needs only two new
// vertex-pair vectors, two square roots and four dot products.  The common
// numerator of both arctangents is p = a . (s_j x s_i) (equal to a . (b x c)
// and c . (d x a) in exact arithmetic, Sec. 3.4.2, but computed from the
// short segment vectors, which keeps FP32 accurate for distant pairs).  The
// two arctangents are merged into one: (d1 + i p)(d2 + i p) has the angle
// atan2(p, d1) + atan2(p, d2), which stays inside (-pi, pi) because the
// pair's parallelogram subtends less than a hemisphere, so
//   theta = atan2(p (d1 + d2), d1 d2 - p^2),  term = theta / (2 pi)
// (the angle-addition idea of the appendix, Alg. 7, applied per term).
#include "lk_internal.h"
#include "atan_poly.h"

namespace lk {
namespace {

template <typename T>
struct V3 {
  T x, y, z;
};
template <typename T>
__device__ __forceinline__ V3<T> operator-(const V3<T>& a, const V3<T>& b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <typename T>
__device__ __forceinline__ T dot(const V3<T>& a, const V3<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

// Own FP32 arctangent: octant reduction to t = min/max in [0, 1], then
// atan(t) = t q(t^2) with q the Remez minimax polynomial of atan_poly.h.
// (0, 0) gives NaN on purpose: it only arises for touching segments.
__device__ __forceinline__ float atan2_minimax(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float mx = fmaxf(ax, ay), mn = fminf(ax, ay);
  const float t = mn * __builtin_amdgcn_rcpf(mx);
  const float s = t * t;
  float q = kAtanQ[LK_ATAN_DEG];
#pragma unroll
  for (int k = LK_ATAN_DEG - 1; k >= 0; --k) q = fmaf(q, s, kAtanQ[k]);
  float r = t * q;
  r = (ay > ax) ? (1.57079632679489662f - r) : r;
  r = (x < 0.0f) ? (3.14159265358979324f - r) : r;
  return copysignf(r, y);
}

template <typename T, int AT>
__device__ __forceinline__ T angle(T y, T x);
template <>
__device__ __forceinline__ float angle<float, 0>(float y, float x) {
  return atan2_minimax(y, x);
}
template <>
__device__ __forceinline__ float angle<float, 1>(float y, float x) {
  return atan2f(y, x);
}
template <>
__device__ __forceinline__ double angle<double, 0>(double y, double x) {
  return atan2(y, x);
}
template <>
__device__ __forceinline__ double angle<double, 1>(double y, double x) {
  return atan2(y, x);
}

// LDS vertex record: 16 bytes for float (one ds_read_b128), 32 for double.
template <typename T>
struct alignas(4 * sizeof(T)) Vtx {
  T x, y, z, w;
};

template <typename Tc, typename Tin>
__device__ __forceinline__ V3<Tc> load_vertex(const Tin* X, int64_t v) {
  return {(Tc)X[3 * v], (Tc)X[3 * v + 1], (Tc)X[3 * v + 2]};
}

// The R consecutive segments of loop B owned by a lane: vertices k_0..k_R and
// segment vectors s_r = k_{r+1} - k_r.  Segments past the end of the item are
// evaluated on repeated vertices and masked out.
template <typename T, int R>
struct Segs {
  V3<T> k[R + 1];
  V3<T> s[R];
  bool valid[R];
};

// Walk state at vertex l_j of loop A, for all R + 1 vertices of the lane:
// V_r = l_j - k_r, N_r = |V_r|, E_r = N_r N_{r+1} + V_r . V_{r+1}.
template <typename T, int R>
struct Walk {
  V3<T> l;
  V3<T> V[R + 1];
  T N[R + 1];
  T E[R];
};

template <typename T, int R>
__device__ __forceinline__ void walk_init(Walk<T, R>& w, const V3<T>& l, const Segs<T, R>& g) {
  w.l = l;
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    w.V[r] = l - g.k[r];
    w.N[r] = fsqrt(dot(w.V[r], w.V[r]));
  }
#pragma unroll
  for (int r = 0; r < R; ++r) w.E[r] = w.N[r] * w.N[r + 1] + dot(w.V[r], w.V[r + 1]);
}

// The Eq. 4 terms of segment (l_j, l_{j+1}) against the lane's R segments;
// returns 2 pi times their (masked) sum and advances the walk to l_{j+1}.
// For segment r: a = V_r, b = V_{r+1} (at l_j), c = v_{r+1}, d = v_r (at
// l_{j+1}); a.b enters through E_r, and the "vertical" products V_r . v_r are
// shared by segments r - 1 and r.
template <typename T, int AT, int R>
__device__ __forceinline__ T walk_step(Walk<T, R>& w, const V3<T>& l1, const Segs<T, R>& g) {
  V3<T> v[R + 1];
  T n[R + 1], vert[R + 1];
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    v[r] = l1 - g.k[r];
    n[r] = fsqrt(dot(v[r], v[r]));
    vert[r] = dot(w.V[r], v[r]);
  }
  const V3<T> sj = l1 - w.l;
  T sum = 0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const V3<T>& a = w.V[r];
    const V3<T>& c = v[r + 1];
    const V3<T>& d = v[r];
    const T na = w.N[r], nb = w.N[r + 1], nc = n[r + 1], nd = n[r];
    const T p = dot(a, cross(sj, g.s[r]));
    const T ca = dot(c, a);
    const T f = nd * nc + dot(d, c);
    const T d1 = nc * w.E[r] + vert[r + 1] * na + ca * nb;
    const T d2 = na * f + vert[r] * nc + ca * nd;
    const T th = angle<T, AT>(p * (d1 + d2), d1 * d2 - p * p);
    sum += g.valid[r] ? th : (T)0;
    w.E[r] = f;
  }
  w.l = l1;
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    w.V[r] = v[r];
    w.N[r] = n[r];
  }
  return sum;
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

// Where the lanes of one work item sit: B block [b0, b0 + nbh) of loop B split
// into `slots` lanes of R segments; if that leaves lanes over, they form
// `groups` that split the item's A range [a0, a0 + nah) into [js, je).
struct Layout {
  int64_t b0, a0;
  int nbh, nah, bi, js, je;
  bool active;
};

template <int R>
__device__ __forceinline__ Layout layout(const WorkRec& r, int64_t local, int chunk, int lane) {
  constexpr int kB = kWave * R;
  Layout L;
  const int64_t nbb = (r.nb + kB - 1) / kB;
  L.b0 = (local % nbb) * kB;
  L.a0 = (local / nbb) * (int64_t)chunk;
  L.nbh = (int)((r.nb - L.b0) < kB ? (r.nb - L.b0) : kB);
  L.nah = (int)((r.na - L.a0) < chunk ? (r.na - L.a0) : chunk);
  const int slots = (L.nbh + R - 1) / R;
  const int groups = kWave / slots;
  L.bi = lane % slots;
  const int g = lane / slots;
  L.active = g < groups;
  L.js = (int)(((int64_t)L.nah * g) / groups);
  L.je = (int)(((int64_t)L.nah * (g + 1)) / groups);
  return L;
}

// Vertex k_{b0 + bi R + r} of loop B for r = 0..R (cyclic; padding lanes
// repeat the last vertex and are masked by Segs::valid).
template <typename Tin, typename Tc, int R>
__device__ __forceinline__ void load_b(const Tin* X, const WorkRec& w, const Layout& L,
                                       V3<Tc>* k) {
  const int first = L.bi * R;
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    int64_t i = L.b0 + first + r;
    if (i >= w.nb) i -= w.nb;
    if (i >= w.nb) i = w.nb - 1;
    k[r] = load_vertex<Tc>(X, w.ob + i);
  }
}

template <typename Tc, int R>
__device__ __forceinline__ void make_segs(const V3<Tc>* k, const Layout& L, Segs<Tc, R>& sg) {
  const int first = L.bi * R;
#pragma unroll
  for (int r = 0; r <= R; ++r) sg.k[r] = k[r];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sg.s[r] = sg.k[r + 1] - sg.k[r];
    sg.valid[r] = first + r < L.nbh;
  }
}

// Walk segments [jlo, jhi) of the item's A range, whose vertices t0 .. are in
// LDS; starts the walk when jlo is the lane's first segment.
template <typename Tc, int AT, int R>
__device__ __forceinline__ void walk_tile(const Vtx<Tc>* lds, int t0, int jlo, int jhi, int js,
                                          Walk<Tc, R>& wk, const Segs<Tc, R>& sg, double& acc) {
  if (jlo == js) {
    const Vtx<Tc> v0 = lds[jlo - t0];
    walk_init(wk, V3<Tc>{v0.x, v0.y, v0.z}, sg);
  }
#pragma unroll 4
  for (int j = jlo; j < jhi; ++j) {
    const Vtx<Tc> v1 = lds[j - t0 + 1];
    acc += (double)walk_step<Tc, AT, R>(wk, V3<Tc>{v1.x, v1.y, v1.z}, sg);
  }
}

// Wave sum of the lanes' partials and its fixed-point addition to the pair.
// `whole`: this item is the pair's only item, so the (zeroed) accumulator is
// simply overwritten and no atomic round trip is needed.
__device__ __forceinline__ void finish_item(double acc, int32_t p, int lane, const DsArgs& A,
                                            bool whole) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) {
    const double v = acc * kInvTwoPi;
    if (!(fabs(v) < 1.0e14)) {
      atomicOr(&A.flags[p], 4u);  // NaN / Inf / absurd magnitude
    } else if (whole) {
      unsigned long long lo, hi;
      to_fixed(v, lo, hi);
      A.acc[2 * (int64_t)p] = lo;
      A.acc[2 * (int64_t)p + 1] = hi;
    } else {
      fixed_add(&A.acc[2 * (int64_t)p], v);
    }
  }
}

__device__ __forceinline__ WorkRec shfl_rec(const WorkRec& r, int src) {
  WorkRec o;
  o.oa = __shfl(r.oa, src);
  o.ob = __shfl(r.ob, src);
  o.na = __shfl(r.na, src);
  o.nb = __shfl(r.nb, src);
  o.p = __shfl(r.p, src);
  o.items = 1;
  return o;
}

template <typename Tin, typename Tc, int AT, int R>
__global__ __launch_bounds__(kWave) void ds_persistent(DsArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Vtx<Tc>* lds = reinterpret_cast<Vtx<Tc>*>(lds_raw);
  const int lane = threadIdx.x;
  const Tin* X = static_cast<const Tin*>(A.xyz);
  const int64_t big_total = *A.s.big_total;
  const int64_t n_big = A.s.counts[1];
  const int64_t n_small = A.s.counts[0];
  const int64_t total = big_total + (n_small + A.batch - 1) / A.batch;

  // the next work index is fetched one item ahead so the atomic's latency
  // overlaps the current item's arithmetic
  unsigned long long wnext = 0;
  if (lane == 0) wnext = atomicAdd(A.s.counter, 1ull);
  for (;;) {
    const int64_t w = (int64_t)__shfl(wnext, 0);
    if (w >= total) break;
    if (lane == 0) wnext = atomicAdd(A.s.counter, 1ull);

    if (w < big_total) {
      // one item of a big pair: position with big_prefix[pos] <= w < big_prefix[pos + 1]
      int64_t lo = 0, hi = n_big;
      while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (A.s.big_prefix[mid] <= w)
          lo = mid;
        else
          hi = mid;
      }
      const WorkRec r = A.s.big[lo];
      const Layout L = layout<R>(r, w - A.s.big_prefix[lo], A.chunk, lane);
      V3<Tc> kv[R + 1];
      load_b<Tin, Tc, R>(X, r, L, kv);
      Segs<Tc, R> sg;
      make_segs<Tc, R>(kv, L, sg);
      Walk<Tc, R> wk;
      double acc = 0.0;
      for (int t0 = 0; t0 < L.nah; t0 += A.tile) {
        const int tl = (L.nah - t0) < A.tile ? (L.nah - t0) : A.tile;
        __syncthreads();
        for (int v = lane; v <= tl; v += kWave) {
          int64_t idx = L.a0 + t0 + v;
          if (idx >= r.na) idx -= r.na;  // closing vertex of the loop
          const V3<Tc> x = load_vertex<Tc>(X, r.oa + idx);
          lds[v] = Vtx<Tc>{x.x, x.y, x.z, (Tc)0};
        }
        __syncthreads();
        const int jlo = L.js > t0 ? L.js : t0;
        const int jhi = L.je < t0 + tl ? L.je : t0 + tl;
        if (L.active && jlo < jhi) walk_tile<Tc, AT, R>(lds, t0, jlo, jhi, L.js, wk, sg, acc);
      }
      finish_item(acc, r.p, lane, A, r.items == 1);
    } else {
      // a batch of small pairs (one item each, loop A of at most kSmallA - 1
      // segments): records are read once per batch, and the next pair's
      // vertices are loaded into registers while the current pair computes
      const int64_t m0 = (w - big_total) * (int64_t)A.batch;
      const int cnt = (int)((n_small - m0) < A.batch ? (n_small - m0) : A.batch);
      WorkRec mine{};
      if (lane < cnt) mine = A.s.small[m0 + lane];
      WorkRec cur = shfl_rec(mine, 0);
      Layout L = layout<R>(cur, 0, A.chunk, lane);
      V3<Tc> kv[R + 1], a_lo, a_hi;
      load_b<Tin, Tc, R>(X, cur, L, kv);
      a_lo = load_vertex<Tc>(X, cur.oa + (lane < cur.na ? lane : 0));
      a_hi = load_vertex<Tc>(X, cur.oa + (lane + kWave < cur.na ? lane + kWave : 0));
      for (int m = 0; m < cnt; ++m) {
        __syncthreads();
        if (lane <= cur.na) lds[lane] = Vtx<Tc>{a_lo.x, a_lo.y, a_lo.z, (Tc)0};
        if (lane + kWave <= cur.na) lds[lane + kWave] = Vtx<Tc>{a_hi.x, a_hi.y, a_hi.z, (Tc)0};
        Segs<Tc, R> sg;
        make_segs<Tc, R>(kv, L, sg);
        const Layout Lc = L;
        const int32_t pc = cur.p;
        if (m + 1 < cnt) {
          cur = shfl_rec(mine, m + 1);
          L = layout<R>(cur, 0, A.chunk, lane);
          load_b<Tin, Tc, R>(X, cur, L, kv);
          a_lo = load_vertex<Tc>(X, cur.oa + (lane < cur.na ? lane : 0));
          a_hi = load_vertex<Tc>(X, cur.oa + (lane + kWave < cur.na ? lane + kWave : 0));
        }
        __syncthreads();
        Walk<Tc, R> wk;
        double acc = 0.0;
        if (Lc.active && Lc.js < Lc.je) walk_tile<Tc, AT, R>(lds, 0, Lc.js, Lc.je, Lc.js, wk, sg, acc);
        finish_item(acc, pc, lane, A, true);
      }
    }
  }
}

template <typename Tc>
size_t lds_bytes(int tile) {
  const int n = tile + 1 > kSmallA ? tile + 1 : kSmallA;
  return (size_t)n * sizeof(Vtx<Tc>);
}

template <typename Tin, typename Tc, int AT, int R>
hipError_t launch_t(const DsArgs& a, int grid, hipStream_t s) {
  const size_t shm = lds_bytes<Tc>(a.tile);
  ds_persistent<Tin, Tc, AT, R><<<dim3(grid), dim3(kWave), shm, s>>>(a);
  return hipGetLastError();
}

template <typename Tin, typename Tc, int AT, int R>
int grid_t(int tile, int n_cu, int waves_per_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ds_persistent<Tin, Tc, AT, R>, kWave,
                                                   lds_bytes<Tc>(tile)) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (waves_per_cu > 0 && waves_per_cu < per_cu) per_cu = waves_per_cu;
  return per_cu * n_cu;
}

// Kernel variants: input type x arithmetic x arctangent form x segments per lane.
struct Variant {
  hipError_t (*launch)(const DsArgs&, int, hipStream_t);
  int (*grid)(int, int, int);
};

template <typename Tin, typename Tc, int AT, int R>
constexpr Variant variant() {
  return Variant{launch_t<Tin, Tc, AT, R>, grid_t<Tin, Tc, AT, R>};
}

Variant pick(bool in_f64, bool compute_f64, int atan_form, int segs) {
  if (compute_f64) {
    if (segs >= 2) return in_f64 ? variant<double, double, 0, 2>() : variant<float, double, 0, 2>();
    return in_f64 ? variant<double, double, 0, 1>() : variant<float, double, 0, 1>();
  }
  if (atan_form == 1) {
    if (segs >= 4) return in_f64 ? variant<double, float, 1, 4>() : variant<float, float, 1, 4>();
    if (segs >= 2) return in_f64 ? variant<double, float, 1, 2>() : variant<float, float, 1, 2>();
    return in_f64 ? variant<double, float, 1, 1>() : variant<float, float, 1, 1>();
  }
  if (segs >= 4) return in_f64 ? variant<double, float, 0, 4>() : variant<float, float, 0, 4>();
  if (segs >= 2) return in_f64 ? variant<double, float, 0, 2>() : variant<float, float, 0, 2>();
  return in_f64 ? variant<double, float, 0, 1>() : variant<float, float, 0, 1>();
}

}  // namespace

int segs_supported(bool compute_f64, int segs) {
  if (compute_f64) return segs >= 2 ? 2 : 1;
  return segs >= 4 ? 4 : (segs >= 2 ? 2 : 1);
}

hipError_t launch_direct_sum(const DsArgs& a, bool in_f64, bool compute_f64, int atan_form,
                             int segs, int grid, hipStream_t s) {
  return pick(in_f64, compute_f64, atan_form, segs).launch(a, grid, s);
}

int direct_sum_grid(bool in_f64, bool compute_f64, int atan_form, int segs, int tile, int n_cu,
                    int waves_per_cu) {
  return pick(in_f64, compute_f64, atan_form, segs).grid(tile, n_cu, waves_per_cu);
}

}  // namespace lk
