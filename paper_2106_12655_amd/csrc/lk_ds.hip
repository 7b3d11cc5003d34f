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

// Segment of loop B owned by a lane.
template <typename T>
struct Seg {
  V3<T> k0, k1, s;  // k_i, k_{i+1}, s_i = k_{i+1} - k_i
};

// Walk state at vertex l_j of loop A.
template <typename T>
struct Walk {
  V3<T> l;     // l_j
  V3<T> a, b;  // l_j - k_i, l_j - k_{i+1}
  T na, nb, e; // |a|, |b|, |a||b| + a.b
};

template <typename T>
__device__ __forceinline__ void walk_init(Walk<T>& w, const V3<T>& l, const Seg<T>& g) {
  w.l = l;
  w.a = l - g.k0;
  w.b = l - g.k1;
  w.na = fsqrt(dot(w.a, w.a));
  w.nb = fsqrt(dot(w.b, w.b));
  w.e = w.na * w.nb + dot(w.a, w.b);
}

// One Eq. 4 term for segment (l_j, l_{j+1}) against the lane's segment;
// returns 2 pi times the term and advances the walk to l_{j+1}.
template <typename T, int AT>
__device__ __forceinline__ T walk_step(Walk<T>& w, const V3<T>& l1, const Seg<T>& g) {
  const V3<T> c = l1 - g.k1;
  const V3<T> d = l1 - g.k0;
  const T nc = fsqrt(dot(c, c));
  const T nd = fsqrt(dot(d, d));
  const V3<T> sj = l1 - w.l;
  const T p = dot(w.a, cross(sj, g.s));
  const T bc = dot(w.b, c);
  const T ca = dot(c, w.a);
  const T ad = dot(w.a, d);
  const T f = nd * nc + dot(d, c);
  const T d1 = nc * w.e + bc * w.na + ca * w.nb;
  const T d2 = w.na * f + ad * nc + ca * nd;
  const T th = angle<T, AT>(p * (d1 + d2), d1 * d2 - p * p);
  w.l = l1;
  w.a = d;
  w.b = c;
  w.na = nd;
  w.nb = nc;
  w.e = f;
  return th;
}

// 128-bit two's-complement fixed point with 64 fraction bits, accumulated with
// 64-bit integer atomics: integer addition is associative, so the pair sum is
// the same whatever order the work items finish in.  Bits below 2^-64 of each
// item's partial are dropped (deterministically).
__device__ __forceinline__ void fixed_add(unsigned long long* acc, double v) {
  const double fl = floor(v);
  const long long hi = (long long)fl;
  const double fr = v - fl;  // exact, in [0, 1)
  const unsigned long long lo = (unsigned long long)(fr * 18446744073709551616.0);
  const unsigned long long old = atomicAdd(&acc[0], lo);
  const unsigned long long carry = (old + lo < old) ? 1ull : 0ull;
  atomicAdd(&acc[1], (unsigned long long)hi + carry);
}

template <typename Tin, typename Tc, int AT>
__global__ __launch_bounds__(kWave) void ds_persistent(DsArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Vtx<Tc>* lds = reinterpret_cast<Vtx<Tc>*>(lds_raw);
  const int lane = threadIdx.x;
  const Tin* X = static_cast<const Tin*>(A.xyz);
  int64_t n_list = A.n_list;
  if (A.n_list_dev) {
    const int64_t nd = *A.n_list_dev;
    n_list = nd < n_list ? nd : n_list;
  }
  const int64_t total = A.prefix[n_list];

  for (;;) {
    unsigned long long wi = 0;
    if (lane == 0) wi = atomicAdd(A.counter, 1ull);
    const int64_t w = (int64_t)__shfl(wi, 0);
    if (w >= total) break;

    // list position q with prefix[q] <= w < prefix[q + 1]
    int64_t lo = 0, hi = n_list;
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (A.prefix[mid] <= w)
        lo = mid;
      else
        hi = mid;
    }
    const int64_t q = lo;
    const int32_t p = A.list ? A.list[q] : (int32_t)q;
    const int32_t ia = A.pairs[2 * p], ib = A.pairs[2 * p + 1];
    const int64_t oa = A.off[ia], na = A.off[ia + 1] - oa;
    const int64_t ob = A.off[ib], nb = A.off[ib + 1] - ob;
    const int64_t local = w - A.prefix[q];
    const int64_t nbb = (nb + kBlockB - 1) / kBlockB;
    const int64_t b0 = (local % nbb) * kBlockB;
    const int64_t a0 = (local / nbb) * (int64_t)A.chunk;
    const int nbh = (int)((nb - b0) < kBlockB ? (nb - b0) : kBlockB);
    const int nah = (int)((na - a0) < A.chunk ? (na - a0) : A.chunk);
    const int groups = kWave / nbh;
    const int bi = lane % nbh;
    const int g = lane / nbh;
    const bool active = g < groups;
    const int js = (int)(((int64_t)nah * g) / groups);
    const int je = (int)(((int64_t)nah * (g + 1)) / groups);

    Seg<Tc> sg;
    {
      const int64_t i0 = b0 + bi;
      const int64_t i1 = (i0 + 1 == nb) ? 0 : i0 + 1;
      sg.k0 = load_vertex<Tc>(X, ob + i0);
      sg.k1 = load_vertex<Tc>(X, ob + i1);
      sg.s = sg.k1 - sg.k0;
    }
    Walk<Tc> wk;
    double acc = 0.0;
    for (int t0 = 0; t0 < nah; t0 += A.tile) {
      const int tl = (nah - t0) < A.tile ? (nah - t0) : A.tile;
      __syncthreads();
      for (int v = lane; v <= tl; v += kWave) {
        int64_t idx = a0 + t0 + v;
        if (idx >= na) idx -= na;  // closing vertex of the loop
        const V3<Tc> x = load_vertex<Tc>(X, oa + idx);
        lds[v] = Vtx<Tc>{x.x, x.y, x.z, (Tc)0};
      }
      __syncthreads();
      const int jlo = js > t0 ? js : t0;
      const int jhi = je < t0 + tl ? je : t0 + tl;
      Tc part = 0;
      if (active && jlo < jhi) {
        if (jlo == js) {
          const Vtx<Tc> v0 = lds[jlo - t0];
          walk_init(wk, V3<Tc>{v0.x, v0.y, v0.z}, sg);
        }
#pragma unroll 4
        for (int j = jlo; j < jhi; ++j) {
          const Vtx<Tc> v1 = lds[j - t0 + 1];
          part += walk_step<Tc, AT>(wk, V3<Tc>{v1.x, v1.y, v1.z}, sg);
        }
      }
      acc += (double)part;
    }
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) {
      const double v = acc * kInvTwoPi;
      if (fabs(v) < 1.0e15)
        fixed_add(&A.acc[2 * (int64_t)p], v);
      else
        atomicOr(&A.flags[p], 4u);  // NaN / Inf / absurd magnitude
    }
  }
}

template <typename Tin, typename Tc, int AT>
size_t lds_bytes(int tile) {
  return (size_t)(tile + 1) * sizeof(Vtx<Tc>);
}

template <typename Tin, typename Tc, int AT>
hipError_t launch_t(const DsArgs& a, int grid, hipStream_t s) {
  const size_t shm = lds_bytes<Tin, Tc, AT>(a.tile);
  ds_persistent<Tin, Tc, AT><<<dim3(grid), dim3(kWave), shm, s>>>(a);
  return hipGetLastError();
}

template <typename Tin, typename Tc, int AT>
int grid_t(int tile, int n_cu, int waves_per_cu) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ds_persistent<Tin, Tc, AT>, kWave,
                                                   lds_bytes<Tin, Tc, AT>(tile)) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (waves_per_cu > 0 && waves_per_cu < per_cu) per_cu = waves_per_cu;
  return per_cu * n_cu;
}

}  // namespace

hipError_t launch_direct_sum(const DsArgs& a, bool in_f64, bool compute_f64, int atan_form,
                             int grid, hipStream_t s) {
  if (compute_f64) {
    return in_f64 ? launch_t<double, double, 0>(a, grid, s) : launch_t<float, double, 0>(a, grid, s);
  }
  if (atan_form == 1)
    return in_f64 ? launch_t<double, float, 1>(a, grid, s) : launch_t<float, float, 1>(a, grid, s);
  return in_f64 ? launch_t<double, float, 0>(a, grid, s) : launch_t<float, float, 0>(a, grid, s);
}

int direct_sum_grid(bool in_f64, bool compute_f64, int atan_form, int tile, int n_cu,
                    int waves_per_cu) {
  if (compute_f64)
    return in_f64 ? grid_t<double, double, 0>(tile, n_cu, waves_per_cu)
                  : grid_t<float, double, 0>(tile, n_cu, waves_per_cu);
  if (atan_form == 1)
    return in_f64 ? grid_t<double, float, 1>(tile, n_cu, waves_per_cu)
                  : grid_t<float, float, 1>(tile, n_cu, waves_per_cu);
  return in_f64 ? grid_t<double, float, 0>(tile, n_cu, waves_per_cu)
                : grid_t<float, float, 0>(tile, n_cu, waves_per_cu);
}

}  // namespace lk
