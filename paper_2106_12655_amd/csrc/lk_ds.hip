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
// segment j+1 are d and c of segment j, so each step needs only the new
// vertex-pair vectors v_r = l_{j+1} - k_r of the lane's vertices, their norms
// and their dot products with the previous ones; the other dot products of
// Eq. 4 follow from carried ones and the lane's segment vectors s_r:
//   c . a = (d - s_r) . a = a . d - s_r . a      (s_r . a carried from the
//                                                  previous step's s_r . d)
//   d . c = d . (d - s_r) = |d|^2 - s_r . d
// The common numerator of both arctangents is p = a . (s_j x s_r) (equal to
// a . (b x c) and c . (d x a) in exact arithmetic, Sec. 3.4.2).  With the
// lane's first vertex k_0 as a local origin, a = V_0 - delta_r where
// V_0 = l_j - k_0 and delta_r = k_r - k_0, so
//   p = s_r . (V_0 x s_j) - s_j . (s_r x delta_r)
// with one cross product per step shared by the lane's R segments and a
// per-lane constant s_r x delta_r; both pieces are built from short vectors,
// which keeps FP32 accurate for distant pairs.  The two arctangents are merged
// into one: (d1 + i p)(d2 + i p) has the angle atan2(p, d1) + atan2(p, d2)
// (the angle-addition idea of the appendix, Alg. 7, applied per term).  Every
// difference vector l(s) - k(t) of the two segments has the same component p
// along s_j x s_r, so the pair's quadrilateral lies in one open hemisphere:
// the angle stays inside (-pi, pi) and has the sign of p, which makes
// d1 + d2 > 0 in exact arithmetic.  Near contact with the crossing close to
// the diagonal a-c both d1 and d2 shrink and their FP32 sum carries no sign,
// so the sign is taken from p (which stays accurate there) and only the
// magnitude from the merged form:
//   theta = atan2(p |d1 + d2|, d1 d2 - p^2),  term = theta / (2 pi)
// The magnitude's error near contact grows like eps |s| / h (h the distance
// of the segments); it stays below 0.5 per term and is caught by the refit
// rule long before h reaches the resolution of the coordinates.
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

__device__ __forceinline__ float fabs_t(float a) { return __builtin_fabsf(a); }
__device__ __forceinline__ double fabs_t(double a) { return __builtin_fabs(a); }
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// FP64 square root from the hardware reciprocal-square-root estimate and two
// Goldschmidt iterations (s -> sqrt(x), h -> 1 / (2 sqrt(x))), then one
// Newton correction on the residual x - s^2.  No range scaling: arguments
// are squared distances of geometry, far from the FP64 limits; x = 0 gives
// NaN, which only happens for coincident vertices (a degenerate pair, flagged).
__device__ __forceinline__ double fsqrt(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double s = x * y, h = 0.5 * y;
  double r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  r = fma(-s, h, 0.5);
  s = fma(s, r, s);
  h = fma(h, r, h);
  return fma(fma(-s, s, x), h, s);
}

// Own FP32 arctangent: octant reduction to t = min/max in [0, 1], then
// atan(t) = t q(t^2) with q the Remez minimax polynomial of atan_poly.h.
// (0, 0) gives NaN on purpose: it only arises for touching segments.
// atan2_reduced takes t = min(|x|, |y|) / max(|x|, |y|) already formed.
__device__ __forceinline__ float atan2_reduced(float y, float x, float t) {
  const float ax = fabsf(x), ay = fabsf(y);
  const float s = t * t;
  float q = kAtanQ[LK_ATAN_DEG];
#pragma unroll
  for (int k = LK_ATAN_DEG - 1; k >= 0; --k) q = fmaf(q, s, kAtanQ[k]);
  float r = t * q;
  r = (ay > ax) ? (1.57079632679489662f - r) : r;
  r = (x < 0.0f) ? (3.14159265358979324f - r) : r;
  return copysignf(r, y);
}

__device__ __forceinline__ float atan2_minimax(float y, float x) {
  const float ax = fabsf(x), ay = fabsf(y);
  return atan2_reduced(y, x, fminf(ax, ay) * __builtin_amdgcn_rcpf(fmaxf(ax, ay)));
}

// Own FP64 arctangent: the same octant reduction, t = min/max from the
// hardware reciprocal estimate with two Newton steps and a residual
// correction (no IEEE division sequence), and the degree-19 polynomial of
// atan_poly.h (relative error 2.5e-16 in FP64 Horner form).
__device__ __forceinline__ double atan2_f64(double y, double x) {
  const double ax = fabs(x), ay = fabs(y);
  const double mx = fmax(ax, ay), mn = fmin(ax, ay);
  double r = __builtin_amdgcn_rcp(mx);
  r = fma(r, fma(-mx, r, 1.0), r);
  r = fma(r, fma(-mx, r, 1.0), r);
  const double q = mn * r;
  const double t = fma(fma(-mx, q, mn), r, q);
  const double s = t * t;
  double p = kAtanQ64[LK_ATAN_DEG64];
#pragma unroll
  for (int k = LK_ATAN_DEG64 - 1; k >= 0; --k) p = fma(p, s, kAtanQ64[k]);
  double a = t * p;
  a = (ay > ax) ? (1.57079632679489661923 - a) : a;
  a = (x < 0.0) ? (3.14159265358979323846 - a) : a;
  return copysign(a, y);
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
  return atan2_f64(y, x);
}
template <>
__device__ __forceinline__ double angle<double, 1>(double y, double x) {
  return atan2(y, x);
}
template <>
__device__ __forceinline__ float angle<float, 2>(float y, float x) {
  return atan2_minimax(y, x);
}
template <>
__device__ __forceinline__ double angle<double, 2>(double y, double x) {
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

// Vertex loads of one work item.  An FP32 pass over FP64 input takes every
// coordinate relative to an origin inside the item (a vertex of its loop-B
// block), subtracted in FP64 before the rounding to FP32: the FP32 values
// then carry relative precision against the item's own extent, not against
// the distance from the coordinate origin (2^-24 of 1e3 is 6e-5, enough to
// move a near contact across its partner).  The terms only use differences
// of vertices, which the shift leaves unchanged in exact arithmetic.  FP32
// input, and FP64 passes, load the values as stored.
template <typename Tin, typename Tc>
struct Frame {
  static constexpr bool kShift = sizeof(Tin) > sizeof(Tc);
  Tin ox = 0, oy = 0, oz = 0;
  __device__ __forceinline__ void set(const Tin* X, int64_t v) {
    if constexpr (kShift) {
      ox = X[3 * v];
      oy = X[3 * v + 1];
      oz = X[3 * v + 2];
    }
  }
  __device__ __forceinline__ V3<Tc> load(const Tin* X, int64_t v) const {
    if constexpr (kShift)
      return {(Tc)(X[3 * v] - ox), (Tc)(X[3 * v + 1] - oy), (Tc)(X[3 * v + 2] - oz)};
    else
      return load_vertex<Tc>(X, v);
  }
};

// The R consecutive segments of loop B owned by a lane: vertices k_0..k_R,
// segment vectors s_r = k_{r+1} - k_r and the constants s_r x (k_r - k_0) of
// the numerator p.  Segments past the end of the item have zero length
// (repeated vertices) and add exactly 0.
template <typename T, int R>
struct Segs {
  V3<T> k[R + 1];
  V3<T> s[R];
  V3<T> m[R];
};

// Walk state at vertex l_j of loop A, for all R + 1 vertices of the lane:
// V_r = l_j - k_r, N_r = |V_r|, E_r = N_r N_{r+1} + V_r . V_{r+1},
// G_r = s_r . V_r.
template <typename T, int R>
struct Walk {
  V3<T> l;
  V3<T> V[R + 1];
  T N[R + 1];
  T E[R];
  T G[R];
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
  for (int r = 0; r < R; ++r) {
    w.E[r] = w.N[r] * w.N[r + 1] + dot(w.V[r], w.V[r + 1]);
    w.G[r] = dot(g.s[r], w.V[r]);
  }
}

// The Eq. 4 terms of segment (l_j, l_{j+1}) against the lane's R segments;
// returns 2 pi times their (masked) sum and advances the walk to l_{j+1}.
// For segment r: a = V_r, b = V_{r+1} (at l_j), c = v_{r+1}, d = v_r (at
// l_{j+1}); a.b enters through E_r, and the "vertical" products V_r . v_r are
// shared by segments r - 1 and r.
template <typename T, int AT, int R>
__device__ __forceinline__ T walk_step(Walk<T, R>& w, const V3<T>& l1, const Segs<T, R>& g) {
  V3<T> v[R + 1];
  T n2[R + 1], n[R + 1], vert[R + 1];
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    v[r] = l1 - g.k[r];
    n2[r] = dot(v[r], v[r]);
    n[r] = fsqrt(n2[r]);
    vert[r] = dot(w.V[r], v[r]);
  }
  const V3<T> sj = l1 - w.l;
  const V3<T> M = cross(w.V[0], sj);
  T X[R], Y[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const T na = w.N[r], nb = w.N[r + 1], nc = n[r + 1], nd = n[r];
    const T gr = dot(g.s[r], v[r]);
    // p = s_r . M - s_j . m_r as one fused chain (the subtraction folded into
    // the first product's addend)
    T p = dot(g.s[r], M);
    if (r > 0) {
      const V3<T>& m = g.m[r];
      p = fmad(g.s[r].x, M.x, fmad(g.s[r].y, M.y, fmad(g.s[r].z, M.z, -dot(sj, m))));
    }
    const T ca = vert[r] - w.G[r];
    const T f = nd * nc + (n2[r] - gr);
    const T d1 = nc * w.E[r] + vert[r + 1] * na + ca * nb;
    const T d2 = na * f + vert[r] * nc + ca * nd;
    Y[r] = p * fabs_t(d1 + d2);  // |.| is a free source modifier
    X[r] = d1 * d2 - p * p;
    w.E[r] = f;
    w.G[r] = gr;
  }
  T sum = 0;
  if constexpr (AT == 0 && sizeof(T) == 4) {
    // the R arctangents in phases (all reciprocals issued together, then the
    // polynomials), which lets the transcendental unit run back to back
    T mx[R], mn[R], inv[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      mx[r] = fmaxf(fabsf(X[r]), fabsf(Y[r]));
      mn[r] = fminf(fabsf(X[r]), fabsf(Y[r]));
    }
#pragma unroll
    for (int r = 0; r < R; ++r) inv[r] = __builtin_amdgcn_rcpf(mx[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) sum += atan2_reduced(Y[r], X[r], mn[r] * inv[r]);
  } else {
#pragma unroll
    for (int r = 0; r < R; ++r) sum += angle<T, AT>(Y[r], X[r]);
  }
  w.l = l1;
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    w.V[r] = v[r];
    w.N[r] = n[r];
  }
  return sum;
}

// Where the lanes of one work item sit: B block [b0, b0 + nbh) of loop B split
// into `slots` lanes of R segments; if that leaves lanes over, they form
// `groups` that split the item's A range [a0, a0 + nah) into [js, je).
struct Layout {
  int64_t b0, a0;
  int nbh, nah, bi, js, je;
  bool active;
};

// 32-bit arithmetic throughout: the plan guarantees fewer than 2^31 items per
// pair and 2^31 vertices per loop, and js/je products stay below 2^30
// (chunk <= 2^24, 64 groups).  `width`: lanes given to the item (a power of
// two dividing 64; `lane` counts within them).
template <int R>
__device__ __forceinline__ Layout layout(const WorkRec& r, int64_t local, int chunk, int lane,
                                         unsigned width = kWave) {
  constexpr unsigned kB = kWave * R;
  Layout L;
  const unsigned nbb = ((unsigned)r.nb + kB - 1) / kB;
  const unsigned loc = (unsigned)local;
  const unsigned bq = loc / nbb;
  L.b0 = (int64_t)((loc - bq * nbb) * kB);
  L.a0 = (int64_t)bq * chunk;
  L.nbh = (int)((r.nb - L.b0) < kB ? (r.nb - L.b0) : kB);
  L.nah = (int)((r.na - L.a0) < chunk ? (r.na - L.a0) : chunk);
  const unsigned slots = ((unsigned)L.nbh + R - 1) / R;
  const unsigned groups = slots <= width ? width / slots : 1u;
  const unsigned g = (unsigned)lane / slots;
  L.bi = (int)((unsigned)lane - g * slots);
  L.active = g < groups;
  L.js = (int)(((unsigned)L.nah * g) / groups);
  L.je = (int)(((unsigned)L.nah * (g + 1)) / groups);
  return L;
}

// Vertex k_{b0 + bi R + r} of loop B for r = 0..R (cyclic).  Past the end
// of the block the lane repeats the block's end vertex, so its padding
// segments have zero length: their Eq. 4 term is exactly 0 (p = 0 and
// d1 d2 > 0 unless a vertex of loop A sits on that vertex, which only
// touching loops do), and the sum needs no mask.  The crossing count still
// masks them (Segs::valid), since a zero-length segment has no certain side.
template <typename Tin, typename Tc, int R>
__device__ __forceinline__ void load_b(const Tin* X, const WorkRec& w, const Layout& L,
                                       const Frame<Tin, Tc>& F, V3<Tc>* k) {
  const int first = L.bi * R;
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    int64_t i = L.b0 + (first + r < L.nbh ? first + r : L.nbh);
    if (i >= w.nb) i -= w.nb;
    k[r] = F.load(X, w.ob + i);
  }
}

template <typename Tc, int R>
__device__ __forceinline__ void make_segs(const V3<Tc>* k, Segs<Tc, R>& sg) {
#pragma unroll
  for (int r = 0; r <= R; ++r) sg.k[r] = k[r];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    sg.s[r] = sg.k[r + 1] - sg.k[r];
    sg.m[r] = cross(sg.s[r], sg.k[r] - sg.k[0]);
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
  // four steps are summed in the compute type before the FP64 lane sum
  int j = jlo;
  for (; j + 4 <= jhi; j += 4) {
    Tc s4 = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const Vtx<Tc> v1 = lds[j + q - t0 + 1];
      s4 += walk_step<Tc, AT, R>(wk, V3<Tc>{v1.x, v1.y, v1.z}, sg);
    }
    acc += (double)s4;
  }
  for (; j < jhi; ++j) {
    const Vtx<Tc> v1 = lds[j - t0 + 1];
    acc += (double)walk_step<Tc, AT, R>(wk, V3<Tc>{v1.x, v1.y, v1.z}, sg);
  }
}

// ---------------------------------------------------------------------------
// Count Crossings (Sec. 2.1, Alg. 4): the linking number is half the signed
// number of crossings of a regular projection.  The projection is along a view
// direction n (uniform over the launch).  Two projected segments cross iff the
// endpoints of each lie strictly on opposite sides of the other's line.  The
// side of a point x relative to the projected line through y with direction e
// is the sign of (x - y) . (n x e), so no coordinate is rotated: a step forms
// u = n x s_j once and every lane holds t_r = n x s_r.  With v_r = l_{j+1} - k_r:
//   side of k_r      w.r.t. segment j's line:  w_r = v_r . u
//   side of l_{j+1}  w.r.t. segment r's line:  q_r = v_r . t_r
// (the side of l_j is the previous step's q_r).  At a crossing the points of
// the two segments over the crossing differ by h n, so the Eq. 4 numerator
// p = a . (s_j x s_r) = v_r . (s_j x s_r) = h n . (s_j x s_r) has the sign of
// the crossing (over tangent x under tangent, against n); the count sums
// sign(p) and the pair's value is half of it.
//
// Every predicate is certified in FP32 on the vertices as given: a value
// counts only when its magnitude exceeds a forward error bound of the form
// tau |first|_inf |second|_inf (about 63 u for w and q, 216 u for p with the
// unit roundoff u = 2^-24, from first-order error analysis of the differences,
// the cross products and the dot products; tau defaults to twice that).  A
// term that is neither certainly crossing nor certainly not crossing, or an
// odd total, makes the pair's value NaN or a half-integer, and the pair is
// counted again by this kernel in FP64 (Tc = double, bounds at u = 2^-53):
// the depth separation of two segments enters |v| but not the side values,
// so at shallow crossings of curves far apart in depth the FP32 bound is
// loose while FP64 decides.  Only a pair that FP64 cannot decide either -- a
// crossing within about 1e-16 of a vertex, overlapping projected segments,
// segments that touch in space -- goes to the FP64 direct sum.  Needs
// |n|_inf <= 1 (the runtime scales n so).
constexpr int kCrossings = 3;  // term form of the kernel's template: crossing count

template <typename T, int R>
struct CcSegs {
  V3<T> k[R + 1];
  V3<T> t[R];    // n x s_r
  T cq[R];       // tau |s_r|_inf: certainty scale of q_r
  T sn[R];       // |s_r|_inf
  V3<T> n;       // view direction
  T tau, tau_p;
  bool valid[R];
};

// Walk state at l_j: the vertex and the certified sides of l_j relative to
// the lane's R segment lines (0 = uncertain).
template <typename T, int R>
struct CcWalk {
  V3<T> l;
  T Q[R];
};

template <typename T>
__device__ __forceinline__ T inf_norm(const V3<T>& a) {
  return fmax(fmax(fabs(a.x), fabs(a.y)), fabs(a.z));
}

// x if |x| > tol, else 0 (the sign survives only when it is certain; NaN -> 0)
template <typename T>
__device__ __forceinline__ T certain(T x, T tol) {
  return fabs(x) > tol ? x : (T)0;
}

template <typename Tc, int R>
__device__ __forceinline__ void make_lane(const V3<Tc>* k, const Layout& L, const DsArgs& A,
                                          CcSegs<Tc, R>& sg) {
  const int first = L.bi * R;
  sg.n = V3<Tc>{A.view[0], A.view[1], A.view[2]};
  sg.tau = (Tc)A.cc_tau;
  sg.tau_p = (Tc)A.cc_tau_p;
#pragma unroll
  for (int r = 0; r <= R; ++r) sg.k[r] = k[r];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const V3<Tc> s = sg.k[r + 1] - sg.k[r];
    sg.t[r] = cross(sg.n, s);
    sg.sn[r] = inf_norm(s);
    sg.cq[r] = sg.tau * sg.sn[r];
    sg.valid[r] = first + r < L.nbh;
  }
}

template <typename Tc, int R>
__device__ __forceinline__ void cc_init(CcWalk<Tc, R>& w, const V3<Tc>& l, const CcSegs<Tc, R>& g) {
  w.l = l;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const V3<Tc> V = l - g.k[r];
    w.Q[r] = certain(dot(V, g.t[r]), g.cq[r] * inf_norm(V));
  }
}

// One step l_j -> l_{j+1} against the lane's R segments: adds the certified
// crossing signs to cnt, sets bad when a term is undecided.
template <typename Tc, int R>
__device__ __forceinline__ void cc_step(CcWalk<Tc, R>& w, const V3<Tc>& l1, const CcSegs<Tc, R>& g,
                                        int& cnt, bool& bad) {
  const V3<Tc> sj = l1 - w.l;
  const V3<Tc> u = cross(g.n, sj);
  const Tc sjn = inf_norm(sj);
  const Tc cw = g.tau * sjn;
  V3<Tc> v[R + 1];
  Tc nv[R + 1], wc[R + 1];
#pragma unroll
  for (int r = 0; r <= R; ++r) {
    v[r] = l1 - g.k[r];
    nv[r] = inf_norm(v[r]);
    wc[r] = certain(dot(v[r], u), cw * nv[r]);
  }
  Tc Wp[R], Qp[R];
  bool cand[R];
  bool any = false;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const Tc qc = certain(dot(v[r], g.t[r]), g.cq[r] * nv[r]);
    Wp[r] = wc[r] * wc[r + 1];  // < 0: k_r, k_{r+1} certainly on opposite sides
    Qp[r] = w.Q[r] * qc;        // < 0: l_j, l_{j+1} certainly on opposite sides
    w.Q[r] = qc;
    // either product certainly positive: certainly no crossing
    cand[r] = g.valid[r] && !(fmax(Wp[r], Qp[r]) > (Tc)0);
    any = any || cand[r];
  }
  w.l = l1;
  if (any) {  // rare: a crossing or an undecided term somewhere in the lane
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!cand[r]) continue;
      const V3<Tc> s = g.k[r + 1] - g.k[r];
      const Tc p = dot(v[r], cross(sj, s));
      const Tc tp = g.tau_p * g.sn[r] * sjn * nv[r];
      if (Wp[r] < (Tc)0 && Qp[r] < (Tc)0 && fabs(p) > tp) {
        cnt += p > (Tc)0 ? 1 : -1;
      } else {
        bad = true;
      }
    }
  }
}

template <typename Tc, int AT, int R>
__device__ __forceinline__ void walk_tile(const Vtx<Tc>* lds, int t0, int jlo, int jhi, int js,
                                          CcWalk<Tc, R>& wk, const CcSegs<Tc, R>& sg,
                                          double& acc) {
  if (jlo == js) {
    const Vtx<Tc> v0 = lds[jlo - t0];
    cc_init(wk, V3<Tc>{v0.x, v0.y, v0.z}, sg);
  }
  int cnt = 0;
  bool bad = false;
#pragma unroll 2
  for (int j = jlo; j < jhi; ++j) {
    const Vtx<Tc> v1 = lds[j - t0 + 1];
    cc_step(wk, V3<Tc>{v1.x, v1.y, v1.z}, sg, cnt, bad);
  }
  acc += bad ? __builtin_nan("") : (double)cnt;
}

// One work item of the crossing count with culling: the item's B block (R
// blocks of 64 segments) has a projected box; loop A's superblocks and then
// blocks whose boxes are disjoint from it are skipped, and every other block
// is staged (65 vertices) and walked from a fresh start.  The box tests are
// uniform over the wave.
template <typename Tin, typename Tc, int R>
__device__ __forceinline__ void cc_item_culled(const DsArgs& A, const Tin* X,
                                               const Frame<Tin, Tc>& F, Vtx<Tc>* lds,
                                               const WorkRec& r, const Layout& L, int lane,
                                               CcWalk<Tc, R>& wk, const CcSegs<Tc, R>& sg,
                                               double& acc) {
  const int32_t ia = A.pairs[2 * (int64_t)r.p], ib = A.pairs[2 * (int64_t)r.p + 1];
  const int64_t o0 = A.off[0];
  const int64_t bslot = (r.ob - o0) / kCcBlock + ib + L.b0 / kCcBlock;
  float4 bb = float4{INFINITY, -INFINITY, INFINITY, -INFINITY};
  bool bok = true;
#pragma unroll
  for (int c = 0; c < R; ++c) {
    if (L.b0 + (int64_t)c * kCcBlock < r.nb) {
      if ((uint64_t)(bslot + c) < (uint64_t)A.cc_nblk) {
        const float4 q = A.cc_blk[bslot + c];
        bb = float4{fminf(bb.x, q.x), fmaxf(bb.y, q.y), fminf(bb.z, q.z), fmaxf(bb.w, q.w)};
      } else {
        bok = false;
      }
    }
  }
  if (!bok) bb = float4{-INFINITY, INFINITY, -INFINITY, INFINITY};  // no box: cull nothing
  const int64_t ablk = (r.oa - o0) / kCcBlock + ia;
  const int64_t asup = (r.oa - o0) / kCcSuper + ia;
  const int a0 = (int)L.a0, a_end = (int)L.a0 + L.nah;
  const int lo_l = a0 + L.js, hi_l = a0 + L.je;  // this lane's segments of A
  for (int sp = a0 / kCcSuper; sp * kCcSuper < a_end; ++sp) {
    if ((uint64_t)(asup + sp) < (uint64_t)A.cc_nsup && boxes_disjoint(A.cc_sup[asup + sp], bb))
      continue;
    const int k0 = max(sp * (kCcSuper / kCcBlock), a0 / kCcBlock);
    const int k1 = min((sp + 1) * (kCcSuper / kCcBlock), (a_end + kCcBlock - 1) / kCcBlock);
    for (int k = k0; k < k1; ++k) {
      if ((uint64_t)(ablk + k) < (uint64_t)A.cc_nblk && boxes_disjoint(A.cc_blk[ablk + k], bb))
        continue;
      const int v0 = k * kCcBlock;
      __syncthreads();
      for (int t = lane; t <= kCcBlock; t += kWave) {
        const int idx = (v0 + t) % r.na;  // the block's vertices, cyclic
        const V3<Tc> x = F.load(X, r.oa + idx);
        lds[t] = Vtx<Tc>{x.x, x.y, x.z, (Tc)0};
      }
      __syncthreads();
      const int jlo = max(v0, lo_l), jhi = min(v0 + kCcBlock, hi_l);
      if (L.active && jlo < jhi)
        walk_tile<Tc, kCrossings, R>(lds, v0, jlo, jhi, jlo, wk, sg, acc);
    }
  }
}

// Per-lane state of the term form AT (the direct sum's, or the crossing count's).
template <typename Tc, int AT, int R>
struct LaneOf {
  using S = Segs<Tc, R>;
  using W = Walk<Tc, R>;
};
template <typename Tc, int R>
struct LaneOf<Tc, kCrossings, R> {
  using S = CcSegs<Tc, R>;
  using W = CcWalk<Tc, R>;
};

template <typename Tc, int R>
__device__ __forceinline__ void make_lane(const V3<Tc>* k, const Layout& L, const DsArgs&,
                                          Segs<Tc, R>& sg) {
  make_segs<Tc, R>(k, sg);
}

// Scale from the lane sums to the pair's value: 1 / (2 pi) for the direct
// sum's angles, 1/2 for crossing signs.
template <int AT>
__device__ __forceinline__ double value_scale() {
  return AT == kCrossings ? 0.5 : kInvTwoPi;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Wave sum of the lanes' partials.  `whole`: this item is the pair's only one,
// so its value is final and the pair is finalised at once (`fpre`: the pair's
// flags as the plan left them, loaded when the item started so that finishing
// does not wait on a load).  Otherwise the sum goes into the pair's fixed-point
// accumulator, and the pair is finalised after this kernel, from the big list.
template <int AT>
__device__ __forceinline__ void finish_item(double acc, int32_t p, int lane, const DsArgs& A,
                                            bool whole, uint32_t fpre) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane != 0) return;
  const double v = acc * value_scale<AT>();
  const bool ok = fabs(v) < 1.0e14;  // false for NaN / Inf / absurd magnitude
  if (whole)
    finalize_pair(A.out, p, v, fpre | (ok ? 0u : kFlagNonfinite));
  else if (ok)
    fixed_add(&A.acc[2 * (int64_t)p], v);
  else
    atomicOr(&A.out.flags[p], kFlagNonfinite);
}

// Every variant must fit in 256 registers per lane (two waves per SIMD); a
// test checks the compiled register counts.  No occupancy attribute is set:
// capping the compiler's register budget made it spread the transcendental
// instructions through the loop, which measured slower.
// PK: R small pairs whose loop B fits one wave's lanes share a wave (the
// throughput layout); without it every small pair gets a whole wave of its
// own, which shortens each lane's walk (the layout for calls with few pairs).
template <typename Tin, typename Tc, int AT, int R, bool PK = true>
__global__ __launch_bounds__(kWave) void ds_persistent(DsArgs A) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  Vtx<Tc>* lds = reinterpret_cast<Vtx<Tc>*>(lds_raw);
  const int lane = threadIdx.x;
  const Tin* X = static_cast<const Tin*>(A.xyz);
  const int64_t big_total = *A.s.big_total;
  const int64_t n_big = A.s.counts[1];
  const int64_t n_small = A.s.counts[0];
  const int64_t total = big_total + (n_small + A.batch - 1) / A.batch;

  // A wave's first work index is its workgroup index, so a launch with fewer
  // items than waves costs no atomic at all; later indices come from the
  // device counter, offset by the grid.  The next index is fetched one item
  // ahead so the atomic's latency overlaps the current item's arithmetic; a
  // fused check's stop flag is read with it (device-scope load, so another
  // wave's store is seen).
  unsigned long long wnext = blockIdx.x;
  int stopnext = 0;
  if (lane == 0 && A.out.stop)
    stopnext = __hip_atomic_load(A.out.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (;;) {
    const int64_t w = (int64_t)__shfl(wnext, 0);
    if (w >= total || __shfl(stopnext, 0)) break;
    if (lane == 0) {
      wnext = gridDim.x + atomicAdd(A.s.counter, 1ull);
      if (A.out.stop)
        stopnext = __hip_atomic_load(A.out.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }

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
      const uint32_t fpre = r.items == 1 ? A.out.flags[r.p] : 0u;
      const Layout L = layout<R>(r, w - A.s.big_prefix[lo], A.chunk, lane);
      Frame<Tin, Tc> F;
      F.set(X, r.ob + L.b0);
      V3<Tc> kv[R + 1];
      load_b<Tin, Tc, R>(X, r, L, F, kv);
      typename LaneOf<Tc, AT, R>::S sg;
      make_lane<Tc, R>(kv, L, A, sg);
      typename LaneOf<Tc, AT, R>::W wk;
      double acc = 0.0;
      bool culled = false;
      if constexpr (AT == kCrossings) {
        if (A.cc_blk) {
          cc_item_culled<Tin, Tc, R>(A, X, F, lds, r, L, lane, wk, sg, acc);
          culled = true;
        }
      }
      // Code placement of the big-item walk loop of the FP32 kernel that
      // big pairs run (R = 4, arctangent form 2): with these four no-ops its
      // first instruction sits 12 bytes past a 32-byte boundary of the
      // kernel, where it measured 570 ms per knit-workload call against
      // 598-645 ms at the other offsets (same instructions, a sweep of 0-16
      // no-ops).  The other walk loops come earlier in the code and do not
      // move; a CPU test checks the placements.
      if constexpr (PK && sizeof(Tin) == 4 && sizeof(Tc) == 4 && AT == 2 && R == 4)
        asm volatile(".rept 4\n s_nop 0\n.endr");
      if (!culled)
      for (int t0 = 0; t0 < L.nah; t0 += A.tile) {
        const int tl = (L.nah - t0) < A.tile ? (L.nah - t0) : A.tile;
        __syncthreads();
        for (int v = lane; v <= tl; v += kWave) {
          int64_t idx = L.a0 + t0 + v;
          if (idx >= r.na) idx -= r.na;  // closing vertex of the loop
          const V3<Tc> x = F.load(X, r.oa + idx);
          lds[v] = Vtx<Tc>{x.x, x.y, x.z, (Tc)0};
        }
        __syncthreads();
        const int jlo = L.js > t0 ? L.js : t0;
        const int jhi = L.je < t0 + tl ? L.je : t0 + tl;
        if (L.active && jlo < jhi) walk_tile<Tc, AT, R>(lds, t0, jlo, jhi, L.js, wk, sg, acc);
      }
      finish_item<AT>(acc, r.p, lane, A, r.items == 1, fpre);
    } else {
      // a batch of small pairs (one item each, loop A of at most kSmallA - 1
      // segments).  Pairs whose loop B has at most 64 segments run R at a
      // time when R > 1, 64 / R lanes each (each lane walks more of loop A,
      // and the per-pair setup, reduction and finalisation are shared); the
      // others run one at a time on the whole wave.  Which way a pair runs
      // depends only on the pair, so results are reproducible.  Records are
      // re-read from the list where needed rather than held in registers
      // across the walks.
      const int64_t m0 = (w - big_total) * (int64_t)A.batch;
      const int cnt = (int)((n_small - m0) < A.batch ? (n_small - m0) : A.batch);
      const WorkRec* recs = A.s.small + m0;
      const int32_t nb_l = lane < cnt ? recs[lane].nb : 0;
      const unsigned long long pmask = __ballot(PK && R > 1 && lane < cnt && nb_l <= kWave);
      unsigned long long smask = __ballot(lane < cnt) & ~pmask;
      const int npk = __popcll(pmask);
      if (npk > 0) {
        constexpr int K = R, S = kWave / R;
        const int seg = lane / S, sl = lane - seg * S;
        Vtx<Tc>* myl = lds + seg * kSmallA;
        for (int r0 = 0; r0 < npk; r0 += K) {
          const bool has = r0 + seg < npk;
          // batch position of the (r0 + seg)-th packed pair
          unsigned long long mm = pmask;
          for (int t = has ? r0 + seg : r0; t > 0; --t) mm &= mm - 1ull;
          const WorkRec cur = recs[__ffsll((long long)mm) - 1];
          const uint32_t fm = A.out.flags[cur.p];
          Frame<Tin, Tc> F;
          F.set(X, cur.ob);
          __syncthreads();
          if (has)
            for (int v = sl; v <= cur.na; v += S) {
              const V3<Tc> x = F.load(X, cur.oa + (v < cur.na ? v : 0));
              myl[v] = Vtx<Tc>{x.x, x.y, x.z, (Tc)0};
            }
          const Layout L = layout<R>(cur, 0, A.chunk, sl, S);
          V3<Tc> kv[R + 1];
          load_b<Tin, Tc, R>(X, cur, L, F, kv);
          typename LaneOf<Tc, AT, R>::S sg;
          make_lane<Tc, R>(kv, L, A, sg);
          __syncthreads();
          typename LaneOf<Tc, AT, R>::W wk;
          double acc = 0.0;
          if (has && L.active && L.js < L.je) walk_tile<Tc, AT, R>(myl, 0, L.js, L.je, L.js, wk, sg, acc);
#pragma unroll
          for (int o = S / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
          if (has && sl == 0) {
            const double v = acc * value_scale<AT>();
            finalize_pair(A.out, cur.p, v, fm | (fabs(v) < 1.0e14 ? 0u : kFlagNonfinite));
          }
        }
      }
      while (smask) {
        const int m = __ffsll((long long)smask) - 1;
        smask &= smask - 1ull;
        const WorkRec cur = recs[m];
        const uint32_t fm = A.out.flags[cur.p];
        const Layout L = layout<R>(cur, 0, A.chunk, lane);
        Frame<Tin, Tc> F;
        F.set(X, cur.ob);
        V3<Tc> kv[R + 1];
        load_b<Tin, Tc, R>(X, cur, L, F, kv);
        const V3<Tc> a_lo = F.load(X, cur.oa + (lane < cur.na ? lane : 0));
        const V3<Tc> a_hi = F.load(X, cur.oa + (lane + kWave < cur.na ? lane + kWave : 0));
        __syncthreads();
        if (lane <= cur.na) lds[lane] = Vtx<Tc>{a_lo.x, a_lo.y, a_lo.z, (Tc)0};
        if (lane + kWave <= cur.na) lds[lane + kWave] = Vtx<Tc>{a_hi.x, a_hi.y, a_hi.z, (Tc)0};
        typename LaneOf<Tc, AT, R>::S sg;
        make_lane<Tc, R>(kv, L, A, sg);
        __syncthreads();
        typename LaneOf<Tc, AT, R>::W wk;
        double acc = 0.0;
        if (L.active && L.js < L.je) walk_tile<Tc, AT, R>(lds, 0, L.js, L.je, L.js, wk, sg, acc);
        finish_item<AT>(acc, cur.p, lane, A, true, fm);
      }
    }
  }
}

// Leaf pairs of the Barnes-Hut traversal (Alg. 6, both nodes leaves): Eq. 4
// over their kBhLeaf x kBhLeaf segment pairs with the walk above.  Like the
// packed small pairs of the direct sum, a wave takes four leaf pairs at a
// time, 16 lanes each: a lane holds 4 consecutive segments of the B leaf, the
// A leaf's vertices are in LDS (FP32 terms, FP64 sums).  A wave works through
// 32 consecutive entries of the list and adds one sum per run of entries of
// the same pair into its fixed-point accumulator.
template <typename Tin>
__global__ __launch_bounds__(kWave) void bh_near_k(BhArgs A) {
  constexpr int K = 4, S = kWave / K, R = 4;  // S * R == kBhLeaf
  static_assert(S * R == kBhLeaf, "a segment of S lanes covers one leaf");
  __shared__ Vtx<float> lds[K][kBhLeaf + 1];
  const int lane = threadIdx.x, seg = lane / S, sl = lane - seg * S;
  const Tin* X = static_cast<const Tin*>(A.xyz);
  const int64_t cnt = A.counts[kBhMaxIters + 1];
  const int64_t n = cnt < A.near_cap ? cnt : A.near_cap;
  constexpr int kChunk = 32;
  for (int64_t c0 = (int64_t)blockIdx.x * kChunk; c0 < n; c0 += (int64_t)gridDim.x * kChunk) {
    const int64_t c1 = (c0 + kChunk) < n ? c0 + kChunk : n;
    double run = 0.0;  // uniform over the wave
    int32_t pr = -1;
    for (int64_t e0 = c0; e0 < c1; e0 += K) {
      const int64_t e = e0 + seg;
      const bool has = e < c1;
      const BhPair w = A.near[has ? e : e0];
      const int32_t i = A.pairs[2 * (int64_t)w.p], j = A.pairs[2 * (int64_t)w.p + 1];
      const int64_t oa = A.off[i], na = A.off[i + 1] - oa;
      const int64_t ob = A.off[j], nb = A.off[j + 1] - ob;
      const int64_t a0 = (int64_t)w.ka * kBhLeaf, b0 = (int64_t)w.kb * kBhLeaf;
      const int ma = (int)((na - a0) < kBhLeaf ? (na - a0) : kBhLeaf);
      const int mb = (int)((nb - b0) < kBhLeaf ? (nb - b0) : kBhLeaf);
      Frame<Tin, float> F;
      F.set(X, ob + b0);
      __syncthreads();
      for (int t = sl; t <= ma; t += S) {
        int64_t idx = a0 + t;
        if (idx >= na) idx -= na;  // closing vertex of the loop
        const V3<float> x = F.load(X, oa + idx);
        lds[seg][t] = Vtx<float>{x.x, x.y, x.z, 0.0f};
      }
      Segs<float, R> sg;
      {
        const int first = sl * R;
        V3<float> kv[R + 1];
#pragma unroll
        for (int r = 0; r <= R; ++r) {
          int64_t ib = b0 + (first + r < mb ? first + r : mb);  // vertex b0 + mb closes the leaf
          if (ib >= nb) ib -= nb;
          kv[r] = F.load(X, ob + ib);
        }
#pragma unroll
        for (int r = 0; r <= R; ++r) sg.k[r] = kv[r];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          sg.s[r] = sg.k[r + 1] - sg.k[r];
          sg.m[r] = cross(sg.s[r], sg.k[r] - sg.k[0]);
        }
      }
      __syncthreads();
      double acc = 0.0;
      if (has) {
        Walk<float, R> wk;
        walk_init(wk, V3<float>{lds[seg][0].x, lds[seg][0].y, lds[seg][0].z}, sg);
        for (int jj = 0; jj < ma; ++jj) {
          const Vtx<float> v1 = lds[seg][jj + 1];
          acc += (double)walk_step<float, 2, R>(wk, V3<float>{v1.x, v1.y, v1.z}, sg);
        }
      }
#pragma unroll
      for (int o = S / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      // the K entries in order: extend the run or flush it (uniform logic)
#pragma unroll
      for (int q = 0; q < K; ++q) {
        if (e0 + q >= c1) break;
        const int32_t pq = __shfl(w.p, q * S);
        const double vq = __shfl(acc, q * S);
        if (pq != pr) {
          if (pr >= 0 && lane == 0) {
            const double v = run * kInvTwoPi;
            if (fabs(v) < 1.0e14)
              fixed_add(&A.acc[2 * (int64_t)pr], v);
            else
              atomicOr(&A.out.flags[pr], kFlagNonfinite);
          }
          pr = pq;
          run = 0.0;
        }
        run += vq;
      }
    }
    if (pr >= 0 && lane == 0) {
      const double v = run * kInvTwoPi;
      if (fabs(v) < 1.0e14)
        fixed_add(&A.acc[2 * (int64_t)pr], v);
      else
        atomicOr(&A.out.flags[pr], kFlagNonfinite);
    }
  }
}

// A tile plus its closing vertex, or R small pairs' loops A side by side.
template <typename Tc, int R>
size_t lds_bytes(int tile) {
  const int n = tile + 1 > R * kSmallA ? tile + 1 : R * kSmallA;
  return (size_t)n * sizeof(Vtx<Tc>);
}

template <typename Tin, typename Tc, int AT, int R, bool PK>
hipError_t launch_t(const DsArgs& a, int grid, hipStream_t s) {
  const size_t shm = lds_bytes<Tc, R>(a.tile);
  if constexpr (PK)
    ds_persistent<Tin, Tc, AT, R><<<dim3(grid), dim3(kWave), shm, s>>>(a);
  else
    ds_persistent<Tin, Tc, AT, R, false><<<dim3(grid), dim3(kWave), shm, s>>>(a);
  return hipGetLastError();
}

template <typename Tin, typename Tc, int AT, int R, bool PK>
int grid_t(int tile, int n_cu, int waves_per_cu) {
  int per_cu = 0;
  hipError_t e;
  if constexpr (PK)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ds_persistent<Tin, Tc, AT, R>, kWave,
                                                     lds_bytes<Tc, R>(tile));
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, ds_persistent<Tin, Tc, AT, R, false>,
                                                     kWave, lds_bytes<Tc, R>(tile));
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  if (waves_per_cu > 0 && waves_per_cu < per_cu) per_cu = waves_per_cu;
  return per_cu * n_cu;
}

// Kernel variants: input type x arithmetic x arctangent form x segments per lane.
struct Variant {
  hipError_t (*launch)(const DsArgs&, int, hipStream_t);
  int (*grid)(int, int, int);
};

template <typename Tin, typename Tc, int AT, int R, bool PK = true>
constexpr Variant variant() {
  return Variant{launch_t<Tin, Tc, AT, R, PK>, grid_t<Tin, Tc, AT, R, PK>};
}

// Unpacked layout for calls with few pairs: the direct-sum forms only (the
// FP32 arctangent forms 0 and 2 give the same values, so both map to 2;
// with R = 1 nothing is packed anyway).
bool pick_unpacked(bool in_f64, bool compute_f64, int atan_form, int segs, Variant* v) {
  if (atan_form == kCrossings || segs < 2) return false;
  if (compute_f64) {
    *v = in_f64 ? variant<double, double, 0, 2, false>() : variant<float, double, 0, 2, false>();
    return true;
  }
  if (atan_form == 1) return false;
  if (segs >= 4)
    *v = in_f64 ? variant<double, float, 2, 4, false>() : variant<float, float, 2, 4, false>();
  else
    *v = in_f64 ? variant<double, float, 2, 2, false>() : variant<float, float, 2, 2, false>();
  return true;
}

Variant pick(bool in_f64, bool compute_f64, int atan_form, int segs, bool unpacked = false) {
  Variant u;
  if (unpacked && pick_unpacked(in_f64, compute_f64, atan_form, segs, &u)) return u;
  if (compute_f64 && atan_form == kCrossings) {
    constexpr int C = kCrossings;
    if (segs >= 2) return in_f64 ? variant<double, double, C, 2>() : variant<float, double, C, 2>();
    return in_f64 ? variant<double, double, C, 1>() : variant<float, double, C, 1>();
  }
  if (compute_f64) {
    if (segs >= 2) return in_f64 ? variant<double, double, 0, 2>() : variant<float, double, 0, 2>();
    return in_f64 ? variant<double, double, 0, 1>() : variant<float, double, 0, 1>();
  }
  if (atan_form == 1) {
    if (segs >= 4) return in_f64 ? variant<double, float, 1, 4>() : variant<float, float, 1, 4>();
    if (segs >= 2) return in_f64 ? variant<double, float, 1, 2>() : variant<float, float, 1, 2>();
    return in_f64 ? variant<double, float, 1, 1>() : variant<float, float, 1, 1>();
  }
  if (atan_form == 2) {
    if (segs >= 4) return in_f64 ? variant<double, float, 2, 4>() : variant<float, float, 2, 4>();
    if (segs >= 2) return in_f64 ? variant<double, float, 2, 2>() : variant<float, float, 2, 2>();
    return in_f64 ? variant<double, float, 2, 1>() : variant<float, float, 2, 1>();
  }
  if (atan_form == kCrossings) {
    constexpr int C = kCrossings;
    if (segs >= 8) return in_f64 ? variant<double, float, C, 8>() : variant<float, float, C, 8>();
    if (segs >= 4) return in_f64 ? variant<double, float, C, 4>() : variant<float, float, C, 4>();
    if (segs >= 2) return in_f64 ? variant<double, float, C, 2>() : variant<float, float, C, 2>();
    return in_f64 ? variant<double, float, C, 1>() : variant<float, float, C, 1>();
  }
  if (segs >= 4) return in_f64 ? variant<double, float, 0, 4>() : variant<float, float, 0, 4>();
  if (segs >= 2) return in_f64 ? variant<double, float, 0, 2>() : variant<float, float, 0, 2>();
  return in_f64 ? variant<double, float, 0, 1>() : variant<float, float, 0, 1>();
}

}  // namespace

int segs_supported(bool compute_f64, int segs, bool crossings) {
  if (compute_f64) return segs >= 2 ? 2 : 1;
  if (crossings && segs >= 8) return 8;
  return segs >= 4 ? 4 : (segs >= 2 ? 2 : 1);
}

hipError_t launch_bh_near(const BhArgs& a, bool in_f64, hipStream_t s) {
  if (in_f64)
    bh_near_k<double><<<4096, kWave, 0, s>>>(a);
  else
    bh_near_k<float><<<4096, kWave, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_direct_sum(const DsArgs& a, bool in_f64, bool compute_f64, int atan_form,
                             int segs, int grid, hipStream_t s, bool unpacked) {
  return pick(in_f64, compute_f64, atan_form, segs, unpacked).launch(a, grid, s);
}

int direct_sum_grid(bool in_f64, bool compute_f64, int atan_form, int segs, int tile, int n_cu,
                    int waves_per_cu, bool unpacked) {
  return pick(in_f64, compute_f64, atan_form, segs, unpacked).grid(tile, n_cu, waves_per_cu);
}

}  // namespace lk
