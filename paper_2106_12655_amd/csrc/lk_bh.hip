// lk_bh.hip -- Barnes-Hut linking numbers (Sec. 3.4.4, Alg. 6) on the GPU.
//
// Trees over consecutive segments (a polyline is already spatially coherent,
// so no sort): leaves of kBhLeaf segments, kBhArity children per node.  The
// leaves are boxed and their moments summed by one wavefront each; each level
// above is one launch, a thread per node, shifting the children's moments to
// the node's centre with the appendix's rules.  The two-tree traversal of
// Alg. 6 runs breadth first: every launch takes the node pairs of one step,
// evaluates the far-field expansion (FP64, monopole + dipole + quadrupole) for
// pairs farther apart than beta (R_A + R_B), hands pairs of two leaves to the
// direct sum (lk_ds.hip) and splits the others into child pairs for the next
// step.  All counts live on the device and every launch has a host-known
// shape, so the sequence can be captured in a HIP graph.  Sums go into the
// pair's 128-bit fixed-point accumulator, so they do not depend on order.
#include "lk_internal.h"

namespace lk {
namespace {

// Largest loop i with (off[i] - off[0]) / span + i <= slot.
__device__ __forceinline__ int32_t find_loop(const int64_t* off, int32_t L, int64_t slot,
                                             int64_t span) {
  const int64_t o0 = off[0];
  int32_t lo = 0, hi = L;
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if ((off[mid] - o0) / span + mid <= slot)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

__device__ __forceinline__ int64_t node_slot(const BhArgs& A, int32_t loop, int h, int64_t k) {
  return A.level_base[h] + (A.off[loop] - A.off[0]) / bh_span(h) + loop + k;
}

// Slots of level h that the device offsets need.
__device__ __forceinline__ int64_t level_slots(const BhArgs& A, int h) {
  return (A.off[A.n_loops] - A.off[0]) / bh_span(h) + A.n_loops + 1;
}

// Lowest level with a single node for a loop of n segments.
__device__ __forceinline__ int root_level(int64_t n) {
  int h = 0;
  while (bh_count(n, h) > 1) ++h;
  return h;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// --------------------------------------------------------------- leaves
// One wavefront (one workgroup) per leaf slot: lane t holds segment t of the
// leaf.  The box covers the leaf's vertices (with the one closing its last
// segment); a segment with vector s and midpoint offset d from the centre
// adds s, s d^T and s (x) d (x) d + s (x) s (x) s / 12 (its exact moments).
// The lanes stage s and d in LDS, and lane j < 39 then sums moment j over
// the segments in order, so the 45 values of the node are written by 45
// lanes at once.  The same pass validates the loops in parallel over their
// leaves (non-finite coordinates, shortest squared segment), folding into the
// per-loop entries with atomics (a minimum of non-negative doubles is a
// minimum of their bit patterns).
static_assert(sizeof(BhNode) == 45 * sizeof(double), "BhNode is c, e, M, D, Q back to back");

template <typename Tin>
__global__ __launch_bounds__(64) void bh_leaves_k(BhArgs A) {
  __shared__ double sd[kBhLeaf][8];  // per segment: s[3], d[3]
  if (blockIdx.x == 0 && threadIdx.x < kBhMaxIters + 3) A.counts[threadIdx.x] = 0;
  const Tin* X = static_cast<const Tin*>(A.xyz);
  const int lane = threadIdx.x;
  const int64_t n_slots = level_slots(A, 0);
  // moment j of this lane: c_M[p] (j < 3), C_D[p][b] (j < 12), C_Q[p][b][c]
  const int j = lane - 6;
  const int jq = j - 12, jd = j - 3;
  const int mp = j < 3 ? j : (j < 12 ? jd / 3 : jq / 9);
  const int mb = j < 12 ? jd % 3 : (jq / 3) % 3;
  const int mc = jq % 3;
  for (int64_t slot = blockIdx.x; slot < n_slots; slot += gridDim.x) {
    const int32_t i = find_loop(A.off, A.n_loops, slot, kBhLeaf);
    const int64_t oi = A.off[i], n = A.off[i + 1] - oi;
    const int64_t k = slot - ((oi - A.off[0]) / kBhLeaf + i);
    // (offsets that decrease make no node: every read stays in the loop)
    if (n <= 0 || k < 0 || k >= bh_count(n, 0)) continue;  // uniform over the workgroup
    const int64_t a = k * kBhLeaf;
    const int m = (int)((n - a) < kBhLeaf ? (n - a) : kBhLeaf);
    double x0[3] = {0, 0, 0}, x1[3] = {0, 0, 0};
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (lane < m) {
      int64_t v1 = a + lane + 1;
      if (v1 >= n) v1 -= n;
      for (int q = 0; q < 3; ++q) {
        x0[q] = (double)X[3 * (oi + a + lane) + q];
        x1[q] = (double)X[3 * (oi + v1) + q];
        lo[q] = fmin(x0[q], x1[q]);
        hi[q] = fmax(x0[q], x1[q]);
      }
    }
    {
      uint32_t f = 0u;
      double mn = INFINITY;
      if (lane < m) {
        if (!isfinite(x0[0]) || !isfinite(x0[1]) || !isfinite(x0[2])) f = kFlagNonfinite | kFlagBadloop;
        const double dx = x1[0] - x0[0], dy = x1[1] - x0[1], dz = x1[2] - x0[2];
        mn = dx * dx + dy * dy + dz * dz;
      }
      for (int o = 32; o > 0; o >>= 1) {
        f |= (uint32_t)__shfl_xor((int)f, o);
        mn = fmin(mn, __shfl_xor(mn, o));
      }
      if (lane == 0) {
        if (f) atomicOr(&A.lf[i], f);
        // the entry only decreases, so a plain read that is not above mn
        // makes the atomic unnecessary (thousands of leaves share one loop)
        if (mn < INFINITY && mn < A.minseg2[i])
          atomicMin(reinterpret_cast<unsigned long long*>(&A.minseg2[i]),
                    (unsigned long long)__double_as_longlong(mn));
      }
    }
    for (int q = 0; q < 3; ++q)
      for (int o = 32; o > 0; o >>= 1) {
        lo[q] = fmin(lo[q], __shfl_xor(lo[q], o));
        hi[q] = fmax(hi[q], __shfl_xor(hi[q], o));
      }
    double c[3], e[3];
    for (int q = 0; q < 3; ++q) {
      c[q] = 0.5 * (lo[q] + hi[q]);
      e[q] = 0.5 * (hi[q] - lo[q]);
    }
    __syncthreads();  // the previous slot's reads of sd are done
    if (lane < m)
      for (int q = 0; q < 3; ++q) {
        sd[lane][q] = x1[q] - x0[q];
        sd[lane][3 + q] = 0.5 * (x0[q] + x1[q]) - c[q];
      }
    __syncthreads();
    double v = 0.0;
    if (j >= 0 && j < 39)
      for (int r = 0; r < m; ++r) {
        const double s0 = sd[r][0], s1 = sd[r][1], s2 = sd[r][2];
        const double d0 = sd[r][3], d1 = sd[r][4], d2 = sd[r][5];
        const double sp = mp == 0 ? s0 : (mp == 1 ? s1 : s2);
        if (j < 3) {
          v += sp;
        } else {
          const double db = mb == 0 ? d0 : (mb == 1 ? d1 : d2);
          if (j < 12) {
            v += sp * db;
          } else {
            const double dc = mc == 0 ? d0 : (mc == 1 ? d1 : d2);
            const double sb = mb == 0 ? s0 : (mb == 1 ? s1 : s2);
            const double sc = mc == 0 ? s0 : (mc == 1 ? s1 : s2);
            v += sp * db * dc + sp * sb * sc * (1.0 / 12.0);
          }
        }
      }
    // node layout: c[3], e[3], M[3], D[9], Q[27] -- 45 doubles, one per lane
    const int64_t dst = A.level_base[0] + slot;
    if (lane < 45 && slot < A.level_cap[0]) {
      const int q = lane % 3;
      const double cq = q == 0 ? c[0] : (q == 1 ? c[1] : c[2]);
      const double eq = q == 0 ? e[0] : (q == 1 ? e[1] : e[2]);
      reinterpret_cast<double*>(&A.nodes[dst])[lane] = lane < 3 ? cq : (lane < 6 ? eq : v);
    }
  }
}

// ---------------------------------------------------------------- levels
// One thread per node of level h (>= 1): the box of its children's boxes,
// and their moments moved to its centre (r = child centre - node centre):
//   c_M += c_Mc;  C_D += C_Dc + c_Mc r^T;
//   C_Q[p][b][c] += C_Qc[p][b][c] + C_Dc[p][b] r_c + C_Dc[p][c] r_b + c_Mc[p] r_b r_c.
__global__ __launch_bounds__(256) void bh_level_k(BhArgs A, int h) {
  const int64_t n_slots = level_slots(A, h);
  const int64_t span = bh_span(h);
  for (int64_t slot = (int64_t)blockIdx.x * 256 + threadIdx.x; slot < n_slots;
       slot += (int64_t)gridDim.x * 256) {
    const int32_t i = find_loop(A.off, A.n_loops, slot, span);
    const int64_t n = A.off[i + 1] - A.off[i];
    const int64_t k = slot - ((A.off[i] - A.off[0]) / span + i);
    const int64_t nch = bh_count(n, h - 1);
    if (n <= 0 || k < 0 || k >= bh_count(n, h) || nch <= 1) continue;  // no such node, or above the root
    if (slot >= A.level_cap[h]) continue;
    const int64_t c0 = k * kBhArity, c1 = (c0 + kBhArity) < nch ? c0 + kBhArity : nch;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    bool ok = true;
    for (int64_t c = c0; c < c1; ++c) {
      const int64_t cs = node_slot(A, i, h - 1, c);
      if ((uint64_t)(cs - A.level_base[h - 1]) >= (uint64_t)A.level_cap[h - 1]) {
        ok = false;
        break;
      }
      const BhNode& ch = A.nodes[cs];
      for (int q = 0; q < 3; ++q) {
        lo[q] = fmin(lo[q], ch.c[q] - ch.e[q]);
        hi[q] = fmax(hi[q], ch.c[q] + ch.e[q]);
      }
    }
    BhNode nd;
    for (int q = 0; q < 3; ++q) {
      nd.c[q] = ok ? 0.5 * (lo[q] + hi[q]) : __builtin_nan("");
      nd.e[q] = ok ? 0.5 * (hi[q] - lo[q]) : __builtin_nan("");
    }
    for (int q = 0; q < 3; ++q) nd.M[q] = 0.0;
    for (int q = 0; q < 9; ++q) nd.D[q] = 0.0;
    for (int q = 0; q < 27; ++q) nd.Q[q] = 0.0;
    if (ok)
      for (int64_t c = c0; c < c1; ++c) {
        const BhNode& ch = A.nodes[node_slot(A, i, h - 1, c)];
        double r[3];
        for (int q = 0; q < 3; ++q) r[q] = ch.c[q] - nd.c[q];
        for (int p = 0; p < 3; ++p) {
          nd.M[p] += ch.M[p];
          for (int b = 0; b < 3; ++b) {
            nd.D[3 * p + b] += ch.D[3 * p + b] + ch.M[p] * r[b];
            for (int cc = 0; cc < 3; ++cc)
              nd.Q[9 * p + 3 * b + cc] += ch.Q[9 * p + 3 * b + cc] + ch.D[3 * p + b] * r[cc] +
                                          ch.D[3 * p + cc] * r[b] + ch.M[p] * r[b] * r[cc];
          }
        }
      }
    A.nodes[A.level_base[h] + slot] = nd;
  }
}

// ------------------------------------------------------------------ roots
__global__ __launch_bounds__(256) void bh_roots_k(BhArgs A, int64_t n_pairs) {
  const int lane = threadIdx.x & 63;
  // the same trip count in every lane (the append is wavefront-collective)
  for (int64_t base = (int64_t)blockIdx.x * 256; base < n_pairs; base += (int64_t)gridDim.x * 256) {
    const int64_t p = base + threadIdx.x;
    bool push = false;
    BhPair root{0, 0, 0, 0};
    if (p < n_pairs) {
      if (A.est) {
        A.est[2 * p] = 0ull;
        A.est[2 * p + 1] = 0ull;
      }
      const int32_t i = A.pairs[2 * p], j = A.pairs[2 * p + 1];
      const bool valid = i >= 0 && j >= 0 && i < A.n_loops && j < A.n_loops && i != j &&
                         (!A.beta_p || A.beta_p[p] > 0.0);
      const int64_t na = valid ? A.off[i + 1] - A.off[i] : 0, nb = valid ? A.off[j + 1] - A.off[j] : 0;
      // pairs without work were finalised by the plan
      if (valid && na >= 1 && nb >= 1 && na <= 0x7fffffffLL && nb <= 0x7fffffffLL) {
        push = true;
        root = BhPair{(int32_t)p, 0, 0, root_level(na) | (root_level(nb) << 8)};
      }
    }
    const unsigned long long m = __ballot(push);
    const int leader = m ? __ffsll((long long)m) - 1 : 0;
    int32_t b0 = 0;
    if (m && lane == leader) b0 = atomicAdd(&A.counts[0], (int32_t)__popcll(m));
    b0 = __shfl(b0, leader);
    if (push) {
      const unsigned long long below = lane ? (~0ull >> (64 - lane)) : 0ull;
      const int64_t at = (int64_t)b0 + __popcll(m & below);
      if (at < A.list_cap)
        A.list[0][at] = root;
      else
        atomicOr(&A.out.flags[root.p], kFlagNonfinite);  // list full: the pair is refitted
    }
  }
}

// ------------------------------------------------------------- far field
// The expansion of the Gauss integral about the two node centres, with the
// derivatives of G = -1/(4 pi |r1 - r2|) at r = c_B - c_A:
//   g = r / (4 pi |r|^3),  H = (I |r|^2 - 3 r r^T) / (4 pi |r|^5),
//   K_abc = -3 (r_a d_bc + r_b d_ac + r_c d_ab) / (4 pi |r|^5) + 15 r_a r_b r_c / (4 pi |r|^7);
//   lambda ~ -[ (M_A x M_B) . g
//             + sum_ab H_ab eps_apq (-D_A[p][b] M_B[q] + M_A[p] D_B[q][b])
//             + 1/2 sum_abc K_abc eps_apq (Q_A[p][b][c] M_B[q] - D_A[p][b] D_B[q][c]
//                                         - D_A[p][c] D_B[q][b] + M_A[p] Q_B[q][b][c]) ].
// eps_apq is non-zero for the six cyclic and anti-cyclic index triples only.
__device__ double far_field(const BhNode& u, const BhNode& v, int order) {
  double r[3];
  for (int q = 0; q < 3; ++q) r[q] = v.c[q] - u.c[q];
  const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double id = 1.0 / sqrt(d2);
  const double f = 0.07957747154594766788;  // 1 / (4 pi)
  const double i3 = f * id * id * id, i5 = i3 * id * id, i7 = i5 * id * id;
  // cross-type contractions: X_a = eps_apq x_p y_q for the index triples
  constexpr int P[3] = {1, 2, 0}, Qx[3] = {2, 0, 1};  // (a, p, q) cyclic: +1, (a, q, p): -1
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int p = P[a], q = Qx[a];
    // eps_apq = +1, eps_aqp = -1
    t1 += (u.M[p] * v.M[q] - u.M[q] * v.M[p]) * r[a] * i3;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double Hab = ((a == b) ? d2 : 0.0) * i5 - 3.0 * r[a] * r[b] * i5;
      const double m = (-u.D[3 * p + b] * v.M[q] + u.M[p] * v.D[3 * q + b]) -
                       (-u.D[3 * q + b] * v.M[p] + u.M[q] * v.D[3 * p + b]);
      t2 += Hab * m;
      if (order >= 2) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double sym = r[a] * (b == c) + r[b] * (a == c) + r[c] * (a == b);
          const double Kabc = -3.0 * sym * i5 + 15.0 * r[a] * r[b] * r[c] * i7;
          const double mp = u.Q[9 * p + 3 * b + c] * v.M[q] - u.D[3 * p + b] * v.D[3 * q + c] -
                            u.D[3 * p + c] * v.D[3 * q + b] + u.M[p] * v.Q[9 * q + 3 * b + c];
          const double mq = u.Q[9 * q + 3 * b + c] * v.M[p] - u.D[3 * q + b] * v.D[3 * p + c] -
                            u.D[3 * q + c] * v.D[3 * p + b] + u.M[q] * v.Q[9 * p + 3 * b + c];
          t3 += 0.5 * Kabc * (mp - mq);
        }
      }
    }
  }
  return -(t1 + t2 + t3);
}

__device__ __forceinline__ double node_radius(const BhNode& n) {
  return sqrt(n.e[0] * n.e[0] + n.e[1] * n.e[1] + n.e[2] * n.e[2]);
}

__device__ __forceinline__ double frob(const double* x, int n) {
  double s = 0.0;
  for (int q = 0; q < n; ++q) s += x[q] * x[q];
  return sqrt(s);
}

// The next-order error estimate of one far node pair (Sec. 3.4.4, with the
// constant k = 1/(4 pi)):
//   |r|^-5 (R_A |c_M,B| ||C_Q,A|| + R_B |c_M,A| ||C_Q,B||
//           + 3 (||C_D,A|| ||C_Q,B|| + ||C_Q,A|| ||C_D,B||)),
// norms Euclidean / Frobenius, R the half box diagonals.
__device__ double far_estimate(const BhNode& u, const BhNode& v) {
  double r[3];
  for (int q = 0; q < 3; ++q) r[q] = v.c[q] - u.c[q];
  const double d2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  const double d = sqrt(d2), d5 = d2 * d * d2;
  const double f = 0.07957747154594766788;  // 1 / (4 pi)
  const double nM1 = frob(u.M, 3), nM2 = frob(v.M, 3);
  const double nD1 = frob(u.D, 9), nD2 = frob(v.D, 9), nQ1 = frob(u.Q, 27), nQ2 = frob(v.Q, 27);
  return f / d5 *
         (node_radius(u) * nM2 * nQ1 + node_radius(v) * nM1 * nQ2 + 3.0 * (nD1 * nQ2 + nQ1 * nD2));
}

// ------------------------------------------------------------ traversal
// Wave-collective append of `n` entries per lane to a list: returns the
// lane's first position (one atomic per wave).
__device__ __forceinline__ int64_t wave_reserve(int32_t* count, int n) {
  const int lane = threadIdx.x & 63;
  int32_t x = n;  // inclusive scan
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  const int32_t total = __shfl(x, 63);
  int32_t b0 = 0;
  if (total > 0 && lane == 0) b0 = atomicAdd(count, total);
  b0 = __shfl(b0, 0);
  return (int64_t)b0 + x - n;
}

// Node (level h, index k) of loop `loop`: its slot, or -1 beyond the buffer.
__device__ __forceinline__ int64_t checked_slot(const BhArgs& A, int32_t loop, int h, int64_t k) {
  const int64_t s = node_slot(A, loop, h, k);
  // unsigned: a slot below the level (offsets that decrease) is refused too
  return (uint64_t)(s - A.level_base[h]) < (uint64_t)A.level_cap[h] ? s : -1;
}

__device__ __forceinline__ bool is_far(double beta, const BhNode& u, const BhNode& v) {
  double d2 = 0.0;
  for (int q = 0; q < 3; ++q) {
    const double dq = v.c[q] - u.c[q];
    d2 += dq * dq;
  }
  return sqrt(d2) > beta * (node_radius(u) + node_radius(v));
}

// One breadth-first step over the node pairs of iteration `it`.  A pair that
// is far is evaluated, a pair of two leaves goes to the leaf list, any other
// is split (the node with children and the larger radius); its child pairs
// are classified at once, so the next step's list holds only pairs that must
// be split again.
__global__ __launch_bounds__(256) void bh_expand_k(BhArgs A, int it) {
  const int lane = threadIdx.x & 63;
  const BhPair* in = A.list[it & 1];
  BhPair* out = A.list[(it + 1) & 1];
  int32_t* n_out = &A.counts[it + 1];
  int32_t* n_near = &A.counts[kBhMaxIters + 1];
  const int64_t n_in = A.counts[it] < A.list_cap ? A.counts[it] : A.list_cap;
  const int64_t stride = (int64_t)gridDim.x * 256;
  // the same trip count in every lane (the appends are wavefront-collective)
  for (int64_t base = (int64_t)blockIdx.x * 256; base < n_in; base += stride) {
    const int64_t e = base + threadIdx.x;
    const bool has = e < n_in;
    const BhPair w = has ? in[e] : BhPair{-1, 0, 0, 0};
    double val = 0.0, err = 0.0;
    bool fail = false;
    const double beta = has && A.beta_p ? A.beta_p[w.p] : A.beta;
    // classification of the pair itself (roots arrive unclassified), then of
    // its children: bit c of near_m / next_m marks child c for that list
    int self = 0;  // 0 none, 1 near, 2 split
    unsigned near_m = 0u, next_m = 0u;
    int split_a = 0, hc = 0;
    int64_t cbase = 0;
    if (has) {
      const int ha = w.lev & 255, hb = w.lev >> 8;
      const int32_t i = A.pairs[2 * (int64_t)w.p], j = A.pairs[2 * (int64_t)w.p + 1];
      const int64_t sa = checked_slot(A, i, ha, w.ka), sb = checked_slot(A, j, hb, w.kb);
      if (sa < 0 || sb < 0) {
        fail = true;
      } else {
        const BhNode& u = A.nodes[sa];
        const BhNode& v = A.nodes[sb];
        if (is_far(beta, u, v)) {
          val = far_field(u, v, A.order);
          if (A.est) err = far_estimate(u, v);
        } else if (ha == 0 && hb == 0) {
          self = 1;
        } else {
          self = 2;
          split_a = ha > 0 && (hb == 0 || node_radius(u) > node_radius(v));
          const int32_t loop = split_a ? i : j;
          const int64_t n = A.off[loop + 1] - A.off[loop];
          hc = (split_a ? ha : hb) - 1;
          const int64_t cnt = bh_count(n, hc);
          cbase = (int64_t)(split_a ? w.ka : w.kb) * kBhArity;
          const int64_t c1 = (cbase + kBhArity) < cnt ? cbase + kBhArity : cnt;
          for (int c = 0; c < (int)(c1 - cbase); ++c) {
            const int64_t sc = checked_slot(A, loop, hc, cbase + c);
            if (sc < 0) {
              fail = true;
              break;
            }
            const BhNode& ch = A.nodes[sc];
            const bool far = split_a ? is_far(beta, ch, v) : is_far(beta, u, ch);
            if (far) {
              val += split_a ? far_field(ch, v, A.order) : far_field(u, ch, A.order);
              if (A.est) err += split_a ? far_estimate(ch, v) : far_estimate(u, ch);
            } else if (hc == 0 && (split_a ? hb : ha) == 0) {
              near_m |= 1u << c;
            } else {
              next_m |= 1u << c;
            }
          }
        }
      }
    }
    if (fail) atomicOr(&A.out.flags[w.p], kFlagNonfinite);  // refitted
    // far-field values (and estimates): one fixed-point add per pair present
    // in the wave
    const bool add = (val != 0.0 || err != 0.0) && !fail;
    unsigned long long rem = __ballot(add);
    while (rem) {
      const int leader = __ffsll((long long)rem) - 1;
      const int32_t pl = __shfl(w.p, leader);
      const bool mine = add && w.p == pl;
      const unsigned long long m = __ballot(mine);
      const double sum = wave_sum(mine ? val : 0.0);
      const double esum = A.est ? wave_sum(mine ? err : 0.0) : 0.0;
      if (lane == leader) {
        if (fabs(sum) < 1.0e14)
          fixed_add(&A.acc[2 * (int64_t)pl], sum);
        else
          atomicOr(&A.out.flags[pl], kFlagNonfinite);  // NaN or absurd: refitted
        if (A.est && esum < 1.0e14) fixed_add(&A.est[2 * (int64_t)pl], esum);
      }
      rem &= ~m;
    }
    if (fail) {
      self = 0;
      near_m = next_m = 0u;
    }
    // leaf pairs to the direct sum
    const int n_near_me = (self == 1 ? 1 : 0) + __popc(near_m);
    int64_t at = wave_reserve(n_near, n_near_me);
    bool over = false;
    if (n_near_me > 0) {
      const int ha = w.lev & 255, hb = w.lev >> 8;
      if (self == 1) {
        if (at < A.near_cap) A.near[at] = w; else over = true;
        ++at;
      }
      for (int c = 0; c < kBhArity; ++c) {
        if (!(near_m >> c & 1u)) continue;
        BhPair ch = w;
        if (split_a) {
          ch.ka = (int32_t)(cbase + c);
          ch.lev = hc | (hb << 8);
        } else {
          ch.kb = (int32_t)(cbase + c);
          ch.lev = ha | (hc << 8);
        }
        if (at < A.near_cap) A.near[at] = ch; else over = true;
        ++at;
      }
    }
    // pairs to split again, for the next step
    const int n_next_me = __popc(next_m);
    at = wave_reserve(n_out, n_next_me);
    if (n_next_me > 0) {
      const int ha = w.lev & 255, hb = w.lev >> 8;
      for (int c = 0; c < kBhArity; ++c) {
        if (!(next_m >> c & 1u)) continue;
        BhPair ch = w;
        if (split_a) {
          ch.ka = (int32_t)(cbase + c);
          ch.lev = hc | (hb << 8);
        } else {
          ch.kb = (int32_t)(cbase + c);
          ch.lev = ha | (hc << 8);
        }
        if (at < A.list_cap) out[at] = ch; else over = true;
        ++at;
      }
    }
    if (over) atomicOr(&A.out.flags[w.p], kFlagNonfinite);  // a list was full: refitted
  }
}

// --------------------------------------------------------------- finalise
__global__ __launch_bounds__(256) void bh_finalize_k(BhArgs A, int64_t n_pairs) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * 256) {
    const int32_t i = A.pairs[2 * p], j = A.pairs[2 * p + 1];
    if (i < 0 || j < 0 || i >= A.n_loops || j >= A.n_loops || i == j) continue;
    const int64_t na = A.off[i + 1] - A.off[i], nb = A.off[j + 1] - A.off[j];
    if (na < 1 || nb < 1 || na > 0x7fffffffLL || nb > 0x7fffffffLL) continue;
    finalize_pair(A.out, (int32_t)p, from_fixed(A.acc[2 * p], A.acc[2 * p + 1]), A.out.flags[p]);
  }
}

// -------------------------------------------------------- adaptive beta
__global__ __launch_bounds__(256) void bh_adapt_k(BhArgs A, int64_t n_pairs, double target,
                                                  double beta_max) {
  // the second traversal's lists and leaf list start empty (the count of
  // pairs evaluated again, at kBhMaxIters + 2, was cleared by the leaf kernel)
  if (blockIdx.x == 0 && threadIdx.x < kBhMaxIters + 2) A.counts[threadIdx.x] = 0;
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * 256) {
    double b = 0.0;
    if (!(A.out.flags[p] & kFlagNonfinite)) {  // a failed pair is refitted anyway
      const double E = from_fixed(A.est[2 * p], A.est[2 * p + 1]);
      const double bt = pow(E / target, 0.25) * A.beta;
      if (bt > A.beta) {
        b = fmin(bt, beta_max);
        A.acc[2 * p] = 0ull;
        A.acc[2 * p + 1] = 0ull;
        atomicAdd(&A.counts[kBhMaxIters + 2], 1);
      }
    }
    A.beta_p[p] = b;
  }
}

inline int grid_for(int64_t n, int per_block, int cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_bh_leaves(const BhArgs& a, bool in_f64, hipStream_t s) {
  const int g = grid_for(a.level_cap[0], 1, 65536);
  if (in_f64)
    bh_leaves_k<double><<<g, 64, 0, s>>>(a);
  else
    bh_leaves_k<float><<<g, 64, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_bh_level(const BhArgs& a, int level, hipStream_t s) {
  bh_level_k<<<grid_for(a.level_cap[level], 256, 4096), 256, 0, s>>>(a, level);
  return hipGetLastError();
}

hipError_t launch_bh_roots(const BhArgs& a, int64_t n_pairs, hipStream_t s) {
  bh_roots_k<<<grid_for(n_pairs, 256, 1024), 256, 0, s>>>(a, n_pairs);
  return hipGetLastError();
}

hipError_t launch_bh_expand(const BhArgs& a, int it, hipStream_t s) {
  bh_expand_k<<<2048, 256, 0, s>>>(a, it);
  return hipGetLastError();
}

hipError_t launch_bh_adapt(const BhArgs& a, int64_t n_pairs, double target, double beta_max,
                           hipStream_t s) {
  bh_adapt_k<<<grid_for(n_pairs, 256, 1024), 256, 0, s>>>(a, n_pairs, target, beta_max);
  return hipGetLastError();
}

hipError_t launch_bh_finalize(const BhArgs& a, int64_t n_pairs, hipStream_t s) {
  bh_finalize_k<<<grid_for(n_pairs, 256, 1024), 256, 0, s>>>(a, n_pairs);
  return hipGetLastError();
}

}  // namespace lk
