/*
 * lk_oracle.c -- plain FP64 CPU oracle for the direct-summation linking number.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header or constant with the HIP
 * library; it is written straight from the paper (Qu & James, "Fast Linking
 * Numbers for Topology Verification of Loopy Structures", SIGGRAPH 2021).
 *
 * What it computes (all in IEEE double, libm atan2/sqrt):
 *   - lko_term:       one segment-pair contribution, Eq. 4 exactly as printed
 *                     (van Oosterom-Strackee signed solid angle of the two
 *                     triangles (a,b,c) and (c,d,a)), divided by 2*pi.
 *   - lko_term_mid:   the midpoint quadrature of Eq. 2 for the same pair
 *                     (inexact; used only as a far-field / sign pin).
 *   - lko_pair:       the double sum of Eq. 3 in the order of Alg. 5:
 *                     outer index i over loop k (gamma_2), inner j over loop l
 *                     (gamma_1), with a Neumaier-compensated sum over j per
 *                     row and a Neumaier sum over fixed blocks of rows.
 *   - lko_pair_anglesum: the angle-summation form of the appendix (Alg. 7),
 *                     a second, differently-organised evaluation of the same
 *                     value (complex-product accumulation, integer wrap count,
 *                     one atan2 per row).
 *   - lko_direct_sum: lko_pair over a pair list with a pthread pool; the
 *                     result per pair does not depend on the thread count.
 *   - lko_loop_flags: per-loop validity (at least 3 vertices, finite
 *                     coordinates, no segment shorter than eps*xi where xi is
 *                     the mean coordinate magnitude -- Sec. 3.3, Alg. 3).
 *   - lko_aabb_pairs: brute-force potential link search (Alg. 2): every i<j
 *                     whose closed axis-aligned boxes overlap, lexicographic.
 *   - lko_crossings:  brute-force crossing count (Sec. 2.1, Alg. 4 without
 *                     the BVH): rotate by a given frame, project to xy, add
 *                     +-1/2 per crossing; flags near-degenerate projections.
 *   - lko_bh_pair:    two-tree Barnes-Hut (Sec. 3.4.4, Alg. 6) over trees of
 *                     consecutive-segment ranges, far field to dipole or
 *                     quadrupole order, Eq. 4 at leaf pairs, with the
 *                     next-order error estimate; lko_bh_node_moments and
 *                     lko_bh_far_pieces expose its moments and far field for
 *                     the pins.
 *   - lko_discretize: the adaptive discretization of Alg. 3 (Sec. 3.3):
 *                     B-spline or polyline loops refined into polylines by
 *                     passes over overlapping piece boxes of paired loops.
 *
 * Readings of the paper used here (also listed in the design notes):
 *   - vertex indices are cyclic: loop of n vertices has n segments, the first
 *     vertex is not repeated (Alg. 5 uses k_{i+1}, l_{j+1} at the last index);
 *   - atan(y/x) means atan2(y, x) (stated with Eq. 4);
 *   - pair (i, j): loop i plays gamma_1 (vertices l, index j), loop j plays
 *     gamma_2 (vertices k, index i);
 *   - the integer is round-half-away-from-zero of the real sum.
 *
 * A global mutation switch (lko_set_mutation) plants deliberate mistakes for
 * the tests that prove the pins catch them; it is 0 (off) by default
 * (1-6: the Eq. 4 term and the pair sum; 7, 8: the Barnes-Hut expansion;
 * 9-12: the discretization of Alg. 3; 13: the Barnes-Hut error estimate).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define LKO_PI 3.14159265358979323846

static int g_mutation = 0;

void lko_set_mutation(int m) { g_mutation = m; }
int lko_get_mutation(void) { return g_mutation; }

/* ---------------------------------------------------------------- vectors */
static void sub3(const double* p, const double* q, double* r) {
  r[0] = p[0] - q[0];
  r[1] = p[1] - q[1];
  r[2] = p[2] - q[2];
}
static double dot3(const double* p, const double* q) {
  return p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
}
static void cross3(const double* p, const double* q, double* r) {
  r[0] = p[1] * q[2] - p[2] * q[1];
  r[1] = p[2] * q[0] - p[0] * q[2];
  r[2] = p[0] * q[1] - p[1] * q[0];
}
static double norm3(const double* p) { return sqrt(dot3(p, p)); }

/* ------------------------------------------------------- Neumaier sums */
typedef struct {
  double s, c;
} nsum;
static void nsum_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static double nsum_get(const nsum* a) { return a->s + a->c; }

/* ------------------------------------------------------------ Eq. 4 term */
/*
 * Contribution of segment (lj -> lj1) of gamma_1 and segment (ki -> ki1) of
 * gamma_2 (Eq. 4):
 *   a = l_j - k_i, b = l_j - k_{i+1}, c = l_{j+1} - k_{i+1}, d = l_{j+1} - k_i
 *   lambda = [atan2(a.(b x c), D1) + atan2(c.(d x a), D2)] / (2 pi)
 *   D1 = |a||b||c| + (a.b)|c| + (c.a)|b| + (b.c)|a|
 *   D2 = |c||d||a| + (c.d)|a| + (a.c)|d| + (d.a)|c|
 * Both numerators are evaluated as printed (no use of the identity that makes
 * them equal), so the identity itself can be checked against this routine.
 */
double lko_term(const double* lj, const double* lj1, const double* ki, const double* ki1) {
  double a[3], b[3], c[3], d[3], t[3];
  if (g_mutation == 4) { /* transposed operand: a = k_i - l_j etc. */
    sub3(ki, lj, a);
    sub3(ki1, lj, b);
    sub3(ki1, lj1, c);
    sub3(ki, lj1, d);
  } else {
    sub3(lj, ki, a);
    sub3(lj, ki1, b);
    sub3(lj1, ki1, c);
    sub3(lj1, ki, d);
  }
  if (g_mutation == 3) sub3(lj1, ki, c); /* wrong index in c */
  double na = norm3(a), nb = norm3(b), nc = norm3(c), nd = norm3(d);
  cross3(b, c, t);
  double p1 = dot3(a, t);
  cross3(d, a, t);
  double p2 = dot3(c, t);
  if (g_mutation == 2) p2 = -p2; /* wrong sign in the second arctangent */
  double d1 = na * nb * nc + dot3(a, b) * nc + dot3(c, a) * nb + dot3(b, c) * na;
  if (g_mutation == 1) d1 = na * nb * nc + dot3(a, b) * nc + dot3(b, c) * na; /* dropped term */
  double d2 = nc * nd * na + dot3(c, d) * na + dot3(a, c) * nd + dot3(d, a) * nc;
  double scale = (g_mutation == 6) ? 4.0 * LKO_PI : 2.0 * LKO_PI;
  return (atan2(p1, d1) + atan2(p2, d2)) / scale;
}

/* Midpoint quadrature of Eq. 2 for one segment pair (r = midpoints,
 * s = segment vectors): (r_j - r_i)/|r_j - r_i|^3 . (s_j x s_i) / (4 pi). */
double lko_term_mid(const double* lj, const double* lj1, const double* ki, const double* ki1) {
  double rj[3], ri[3], sj[3], si[3], R[3], x[3];
  for (int q = 0; q < 3; ++q) {
    rj[q] = 0.5 * (lj[q] + lj1[q]);
    ri[q] = 0.5 * (ki[q] + ki1[q]);
  }
  sub3(lj1, lj, sj);
  sub3(ki1, ki, si);
  sub3(rj, ri, R);
  cross3(sj, si, x);
  double r = norm3(R);
  return dot3(R, x) / (r * r * r) / (4.0 * LKO_PI);
}

/* ------------------------------------------------------- one loop pair */
/* Rows are grouped in fixed blocks so that the threaded driver can split a
 * huge pair without changing the result: row block sums are Neumaier sums of
 * Neumaier row sums, and the pair value is a Neumaier sum of block sums in
 * order. */
#define LKO_ROWBLOCK 1024

static double row_block(const double* L, int64_t nl, const double* K, int64_t nk, int64_t i0,
                        int64_t i1) {
  nsum blk = {0, 0};
  int64_t njs = (g_mutation == 5) ? nl - 1 : nl; /* mutation 5: open loop */
  for (int64_t i = i0; i < i1; ++i) {
    const double* ki = K + 3 * i;
    const double* ki1 = K + 3 * ((i + 1) % nk);
    nsum row = {0, 0};
    for (int64_t j = 0; j < njs; ++j) {
      const double* lj = L + 3 * j;
      const double* lj1 = L + 3 * ((j + 1) % nl);
      nsum_add(&row, lko_term(lj, lj1, ki, ki1));
    }
    nsum_add(&blk, nsum_get(&row));
  }
  return nsum_get(&blk);
}

/* Linking number of gamma_1 = loop L (nl vertices) and gamma_2 = loop K (nk
 * vertices), both as xyz triples, following Alg. 5. */
double lko_pair(const double* L, int64_t nl, const double* K, int64_t nk) {
  nsum tot = {0, 0};
  for (int64_t i0 = 0; i0 < nk; i0 += LKO_ROWBLOCK) {
    int64_t i1 = i0 + LKO_ROWBLOCK < nk ? i0 + LKO_ROWBLOCK : nk;
    nsum_add(&tot, row_block(L, nl, K, nk, i0, i1));
  }
  return nsum_get(&tot);
}

/* s(x, y) of Alg. 7: +1 when the angle of (x, y) lies in (0, pi], else -1. */
static int half_plane(double x, double y) { return (y > 0.0 || (y == 0.0 && x < 0.0)) ? 1 : -1; }

/* The angle-summation evaluation of the appendix (Alg. 7).  Per row i the
 * contributions are multiplied together as complex numbers; every time the
 * accumulated angle passes through the negative real axis an integer turn is
 * recorded, and one atan2 at the end adds the remainder.  Used to pin the
 * equivalence of both forms, not as the main oracle. */
double lko_pair_anglesum(const double* L, int64_t nl, const double* K, int64_t nk) {
  nsum tot = {0, 0};
  for (int64_t i = 0; i < nk; ++i) {
    const double* ki = K + 3 * i;
    const double* ki1 = K + 3 * ((i + 1) % nk);
    double xs = 1.0, ys = 0.0;
    int S = -1;
    long turns = 0; /* whole turns (2*pi) of the summed angle, i.e. whole units of linking */
    for (int64_t j = 0; j < nl; ++j) {
      const double* lj = L + 3 * j;
      const double* lj1 = L + 3 * ((j + 1) % nl);
      double a[3], b[3], c[3], d[3], t[3];
      sub3(lj, ki, a);
      sub3(lj, ki1, b);
      sub3(lj1, ki1, c);
      sub3(lj1, ki, d);
      double na = norm3(a), nb = norm3(b), nc = norm3(c), nd = norm3(d);
      cross3(b, c, t);
      double p = dot3(a, t);
      double d1 = na * nb * nc + dot3(a, b) * nc + dot3(b, c) * na + dot3(c, a) * nb;
      double d2 = na * nd * nc + dot3(a, d) * nc + dot3(d, c) * na + dot3(c, a) * nd;
      double xp = d1 * d2 - p * p;
      double yp = p * (d1 + d2);
      int s1 = half_plane(d1, p), s2 = half_plane(d2, p), sp = half_plane(xp, yp);
      if (s1 * s2 > 0 && s1 * sp < 0) turns += s1;
      double xpp = xs * xp - ys * yp;
      double ypp = xs * yp + ys * xp;
      int spp = half_plane(xpp, ypp);
      if (sp * S > 0 && spp * S < 0) turns += S;
      S = spp;
      double m = fabs(xpp) > fabs(ypp) ? fabs(xpp) : fabs(ypp);
      xs = xpp / m;
      ys = ypp / m;
    }
    /* each recorded turn is one full turn (2*pi) of the summed angles, and the
     * summed angles are 2*pi times the linking contribution */
    nsum_add(&tot, (double)turns + atan2(ys, xs) / (2.0 * LKO_PI));
  }
  return nsum_get(&tot);
}

/* ------------------------------------------------------ threaded driver */
typedef struct {
  const double* xyz;
  const int64_t* off;
  const int32_t* pairs;
  int64_t npairs;
  /* work items: (pair, row block) */
  const int64_t* item_start; /* first item of each pair, npairs+1 entries */
  double* block_out;         /* one partial per item */
  int64_t next;              /* shared counter */
  pthread_mutex_t mu;
} lko_job;

static int64_t find_pair(const int64_t* start, int64_t n, int64_t w) {
  int64_t lo = 0, hi = n; /* largest p with start[p] <= w */
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (start[mid] <= w)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

static void* worker(void* arg) {
  lko_job* J = (lko_job*)arg;
  const int64_t total = J->item_start[J->npairs];
  for (;;) {
    pthread_mutex_lock(&J->mu);
    int64_t w = J->next;
    J->next += 1;
    pthread_mutex_unlock(&J->mu);
    if (w >= total) break;
    int64_t p = find_pair(J->item_start, J->npairs, w);
    int64_t blk = w - J->item_start[p];
    int32_t li = J->pairs[2 * p], lj = J->pairs[2 * p + 1];
    const double* L = J->xyz + 3 * J->off[li];
    int64_t nl = J->off[li + 1] - J->off[li];
    const double* K = J->xyz + 3 * J->off[lj];
    int64_t nk = J->off[lj + 1] - J->off[lj];
    int64_t i0 = blk * LKO_ROWBLOCK;
    int64_t i1 = i0 + LKO_ROWBLOCK < nk ? i0 + LKO_ROWBLOCK : nk;
    J->block_out[w] = row_block(L, nl, K, nk, i0, i1);
  }
  return NULL;
}

/*
 * Linking numbers for a pair list.  xyz: V x 3 doubles; off: L+1 vertex
 * offsets; pairs: P x 2 loop indices (loop pairs[2p] is gamma_1).  Writes the
 * real sum to out_real[p] and round-half-away-from-zero to out_int[p] (either
 * may be NULL).  Pairs with an index out of range or i == j get NaN and
 * INT32_MIN.  Returns 0, or -1 on allocation failure.
 */
int lko_direct_sum(const double* xyz, const int64_t* off, int32_t nloops, const int32_t* pairs,
                   int64_t npairs, double* out_real, int32_t* out_int, int nthreads) {
  int64_t* start = (int64_t*)malloc(sizeof(int64_t) * (size_t)(npairs + 1));
  if (!start) return -1;
  start[0] = 0;
  for (int64_t p = 0; p < npairs; ++p) {
    int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
    int64_t nb = 0;
    if (a >= 0 && b >= 0 && a < nloops && b < nloops && a != b) {
      int64_t nk = off[b + 1] - off[b];
      nb = (nk + LKO_ROWBLOCK - 1) / LKO_ROWBLOCK;
    }
    start[p + 1] = start[p] + nb;
  }
  double* blocks = (double*)malloc(sizeof(double) * (size_t)(start[npairs] + 1));
  if (!blocks) {
    free(start);
    return -1;
  }
  lko_job J;
  J.xyz = xyz;
  J.off = off;
  J.pairs = pairs;
  J.npairs = npairs;
  J.item_start = start;
  J.block_out = blocks;
  J.next = 0;
  pthread_mutex_init(&J.mu, NULL);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  pthread_t th[256];
  int started = 0;
  for (int t = 1; t < nthreads; ++t)
    if (pthread_create(&th[started], NULL, worker, &J) == 0) ++started;
  worker(&J);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  pthread_mutex_destroy(&J.mu);
  for (int64_t p = 0; p < npairs; ++p) {
    int32_t a = pairs[2 * p], b = pairs[2 * p + 1];
    double v;
    if (!(a >= 0 && b >= 0 && a < nloops && b < nloops && a != b)) {
      v = NAN;
    } else {
      nsum tot = {0, 0};
      for (int64_t w = start[p]; w < start[p + 1]; ++w) nsum_add(&tot, blocks[w]);
      v = nsum_get(&tot);
    }
    if (out_real) out_real[p] = v;
    if (out_int) out_int[p] = isfinite(v) ? (int32_t)lround(v) : INT32_MIN;
  }
  free(blocks);
  free(start);
  return 0;
}

/* ----------------------------------------------------------- verification */
/*
 * The before/after comparison of Sec. 3.1 ("Fast Verification"): the current
 * sparse linking matrix (pairs, lk)[n] against the expected one
 * (exp_pairs, exp_lk)[n_exp], both sorted lexicographically by (i, j) with no
 * duplicates.  A pair missing from one side has the value 0 there (a pair
 * the potential link search no longer lists has separated boxes, so its
 * linking number is 0).  Every pair whose two values differ is a mismatch.
 * The first `cap` mismatches in pair order go to out[cap][4] as
 * (i, j, current, expected); returns their total count.
 */
static int key_cmp(const int32_t* a, const int32_t* b) {
  if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
  if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
  return 0;
}

int64_t lko_verify(const int32_t* pairs, const int32_t* lk, int64_t n, const int32_t* exp_pairs,
                   const int32_t* exp_lk, int64_t n_exp, int32_t* out, int64_t cap) {
  int64_t a = 0, b = 0, count = 0;
  while (a < n || b < n_exp) {
    int c;
    if (a == n)
      c = 1;
    else if (b == n_exp)
      c = -1;
    else
      c = key_cmp(&pairs[2 * a], &exp_pairs[2 * b]);
    const int32_t* key = c <= 0 ? &pairs[2 * a] : &exp_pairs[2 * b];
    /* mutation 14: a pair only in the expected list takes its expected value */
    const int32_t got = c <= 0 ? lk[a] : (g_mutation == 14 ? exp_lk[b] : 0);
    const int32_t want = c >= 0 ? exp_lk[b] : 0;
    if (got != want) {
      if (count < cap) {
        out[4 * count] = key[0];
        out[4 * count + 1] = key[1];
        out[4 * count + 2] = got;
        out[4 * count + 3] = want;
      }
      ++count;
    }
    if (c <= 0) ++a;
    if (c >= 0) ++b;
  }
  return count;
}

/* ----------------------------------------------------------- validation */
/* Loop flags: 16 = bad loop (fewer than 3 vertices, or a segment of length
 * below eps * xi, Alg. 3's zero-length test), 4 = non-finite coordinate.
 * xi = mean |coordinate| over every coordinate of every vertex. */
int lko_loop_flags(const double* xyz, const int64_t* off, int32_t nloops, double eps,
                   uint32_t* flags) {
  int64_t nv = off[nloops] - off[0];
  double acc = 0.0;
  for (int64_t v = off[0]; v < off[nloops]; ++v)
    for (int q = 0; q < 3; ++q) acc += fabs(xyz[3 * v + q]);
  double xi = nv > 0 ? acc / (3.0 * (double)nv) : 0.0;
  for (int32_t l = 0; l < nloops; ++l) {
    uint32_t f = 0;
    int64_t n = off[l + 1] - off[l];
    const double* X = xyz + 3 * off[l];
    if (n < 3) f |= 16u;
    for (int64_t s = 0; s < n; ++s) {
      for (int q = 0; q < 3; ++q)
        if (!isfinite(X[3 * s + q])) f |= 4u;
      double e[3];
      sub3(X + 3 * ((s + 1) % n), X + 3 * s, e);
      if (n >= 2 && norm3(e) < eps * xi) f |= 16u;
    }
    flags[l] = f;
  }
  return 0;
}

/* ------------------------------------------------- potential link search */
/* All pairs i<j whose closed AABBs (vertex min/max) overlap on x, y and z,
 * in lexicographic order.  Writes at most cap pairs and returns the total
 * count. */
int64_t lko_aabb_pairs(const double* xyz, const int64_t* off, int32_t nloops, int32_t* out,
                       int64_t cap) {
  double* box = (double*)malloc(sizeof(double) * 6 * (size_t)(nloops > 0 ? nloops : 1));
  if (!box) return -1;
  for (int32_t l = 0; l < nloops; ++l) {
    double* B = box + 6 * l;
    B[0] = B[1] = B[2] = INFINITY;
    B[3] = B[4] = B[5] = -INFINITY;
    for (int64_t v = off[l]; v < off[l + 1]; ++v)
      for (int q = 0; q < 3; ++q) {
        double x = xyz[3 * v + q];
        if (x < B[q]) B[q] = x;
        if (x > B[3 + q]) B[3 + q] = x;
      }
  }
  int64_t n = 0;
  for (int32_t i = 0; i < nloops; ++i)
    for (int32_t j = i + 1; j < nloops; ++j) {
      const double* P = box + 6 * i;
      const double* Q = box + 6 * j;
      int ov = 1;
      for (int q = 0; q < 3; ++q)
        if (P[q] > Q[3 + q] || Q[q] > P[3 + q]) ov = 0;
      if (ov) {
        if (n < cap) {
          out[2 * n] = i;
          out[2 * n + 1] = j;
        }
        ++n;
      }
    }
  free(box);
  return n;
}

/* --------------------------------------------------- crossing count */
/*
 * Brute-force crossings (the count-crossings definition of Sec. 2.1 without
 * acceleration).  R is a row-major 3x3 rotation; both loops are mapped by
 * x -> R x and projected onto the xy plane, viewed from +z.  Every pair of
 * projected segments that cross contributes +-1/2 with sign
 * sign( (t_over x t_under) . z ), t = segment direction, "over" = larger z at
 * the crossing.  If any segment pair is close to a non-regular configuration
 * (parallel, crossing near an endpoint, or equal depth), *degenerate is set to
 * 1 and the caller should draw a new frame.
 */
double lko_crossings(const double* L, int64_t nl, const double* K, int64_t nk, const double* R,
                     int* degenerate) {
  double* PL = (double*)malloc(sizeof(double) * 3 * (size_t)nl);
  double* PK = (double*)malloc(sizeof(double) * 3 * (size_t)nk);
  *degenerate = 0;
  if (!PL || !PK) {
    free(PL);
    free(PK);
    *degenerate = 1;
    return 0.0;
  }
  double scale = 0.0;
  for (int64_t v = 0; v < nl; ++v)
    for (int q = 0; q < 3; ++q) {
      PL[3 * v + q] = R[3 * q] * L[3 * v] + R[3 * q + 1] * L[3 * v + 1] + R[3 * q + 2] * L[3 * v + 2];
      if (fabs(PL[3 * v + q]) > scale) scale = fabs(PL[3 * v + q]);
    }
  for (int64_t v = 0; v < nk; ++v)
    for (int q = 0; q < 3; ++q) {
      PK[3 * v + q] = R[3 * q] * K[3 * v] + R[3 * q + 1] * K[3 * v + 1] + R[3 * q + 2] * K[3 * v + 2];
      if (fabs(PK[3 * v + q]) > scale) scale = fabs(PK[3 * v + q]);
    }
  const double tol = 1e-12;
  long twice = 0; /* sum of signs; the linking number is half of it */
  for (int64_t i = 0; i < nk; ++i) {
    const double* p0 = PK + 3 * i;
    const double* p1 = PK + 3 * ((i + 1) % nk);
    double ux = p1[0] - p0[0], uy = p1[1] - p0[1];
    for (int64_t j = 0; j < nl; ++j) {
      const double* q0 = PL + 3 * j;
      const double* q1 = PL + 3 * ((j + 1) % nl);
      double vx = q1[0] - q0[0], vy = q1[1] - q0[1];
      double den = ux * vy - uy * vx; /* cross(u, v) */
      double wx = q0[0] - p0[0], wy = q0[1] - p0[1];
      double su = (wx * vy - wy * vx); /* t * den  for point p0 + t u */
      double sv = (wx * uy - wy * ux); /* s * den  for point q0 + s v */
      double lu = sqrt(ux * ux + uy * uy), lv = sqrt(vx * vx + vy * vy);
      if (fabs(den) <= tol * lu * lv) {
        /* (near-)parallel projected segments: degenerate only if they touch */
        double dist = fabs(wx * uy - wy * ux) / (lu > 0 ? lu : 1.0);
        if (dist <= 1e-9 * scale) *degenerate = 1;
        continue;
      }
      double t = su / den, s = sv / den;
      double et = 1e-9, es = 1e-9;
      if (t < -et || t > 1.0 + et || s < -es || s > 1.0 + es) continue;
      if (t < et || t > 1.0 - et || s < es || s > 1.0 - es) {
        *degenerate = 1; /* crossing at (or too close to) a vertex */
        continue;
      }
      double zk = p0[2] + t * (p1[2] - p0[2]);
      double zl = q0[2] + s * (q1[2] - q0[2]);
      if (fabs(zk - zl) <= 1e-9 * scale) {
        *degenerate = 1; /* the curves (nearly) meet in space */
        continue;
      }
      /* over segment first: sign of (t_over x t_under).z */
      double c = (zk > zl) ? (ux * vy - uy * vx) : (vx * uy - vy * ux);
      twice += (c > 0) ? 1 : -1;
    }
  }
  free(PL);
  free(PK);
  return 0.5 * (double)twice;
}

/* ------------------------------------------------------------ Barnes-Hut */
/*
 * Two-tree Barnes-Hut linking number of Sec. 3.4.4 (Alg. 6), FP64.
 *
 * Trees: a loop of n segments is cut into leaves of `leaf` consecutive
 * segments; a node of level h covers leaf * arity^h consecutive segments (the
 * last node of a level may cover fewer) and its children are the nodes of
 * level h - 1 inside it; the root is the lowest level with a single node.  A
 * node's centre is the centre of the axis-aligned box of its vertices (the
 * vertex that closes its last segment included) and R is half the box
 * diagonal.
 *
 * Moments about the centre (the monopole, dipole and quadrupole moments of
 * Sec. 3.4.4), computed directly from the node's segments: a segment with
 * vector s and midpoint m, d = m - centre, adds s to c_M, s d^T to C_D and
 * s (x) d (x) d + s (x) s (x) s / 12 to C_Q (the integrals over the segment).
 *
 * Evaluation (Alg. 6): nodes with |c2 - c1| > beta (R1 + R2) use the far-field
 * expansion (lambda = -(sum of the expansion terms) for the Taylor series of
 * the Gauss integral in both curves), to `order` 1 (monopole and dipole
 * terms) or 2 (also the quadrupole term), with the derivatives of
 * G = -1/(4 pi |r1 - r2|) at r = c2 - c1; two leaves use Eq. 4 over all their
 * segment pairs; otherwise the node that has children and the larger R is
 * split.  Reading: a leaf is never split (the printed algorithm would recurse
 * into the children of a leaf when its R is the larger one).
 *
 * *err_est (when not NULL) receives the next-order error estimate summed over
 * the far-field node pairs, with the constant k = 1/(4 pi) (the paper leaves k
 * unspecified).
 */
typedef struct {
  double c[3], R;
  double M[3], D[9], Q[27];
  int64_t a, b; /* segments [a, b) */
  int level;
  int64_t k; /* index within its level */
} bh_node;

typedef struct {
  const double* P; /* vertices */
  int64_t n;       /* segments = vertices */
  int64_t leaf, arity;
  int levels;
  int64_t* start; /* first node of each level in nodes[] */
  int64_t* count; /* nodes per level */
  bh_node* nodes;
} bh_tree;

static const double* bh_vtx(const bh_tree* t, int64_t v) { return t->P + 3 * (v % t->n); }

static void bh_node_init(const bh_tree* t, bh_node* nd) {
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t v = nd->a; v <= nd->b; ++v) {
    const double* x = bh_vtx(t, v);
    for (int q = 0; q < 3; ++q) {
      if (x[q] < lo[q]) lo[q] = x[q];
      if (x[q] > hi[q]) hi[q] = x[q];
    }
  }
  double diag = 0.0;
  for (int q = 0; q < 3; ++q) {
    nd->c[q] = 0.5 * (lo[q] + hi[q]);
    diag += (hi[q] - lo[q]) * (hi[q] - lo[q]);
  }
  nd->R = 0.5 * sqrt(diag);
  memset(nd->M, 0, sizeof(nd->M));
  memset(nd->D, 0, sizeof(nd->D));
  memset(nd->Q, 0, sizeof(nd->Q));
  for (int64_t s = nd->a; s < nd->b; ++s) {
    const double* x0 = bh_vtx(t, s);
    const double* x1 = bh_vtx(t, s + 1);
    double sv[3], d[3];
    for (int q = 0; q < 3; ++q) {
      sv[q] = x1[q] - x0[q];
      d[q] = 0.5 * (x0[q] + x1[q]) - nd->c[q];
    }
    const double q12 = (g_mutation == 8) ? 0.0 : 1.0 / 12.0; /* mutation 8: drops s(x)s(x)s/12 */
    for (int p = 0; p < 3; ++p) {
      nd->M[p] += sv[p];
      for (int b = 0; b < 3; ++b) {
        nd->D[3 * p + b] += sv[p] * d[b];
        for (int c = 0; c < 3; ++c)
          nd->Q[9 * p + 3 * b + c] += sv[p] * d[b] * d[c] + q12 * sv[p] * sv[b] * sv[c];
      }
    }
  }
}

static int bh_build(bh_tree* t, const double* P, int64_t n, int64_t leaf, int64_t arity) {
  t->P = P;
  t->n = n;
  t->leaf = leaf;
  t->arity = arity;
  int levels = 1;
  int64_t span = leaf, total = 0;
  while ((n + span - 1) / span > 1) {
    span *= arity;
    ++levels;
  }
  t->levels = levels;
  t->start = (int64_t*)malloc(sizeof(int64_t) * levels);
  t->count = (int64_t*)malloc(sizeof(int64_t) * levels);
  span = leaf;
  for (int h = 0; h < levels; ++h) {
    t->start[h] = total;
    t->count[h] = (n + span - 1) / span;
    total += t->count[h];
    span *= arity;
  }
  t->nodes = (bh_node*)malloc(sizeof(bh_node) * (size_t)total);
  if (!t->start || !t->count || !t->nodes) return 0;
  span = leaf;
  for (int h = 0; h < levels; ++h) {
    for (int64_t k = 0; k < t->count[h]; ++k) {
      bh_node* nd = &t->nodes[t->start[h] + k];
      nd->a = k * span;
      nd->b = (k + 1) * span < n ? (k + 1) * span : n;
      nd->level = h;
      nd->k = k;
      bh_node_init(t, nd);
    }
    span *= arity;
  }
  return 1;
}

static void bh_free(bh_tree* t) {
  free(t->start);
  free(t->count);
  free(t->nodes);
}

static double fro(const double* x, int n) {
  double s = 0.0;
  for (int q = 0; q < n; ++q) s += x[q] * x[q];
  return sqrt(s);
}

/* Far field of nodes u (curve 1) and v (curve 2). */
static double bh_far(const bh_node* u, const bh_node* v, int order, double* err) {
  static const int eps[3][3][3] = {{{0, 0, 0}, {0, 0, 1}, {0, -1, 0}},
                                   {{0, 0, -1}, {0, 0, 0}, {1, 0, 0}},
                                   {{0, 1, 0}, {-1, 0, 0}, {0, 0, 0}}};
  double r[3];
  sub3(v->c, u->c, r);
  const double d2 = dot3(r, r), d = sqrt(d2), f = 1.0 / (4.0 * LKO_PI);
  const double d3 = d2 * d, d5 = d3 * d2, d7 = d5 * d2;
  double g[3], H[9], K[27];
  for (int a = 0; a < 3; ++a) g[a] = f * r[a] / d3;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) H[3 * a + b] = f * ((a == b ? d2 : 0.0) - 3.0 * r[a] * r[b]) / d5;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c) {
        const double sym = r[a] * (b == c) + r[b] * (a == c) + r[c] * (a == b);
        K[9 * a + 3 * b + c] = f * (-3.0 * sym / d5 + 15.0 * r[a] * r[b] * r[c] / d7);
      }
  /* T1 = (M1 x M2) . g */
  double t1 = 0.0, t2 = 0.0, t3 = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int p = 0; p < 3; ++p)
      for (int q = 0; q < 3; ++q) {
        if (!eps[a][p][q]) continue;
        const double e = eps[a][p][q];
        t1 += e * u->M[p] * v->M[q] * g[a];
        /* T2: sum_b H_ab (-D1[p][b] M2[q] + M1[p] D2[q][b]) */
        for (int b = 0; b < 3; ++b) {
          const double m = -u->D[3 * p + b] * v->M[q] + u->M[p] * v->D[3 * q + b];
          t2 += e * H[3 * a + b] * ((g_mutation == 7) ? -m : m); /* mutation 7: dipole sign */
        }
        if (order >= 2)
          for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
              const double m = u->Q[9 * p + 3 * b + c] * v->M[q] -
                               u->D[3 * p + b] * v->D[3 * q + c] -
                               u->D[3 * p + c] * v->D[3 * q + b] +
                               u->M[p] * v->Q[9 * q + 3 * b + c];
              t3 += 0.5 * e * K[9 * a + 3 * b + c] * m;
            }
      }
  if (err) {
    const double nM1 = norm3(u->M), nM2 = norm3(v->M);
    const double nD1 = fro(u->D, 9), nD2 = fro(v->D, 9), nQ1 = fro(u->Q, 27), nQ2 = fro(v->Q, 27);
    const double cross = (g_mutation == 13) ? 0.0 : 3.0 * (nD1 * nQ2 + nQ1 * nD2); /* mutation 13 */
    *err += f / d5 * (u->R * nM2 * nQ1 + v->R * nM1 * nQ2 + cross);
  }
  return -(t1 + t2 + t3);
}

static double bh_rec(const bh_tree* A, const bh_tree* B, const bh_node* u, const bh_node* v,
                     double beta, int order, double* err) {
  double r[3];
  sub3(v->c, u->c, r);
  if (norm3(r) > beta * (u->R + v->R)) return bh_far(u, v, order, err);
  const int leaf_u = u->level == 0, leaf_v = v->level == 0;
  if (leaf_u && leaf_v) {
    double s = 0.0;
    for (int64_t j = u->a; j < u->b; ++j)
      for (int64_t i = v->a; i < v->b; ++i)
        s += lko_term(bh_vtx(A, j), bh_vtx(A, j + 1), bh_vtx(B, i), bh_vtx(B, i + 1));
    return s;
  }
  double s = 0.0;
  if (!leaf_u && (leaf_v || u->R > v->R)) {
    const int h = u->level - 1;
    for (int64_t k = u->k * A->arity; k < (u->k + 1) * A->arity && k < A->count[h]; ++k)
      s += bh_rec(A, B, &A->nodes[A->start[h] + k], v, beta, order, err);
  } else {
    const int h = v->level - 1;
    for (int64_t k = v->k * B->arity; k < (v->k + 1) * B->arity && k < B->count[h]; ++k)
      s += bh_rec(A, B, u, &B->nodes[B->start[h] + k], beta, order, err);
  }
  return s;
}

double lko_bh_pair(const double* L, int64_t nl, const double* K, int64_t nk, double beta,
                   int order, int64_t leaf, int64_t arity, double* err_est) {
  bh_tree A, B;
  memset(&A, 0, sizeof(A));
  memset(&B, 0, sizeof(B));
  if (err_est) *err_est = 0.0;
  if (nl < 1 || nk < 1 || leaf < 1 || arity < 2) return NAN;
  if (!bh_build(&A, L, nl, leaf, arity) || !bh_build(&B, K, nk, leaf, arity)) {
    bh_free(&A);
    bh_free(&B);
    return NAN;
  }
  const double v = bh_rec(&A, &B, &A.nodes[A.start[A.levels - 1]], &B.nodes[B.start[B.levels - 1]],
                          beta, order, err_est);
  bh_free(&A);
  bh_free(&B);
  return v;
}

/* Moments of the node covering segments [a, b) of one loop about the centre
 * of its box, computed directly (for the shift-rule pin).  out: c[3], R,
 * M[3], D[9], Q[27] (43 values). */
void lko_bh_node_moments(const double* P, int64_t n, int64_t a, int64_t b, double* out) {
  bh_tree t;
  memset(&t, 0, sizeof(t));
  t.P = P;
  t.n = n;
  bh_node nd;
  nd.a = a;
  nd.b = b;
  nd.level = 0;
  nd.k = 0;
  bh_node_init(&t, &nd);
  memcpy(out, nd.c, 3 * sizeof(double));
  out[3] = nd.R;
  memcpy(out + 4, nd.M, 3 * sizeof(double));
  memcpy(out + 7, nd.D, 9 * sizeof(double));
  memcpy(out + 16, nd.Q, 27 * sizeof(double));
}

/* Far-field estimate for the node of loop 1 covering segments [a1, b1) and
 * the node of loop 2 covering [a2, b2) (moments about their box centres), and
 * the exact Eq. 4 sum over the same segment pairs (*exact).  For the pins of
 * the expansion's order. */
double lko_bh_far_pieces(const double* P1, int64_t n1, int64_t a1, int64_t b1, const double* P2,
                         int64_t n2, int64_t a2, int64_t b2, int order, double* exact) {
  bh_tree t1, t2;
  memset(&t1, 0, sizeof(t1));
  memset(&t2, 0, sizeof(t2));
  t1.P = P1;
  t1.n = n1;
  t2.P = P2;
  t2.n = n2;
  bh_node u, v;
  u.a = a1;
  u.b = b1;
  u.level = 0;
  u.k = 0;
  v.a = a2;
  v.b = b2;
  v.level = 0;
  v.k = 0;
  bh_node_init(&t1, &u);
  bh_node_init(&t2, &v);
  if (exact) {
    double s = 0.0;
    for (int64_t j = a1; j < b1; ++j)
      for (int64_t i = a2; i < b2; ++i)
        s += lko_term(bh_vtx(&t1, j), bh_vtx(&t1, j + 1), bh_vtx(&t2, i), bh_vtx(&t2, i + 1));
    *exact = s;
  }
  return bh_far(&u, &v, order, NULL);
}

/* ---------------------------------------------------------- discretization */
/*
 * Adaptive discretization of Sec. 3.3 (Alg. 3), FP64.
 *
 * Input loops (kind 0): closed uniform cubic B-splines.  Loop i has control
 * points ctrl[cp_off[i] .. cp_off[i+1]) (m of them) and m spans; span s uses
 * control points s-1, s, s+1, s+2 (cyclic) and is written as the cubic Bezier
 * piece b0 = (q0 + 4 q1 + q2)/6, b1 = (2 q1 + q2)/3, b2 = (q1 + 2 q2)/3,
 * b3 = (q1 + 4 q2 + q3)/6.  Kind 1: closed polylines; segment s from vertex s
 * to s+1 is the piece (v_s, v_s, v_s+1, v_s+1) and is split at its midpoint.
 * A piece's bounding box is the box of its four points (the curve lies in
 * their convex hull, which the paper's proofs require of the bounding
 * volume).
 *
 * Validation first: a loop with fewer than 3 points, a non-finite
 * coordinate, or a piece whose box diagonal is below eps * xi (the
 * zero-length test; xi = mean over all points of (|x| + |y| + |z|) / 3) is
 * flagged BADLOOP (16), and pairs that name such a loop, name a loop outside
 * [0, L) or name the same loop twice take no part in the refinement.
 *
 * Passes: every unprocessed piece of loop i whose box overlaps (closed
 * intervals) the box of an unprocessed piece of loop j, for a pair (i, j), is
 * under-refined and is split at t = 1/2 by de Casteljau's construction; every
 * other unprocessed piece becomes final.  Pieces keep the curve's parameter
 * order, so the polyline is the list of the pieces' start points (the final
 * sort of the paper is implicit).  When a split gives a child whose box
 * diagonal is below eps * xi the loop is flagged `intersect_flag` (the
 * paper's "curves intersect" error) and both children become final; pieces
 * still unprocessed after max_passes get the same flag.
 *
 * Returns the number of output vertices (writing xyz only when it fits
 * `cap`), out_off[L+1] and loop_flags[L] (may be NULL); -1 on allocation
 * failure.
 */
typedef struct {
  double b[4][3];
  int done;
} dz_piece;

typedef struct {
  dz_piece* p;
  int64_t n, cap;
} dz_list;

static int dz_push(dz_list* l, const dz_piece* x) {
  if (l->n == l->cap) {
    int64_t nc = l->cap ? 2 * l->cap : 16;
    dz_piece* q = (dz_piece*)realloc(l->p, sizeof(dz_piece) * (size_t)nc);
    if (!q) return 0;
    l->p = q;
    l->cap = nc;
  }
  l->p[l->n++] = *x;
  return 1;
}

static void dz_box(const dz_piece* x, double* lo, double* hi) {
  for (int q = 0; q < 3; ++q) {
    lo[q] = x->b[0][q];
    hi[q] = x->b[0][q];
    for (int k = 1; k < 4; ++k) {
      if (x->b[k][q] < lo[q]) lo[q] = x->b[k][q];
      if (x->b[k][q] > hi[q]) hi[q] = x->b[k][q];
    }
  }
}

/* squared diagonal of the box */
static double dz_diag2(const dz_piece* x) {
  double lo[3], hi[3];
  dz_box(x, lo, hi);
  const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
  return dx * dx + dy * dy + dz * dz;
}

static int dz_overlap(const dz_piece* a, const dz_piece* b) {
  double la[3], ha[3], lb[3], hb[3];
  dz_box(a, la, ha);
  dz_box(b, lb, hb);
  for (int q = 0; q < 3; ++q)
    if (!(la[q] <= hb[q] && lb[q] <= ha[q])) return 0;
  return 1;
}

/* halves of the parameter domain */
static void dz_split(const dz_piece* x, int linear, dz_piece* l, dz_piece* r) {
  for (int q = 0; q < 3; ++q) {
    if (linear) {
      const double m = 0.5 * (x->b[0][q] + x->b[3][q]);
      l->b[0][q] = l->b[1][q] = x->b[0][q];
      l->b[2][q] = l->b[3][q] = m;
      r->b[0][q] = r->b[1][q] = m;
      r->b[2][q] = r->b[3][q] = x->b[3][q];
      continue;
    }
    const double m01 = 0.5 * (x->b[0][q] + x->b[1][q]);
    const double m12 = 0.5 * (x->b[1][q] + x->b[2][q]);
    const double m23 = 0.5 * (x->b[2][q] + x->b[3][q]);
    const double m012 = 0.5 * (m01 + m12);
    const double m123 = 0.5 * (m12 + m23);
    const double m = (g_mutation == 10) ? 0.5 * (m01 + m23) : 0.5 * (m012 + m123);
    l->b[0][q] = x->b[0][q];
    l->b[1][q] = m01;
    l->b[2][q] = m012;
    l->b[3][q] = m;
    r->b[0][q] = m;
    r->b[1][q] = m123;
    r->b[2][q] = m23;
    r->b[3][q] = x->b[3][q];
  }
  l->done = r->done = 0;
}

int64_t lko_discretize(const double* ctrl, const int64_t* cp_off, int32_t L, int kind,
                       const int32_t* pairs, int64_t P, double eps, int max_passes,
                       uint32_t intersect_flag, double* out_xyz, int64_t* out_off, int64_t cap,
                       uint32_t* loop_flags) {
  const int linear = kind == 1;
  dz_list* lists = (dz_list*)calloc((size_t)(L > 0 ? L : 1), sizeof(dz_list));
  uint32_t* flags = (uint32_t*)calloc((size_t)(L > 0 ? L : 1), sizeof(uint32_t));
  if (!lists || !flags) {
    free(lists);
    free(flags);
    return -1;
  }
  /* xi: mean of (|x| + |y| + |z|) / 3 over every input point */
  const int64_t ncp = cp_off[L] - cp_off[0];
  double xs = 0.0;
  for (int64_t v = cp_off[0]; v < cp_off[L]; ++v)
    xs += fabs(ctrl[3 * v]) + fabs(ctrl[3 * v + 1]) + fabs(ctrl[3 * v + 2]);
  const double xi = ncp > 0 ? xs / (3.0 * (double)ncp) : 0.0;
  const double lim = eps * xi;
  const double lim2 = lim * lim;
  int ok = 1;
  for (int32_t i = 0; i < L && ok; ++i) {
    const int64_t o = cp_off[i], m = cp_off[i + 1] - o;
    if (m < 3) flags[i] |= 16u;
    for (int64_t v = 0; v < 3 * m; ++v)
      if (!isfinite(ctrl[3 * o + v])) flags[i] |= 16u;
    for (int64_t s = 0; s < m; ++s) {
      dz_piece x;
      const double* q1 = ctrl + 3 * (o + s);
      const double* q2 = ctrl + 3 * (o + (s + 1) % m);
      if (linear) {
        for (int q = 0; q < 3; ++q) {
          x.b[0][q] = x.b[1][q] = q1[q];
          x.b[2][q] = x.b[3][q] = q2[q];
        }
      } else {
        const double* q0 = ctrl + 3 * (o + (s + m - 1) % m);
        const double* q3 = ctrl + 3 * (o + (s + 2) % m);
        for (int q = 0; q < 3; ++q) {
          x.b[0][q] = (g_mutation == 11) ? q1[q] : (q0[q] + 4.0 * q1[q] + q2[q]) / 6.0;
          x.b[1][q] = (2.0 * q1[q] + q2[q]) / 3.0;
          x.b[2][q] = (q1[q] + 2.0 * q2[q]) / 3.0;
          x.b[3][q] = (q1[q] + 4.0 * q2[q] + q3[q]) / 6.0;
        }
      }
      x.done = 0;
      if (dz_diag2(&x) < lim2) flags[i] |= 16u;
      ok &= dz_push(&lists[i], &x);
    }
  }
  /* passes */
  for (int pass = 0; pass < max_passes && ok; ++pass) {
    int64_t unproc = 0;
    for (int32_t i = 0; i < L; ++i)
      for (int64_t k = 0; k < lists[i].n; ++k) unproc += !lists[i].p[k].done;
    if (unproc == 0) break;
    char** mark = (char**)calloc((size_t)L, sizeof(char*));
    if (!mark) {
      ok = 0;
      break;
    }
    for (int32_t i = 0; i < L; ++i) {
      mark[i] = (char*)calloc((size_t)(lists[i].n + 1), 1);
      if (!mark[i]) ok = 0;
    }
    for (int64_t p = 0; p < P && ok; ++p) {
      const int32_t i = pairs[2 * p], j = pairs[2 * p + 1];
      if (i < 0 || j < 0 || i >= L || j >= L || i == j) continue;
      if ((flags[i] | flags[j]) & 16u) continue;
      for (int64_t a = 0; a < lists[i].n; ++a) {
        if (lists[i].p[a].done) continue;
        for (int64_t b = 0; b < lists[j].n; ++b) {
          if (lists[j].p[b].done) continue;
          if (dz_overlap(&lists[i].p[a], &lists[j].p[b])) {
            mark[i][a] = 1;
            if (g_mutation != 9) mark[j][b] = 1; /* mutation 9: one side only */
          }
        }
      }
    }
    for (int32_t i = 0; i < L && ok; ++i) {
      dz_list nl = {0, 0, 0};
      for (int64_t k = 0; k < lists[i].n; ++k) {
        dz_piece x = lists[i].p[k];
        if (!x.done && !mark[i][k]) x.done = 1;
        if (x.done) {
          ok &= dz_push(&nl, &x);
          continue;
        }
        dz_piece l, r;
        dz_split(&x, linear, &l, &r);
        if (dz_diag2(&l) < lim2 || dz_diag2(&r) < lim2) {
          flags[i] |= intersect_flag;
          l.done = r.done = 1;
        }
        if (g_mutation == 12) { /* mutation 12: children out of order */
          ok &= dz_push(&nl, &r);
          ok &= dz_push(&nl, &l);
        } else {
          ok &= dz_push(&nl, &l);
          ok &= dz_push(&nl, &r);
        }
      }
      free(lists[i].p);
      lists[i] = nl;
    }
    for (int32_t i = 0; i < L; ++i) free(mark[i]);
    free(mark);
  }
  int64_t total = -1;
  if (ok) {
    total = 0;
    for (int32_t i = 0; i < L; ++i) {
      out_off[i] = total;
      for (int64_t k = 0; k < lists[i].n; ++k) {
        if (!lists[i].p[k].done) flags[i] |= intersect_flag;
        if (total < cap && out_xyz)
          for (int q = 0; q < 3; ++q) out_xyz[3 * total + q] = lists[i].p[k].b[0][q];
        ++total;
      }
    }
    out_off[L] = total;
    if (loop_flags) memcpy(loop_flags, flags, sizeof(uint32_t) * (size_t)L);
  }
  for (int32_t i = 0; i < L; ++i) free(lists[i].p);
  free(lists);
  free(flags);
  return total;
}
