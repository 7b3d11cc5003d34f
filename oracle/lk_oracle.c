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
 * the tests that prove the pins catch them; it is 0 (off) by default.
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
