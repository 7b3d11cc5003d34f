/*
 * lk.h -- C ABI of the MI355X direct-summation linking-number library (liblk.so).
 *
 * The library evaluates, for every candidate pair of closed polylines, the
 * exact polyline form of the Gauss linking integral: the sum over all
 * segment pairs of the signed-solid-angle term of Eq. 4 (Sec. 2.1, "Direct
 * Summation Methods"; the double sum of Eq. 3 / Alg. 5, Sec. 3.4.2), reduces it
 * to one real number per loop pair and rounds it to the integer linking
 * number.  Around that hot path it offers the potential link search of
 * Alg. 2 (Sec. 3.2), the discretization of spline curves into polylines with
 * the same linking numbers (Alg. 3, Sec. 3.3), the count-crossings and
 * Barnes-Hut methods as other modes of the same call (Alg. 4 and 6,
 * Sec. 2.1 and 3.4.4), the before/after comparison with early exit that the
 * method overview (Sec. 3.1, "Fast Verification") describes, and a
 * verification server for streams of such checks.
 *
 * Conventions shared by every call
 *   - Geometry: xyz is a contiguous row-major array of V vertices x 3
 *     coordinates (float32 or float64, see lk_dtype).  Loop l owns vertices
 *     loop_offsets[l] .. loop_offsets[l+1]-1 (int64, n_loops+1 entries,
 *     non-decreasing; calls that size buffers from the offsets -- the
 *     CROSSINGS and BARNES_HUT modes and lk_discretize -- check this and
 *     return LK_EINVAL, the direct sum treats a loop of negative size as an
 *     invalid loop).  A loop of n vertices is closed: segment s joins vertex
 *     s to vertex (s+1) mod n; the first vertex is not repeated.
 *   - Pairs: int32 [n][2] row-major loop indices.  For pair (i, j) loop i plays
 *     gamma_1 of Eq. 4 (vertices l, index j) and loop j plays gamma_2
 *     (vertices k, index i).  The linking number is symmetric, so the order
 *     only fixes which loop is tiled.
 *   - Memory: every array argument is a DEVICE pointer on the context's device
 *     unless marked (host).  The caller owns all of them; the library never
 *     frees or keeps them after the call returns.
 *   - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *     stream).  Work is enqueued on it; calls return once the work is enqueued
 *     unless documented to synchronise.  Calls on one context must not overlap
 *     (one context per host thread, or serialise).
 *   - Errors: every call returns lk_status.  A non-OK status leaves outputs
 *     unspecified and sets a message readable with lk_last_error.  Problems of
 *     individual pairs (bad indices, degenerate loops, non-finite sums) are
 *     never host errors: they are reported per pair in the flags output.
 */
#ifndef LK_H_
#define LK_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lk_ctx lk_ctx;

typedef enum {
  LK_OK = 0,
  LK_EINVAL = -1,    /* bad argument (null pointer, negative size, unknown enum) */
  LK_ENOMEM = -2,    /* device or host allocation failed */
  LK_EDEVICE = -3,   /* a HIP runtime call failed */
  LK_ECAPACITY = -4, /* output buffer too small; the required size is returned */
  LK_EBUSY = -5,     /* resource in use (server slot table full, stream capturing) */
  LK_ENOTFOUND = -6  /* unknown request or handle */
} lk_status;

typedef enum { LK_F32 = 0, LK_F64 = 1 } lk_dtype;

/* PLAIN_F64: every term, sum and reduction in FP64 (FP32 input is promoted
 * exactly).  MIXED: terms in FP32, per-thread sums in FP32 over at most one
 * LDS tile, everything from the per-tile partial upwards in FP64, and every
 * pair whose |value - round(value)| exceeds the refit threshold (default 0.05)
 * recomputed entirely in FP64 from the caller's input.
 * CROSSINGS: Count Crossings (Sec. 2.1, Alg. 4) in place of the FP32 direct
 * sum: the value is half the signed number of crossings of the projection
 * along the context's view direction (lk_set_view_direction).  Every side
 * test and crossing sign is decided in FP32 only when its magnitude exceeds a
 * forward error bound, on the vertices as given (FP64 input is rounded to
 * FP32 for this pass), so for FP32 input a certified count is exact.  A pair
 * with an undecided test (a crossing at or near a vertex, near-parallel or
 * nearly touching segments) or an odd count is counted again in FP64 (the
 * same predicates with bounds at the FP64 unit roundoff), and a pair still
 * undecided there goes to the FP64 direct sum; both set LK_FLAG_REFIT.
 * lk_real is the count / 2 for every counted pair.  As Alg. 4 bounds its search with a BVH, the count skips
 * blocks of 64 consecutive vertices (and of 4096) whose projected boxes are
 * disjoint from the other loop's block (LK_OPT_CROSSING_CULL).  To size those
 * boxes the first CROSSINGS call with a given offsets array reads its
 * vertex count from the device, which synchronises the stream once.  The
 * count is kept per (offsets pointer, loop count): if later offsets at the
 * same address describe more vertices (a reused allocation), results stay
 * exact, but culling covers only the slots counted first and the pairs
 * beyond them are counted without it. */
/* BARNES_HUT: the two-tree Barnes-Hut method (Sec. 3.4.4, Alg. 6), an
 * approximation with the direct sum's Eq. 4 at the leaves: trees over runs of
 * 64 consecutive segments (8 children per node), node pairs farther apart
 * than beta times the sum of their box radii use the far-field expansion to
 * the given order (LK_OPT_BH_BETA_MILLI, LK_OPT_BH_ORDER; default beta 4,
 * quadrupole order) in FP64, leaf pairs the FP32 term with FP64 sums.  Pairs
 * whose value is farther than the refit threshold from an integer are
 * recomputed by the FP64 direct sum, as in MIXED.  Like CROSSINGS, the first
 * call for an offsets array reads its vertex count (one synchronisation);
 * trees that a reused allocation with more vertices would outgrow are not
 * built, and those pairs go to the FP64 direct sum. */
typedef enum { LK_PLAIN_F64 = 0, LK_MIXED = 1, LK_CROSSINGS = 2, LK_BARNES_HUT = 3 } lk_mode;

/* Per-pair flags (bit set). */
enum {
  LK_FLAG_REFIT = 1u,     /* value came from the FP64 refit (MIXED only) */
  LK_FLAG_AMBIGUOUS = 2u, /* |value - round(value)| > threshold in FP64 too */
  LK_FLAG_NONFINITE = 4u, /* NaN/Inf in the sum (degenerate or intersecting input) */
  LK_FLAG_BADPAIR = 8u,   /* i == j or an index outside [0, n_loops) */
  LK_FLAG_BADLOOP = 16u,  /* a loop has < 3 vertices, a non-finite coordinate, or a
                             segment shorter than eps * xi (Alg. 3 zero-length test,
                             xi = mean |coordinate| over the call's vertices,
                             eps = machine epsilon of the input dtype) */
  LK_FLAG_SKIPPED = 32u,  /* lk_direct_sum_check with early exit stopped before this
                             pair's sum was complete (no value, LK_INT_INVALID) */
  LK_FLAG_INTERSECT = 64u /* lk_discretize (a loop flag): refinement of this loop reached
                             a piece shorter than eps * xi, or the pass limit, so the
                             curve comes within about that distance of a paired loop */
};

/* Integer reported for pairs whose value is not finite or whose indices are bad. */
#define LK_INT_INVALID INT32_MIN

/* ---------------------------------------------------------------- context */
/* Create a context on HIP device `device` (owns workspace, the kernel
 * configuration table and the captured-graph cache).  *out receives the
 * handle.  Returns LK_EDEVICE if the device cannot be used. */
lk_status lk_create(lk_ctx** out, int device);

/* Destroy a context (synchronises its device first).  NULL is ignored. */
void lk_destroy(lk_ctx* ctx);

/* Message for the last non-OK status returned on this context ("" if none).
 * The pointer stays valid until the next call on the context. */
const char* lk_last_error(const lk_ctx* ctx);

/* ---------------------------------------------------- potential link search */
/* Alg. 2 (Sec. 3.2): every loop pair i < j whose closed axis-aligned boxes
 * (vertex min/max per loop) overlap on all three axes, in lexicographic order,
 * written to pairs_out [capacity][2].  Synchronises the stream (the count is
 * needed on the host).  *n_pairs (host) receives the number of pairs; if it
 * exceeds `capacity`, nothing is written and LK_ECAPACITY is returned with
 * *n_pairs = required size.  Loops with no vertex get no pair.  The search
 * stands in for the paper's box tree: from 2,048 loops on (LK_OPT_PAIR_SEARCH)
 * the boxes are binned on a hashed grid by their min corners, and each box is
 * tested only against the boxes of its 27 neighbouring cells (large or
 * non-finite boxes against all); below that, all L (L - 1) / 2 box pairs are
 * tested.  Both give exactly the same pairs. */
lk_status lk_build_pairs(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* loop_offsets,
                         int32_t n_loops, int32_t* pairs_out, int64_t capacity,
                         int64_t* n_pairs /* host */, void* stream);

/* ------------------------------------------------------------ direct sum */
/* For each pair p = (i, j):
 *   lk_real[p] = sum over segments j' of loop i and i' of loop j of the Eq. 4
 *                term (FP64 result),
 *   lk_int[p]  = round-half-away-from-zero(lk_real[p]), or LK_INT_INVALID,
 *   flags[p]   = LK_FLAG_* bits.
 * lk_real/lk_int/flags are [n_pairs] device arrays; flags may be NULL.
 * Asynchronous.  The sequence of kernels is captured once per argument set
 * into a HIP graph and replayed on later identical calls (see LK_OPT_GRAPH).
 * Results are bitwise reproducible for identical inputs and configuration,
 * independent of what else runs on the device. */
lk_status lk_direct_sum(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* loop_offsets,
                        int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                        double* lk_real, int32_t* lk_int, uint32_t* flags, void* stream);

/* Direct sum fused with the certificate check (Sec. 3.1, "Fast
 * Verification", and its early-exit strategy): as lk_direct_sum, and each
 * pair's final integer is compared with expected[p] (int32 [n_pairs], device)
 * as soon as it is known.  A pair is a mismatch when its integer differs or
 * when it cannot be certified (LK_FLAG_NONFINITE, AMBIGUOUS, BADPAIR or
 * BADLOOP).  *n_mismatch (int64, device) receives the count; nothing is
 * copied to the host, so the call is asynchronous and graph-capturable.
 * early_exit != 0: once a mismatch is found, the kernels stop taking new
 * work.  Pairs whose sum was not completed then carry LK_FLAG_SKIPPED,
 * LK_INT_INVALID and a NaN real, and the count covers the pairs compared
 * before the stop (at least 1).  For the simulation use of Sec. 3.1, pass the
 * union of the current candidate pairs and the expected non-zero pairs, with
 * expected 0 for pairs that are new. */
lk_status lk_direct_sum_check(lk_ctx* ctx, const void* xyz, int dtype,
                              const int64_t* loop_offsets, int32_t n_loops, const int32_t* pairs,
                              int64_t n_pairs, const int32_t* expected, int early_exit, int mode,
                              double* lk_real, int32_t* lk_int, uint32_t* flags,
                              int64_t* n_mismatch /* device */, void* stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * computation and kernels as lk_direct_sum in the PLAIN_F64 and MIXED modes
 * (bitwise equal results for the same context options), with the call's
 * workspace in one static device array of the library (about 17.6 MiB, held
 * by each device the library runs on until the process ends) instead of the
 * context's buffers.  The call allocates nothing: no hipMalloc, hipFree or
 * graph instantiation; the kernels are launched eagerly on `stream` (which a
 * caller may be capturing).  The device's address of the array is looked up
 * once per device when a context is created on it.
 *   - Limits: n_loops <= 65536 and n_pairs <= 131072; larger calls return
 *     LK_ECAPACITY and enqueue nothing.  Other modes return LK_EINVAL.
 *   - flags may be NULL (the flags then live in the static array).
 *   - Every call on one device shares that device's array, which keeps the
 *     last call's contents (each call initialises what it reads): calls that
 *     overlap on one device -- on different streams, from any context or
 *     thread -- race and give undefined results.  Serialise them (one stream,
 *     or events).
 *   - lk_get_stats afterwards reports the configuration used but no refit
 *     count.
 * Arguments, layout, ownership and errors are otherwise those of
 * lk_direct_sum. */
lk_status lk_direct_sum_noalloc(lk_ctx* ctx, const void* xyz, int dtype,
                                const int64_t* loop_offsets, int32_t n_loops,
                                const int32_t* pairs, int64_t n_pairs, int mode, double* lk_real,
                                int32_t* lk_int, uint32_t* flags, void* stream);

/* --------------------------------------------------------------- verify */
/* Compare the current sparse linking matrix (pairs, lk)[n] with the expected
 * one (exp_pairs, exp_lk)[n_exp]; both pair lists sorted lexicographically
 * with i < j and no duplicates (Sec. 3.1, "Fast Verification").  A pair only
 * in the current list is expected to be 0; a pair only in the expected list
 * counts as 0 now (its boxes separated), so it is a mismatch when its
 * expected value is non-zero.  Synchronises.  *n_mismatch (host) receives the
 * number of mismatches; the first min(count, cap) of them in pair order are
 * written to mismatches [cap][4] as (i, j, got, expected).  With
 * early_exit != 0 the call stops at the first mismatch in pair order:
 * *n_mismatch is 0 or 1 and at most that record is written. */
lk_status lk_verify(lk_ctx* ctx, const int32_t* pairs, const int32_t* lk, int64_t n,
                    const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp, int early_exit,
                    int64_t* n_mismatch /* host */, int32_t* mismatches, int64_t cap, void* stream);

/* --------------------------------------------------------- discretization */
/* Curve kinds of lk_discretize. */
typedef enum {
  LK_DZ_BSPLINE = 0, /* closed uniform cubic B-spline: loop l's points are its m control
                        points and it has m spans; span s is the cubic of control points
                        s-1, s, s+1, s+2 (cyclic) */
  LK_DZ_POLYLINE = 1 /* closed polyline: m vertices, m segments */
} lk_curve_kind;

typedef struct {
  int32_t passes;      /* refinement passes run */
  int32_t reserved;
  int64_t input_spans; /* spans (B-spline) or segments (polyline) of the input */
  int64_t vertices;    /* output vertices (= output segments) */
  int64_t splits;      /* pieces split over all passes */
  int64_t unfinished;  /* pieces still unprocessed when the pass limit stopped the
                          refinement (their loops are flagged LK_FLAG_INTERSECT) */
} lk_dz_info;

/* Discretization (Sec. 3.3, Alg. 3): closed curves -> closed polylines with
 * the same linking numbers.  Every span is a cubic Bezier piece (a polyline
 * segment is a linear one) bounded by the box of its control points, which
 * contains the curve.  Each pass splits every unprocessed piece whose box
 * overlaps (closed intervals) the box of an unprocessed piece of a loop it is
 * paired with, at the middle of its parameter domain (de Casteljau; the
 * midpoint of a segment); every other unprocessed piece becomes final.  When
 * nothing is unprocessed, loop l's polyline is its pieces' start points in
 * parameter order.  By the argument of App. A, every loop can then be
 * deformed into its polyline inside boxes that no other paired loop enters.
 *   ctrl [N][3] FP64 and ctrl_offsets [n_loops+1] (int64, non-decreasing) give
 *     the points of each loop as in the geometry convention above; kind is an
 *     lk_curve_kind; pairs [n_pairs][2] are the candidate loop pairs (e.g. from
 *     lk_build_pairs on the control points, whose boxes contain the curves).
 *   xyz_out [capacity][3] FP64 receives the vertices, offsets_out [n_loops+1]
 *     (int64, from 0) the loops' ranges, loop_flags [n_loops] (may be NULL)
 *     LK_FLAG_BADLOOP (fewer than 3 points, a non-finite coordinate, or a
 *     span whose box diagonal is below eps * xi, eps = 2^-52; such a loop's
 *     pairs take no part and it is not refined) and LK_FLAG_INTERSECT.
 *   *n_vertices (host) receives the output vertex count; *info (host, may be
 *     NULL) the pass statistics.
 * All arrays but n_vertices and info are device arrays.  Synchronises the
 * stream after every pass (the next pass is sized from the counts), so it
 * cannot be captured (LK_EBUSY on a capturing stream).  If the vertices do not
 * fit `capacity`, offsets_out and loop_flags are still written, xyz_out is
 * not, and LK_ECAPACITY is returned.  The result is bitwise reproducible and
 * does not depend on the order of the pairs. */
lk_status lk_discretize(lk_ctx* ctx, const double* ctrl, const int64_t* ctrl_offsets,
                        int32_t n_loops, int kind, const int32_t* pairs, int64_t n_pairs,
                        double* xyz_out, int64_t capacity, int64_t* offsets_out,
                        uint32_t* loop_flags, int64_t* n_vertices /* host */,
                        lk_dz_info* info /* host */, void* stream);


/* ------------------------------------------------------ options and stats */
enum {
  LK_OPT_REFIT_THRESHOLD_PPM = 1, /* refit threshold in millionths (default 50000 = 0.05) */
  LK_OPT_GRAPH = 2,               /* 1 = capture/replay HIP graphs (default), 0 = eager */
  LK_OPT_TIMING = 3,              /* n > 0: time the kernels of the next calls with HIP events
                                     (eager launches, a ring of n calls); 0 = off.  Setting it
                                     synchronises the device and clears the ring. */
  LK_OPT_TILE_A = 4,              /* FP32 LDS tile of loop A in vertices (0 = tuned) */
  LK_OPT_CHUNK_A = 5,             /* vertices of A per work item (0 = tuned) */
  LK_OPT_WAVES_PER_CU = 6,        /* persistent waves per compute unit (0 = occupancy) */
  LK_OPT_ATAN = 7,                /* FP32 arctangent: 0 = own minimax, the R terms of a step
                                     in phases; 1 = HIP atan2f; 2 = own minimax, term by
                                     term (same values as 0, another instruction order) */
  LK_OPT_SEGS_PER_LANE = 8,       /* FP32 kernel: segments of loop B per lane, 1/2/4, and 8 for
                                     CROSSINGS (0 = tuned; the direct sum uses 4 for 8) */
  LK_OPT_SEGS_PER_LANE_F64 = 9,   /* FP64 kernel: segments of loop B per lane, 1/2 (0 = tuned) */
  LK_OPT_SMALL_BATCH = 10,        /* small pairs claimed per work-counter step, 1..64 (0 = tuned);
                                     the FP32 passes use at least the segments per lane */
  LK_OPT_CROSSING_TOL = 11,       /* CROSSINGS: multiplier of the certainty bounds, 1..2^20
                                     (default 1); larger values send more pairs to the FP64
                                     direct sum, never fewer */
  LK_OPT_CROSSING_CULL = 12,      /* CROSSINGS: 1 = skip vertex blocks and pairs whose projected
                                     boxes are disjoint (default), 0 = test every segment pair;
                                     the results are the same */
  LK_OPT_BH_BETA_MILLI = 13,      /* BARNES_HUT: far-field ratio beta x 1000, 500..1e6
                                     (default 4000) */
  LK_OPT_BH_ORDER = 14,           /* BARNES_HUT: 1 = monopole and dipole terms, 2 = also the
                                     quadrupole term (default) */
  LK_OPT_DZ_MAX_PASSES = 15,      /* lk_discretize: most refinement passes, 1..1000 (default 64;
                                     pieces left unprocessed flag their loop INTERSECT) */
  LK_OPT_BH_ADAPTIVE = 16,        /* BARNES_HUT: 1 = adaptive beta (Sec. 3.4.4): the first
                                     traversal at beta (LK_OPT_BH_BETA_MILLI, as beta_init) sums
                                     each pair's next-order error estimate E (constant
                                     k = 1/(4 pi)); a pair with beta_t = (E / E_target)^(1/4) beta
                                     above beta is evaluated again at min(beta_t, beta_max).
                                     0 = one traversal at beta (default) */
  LK_OPT_BH_BETA_MAX_MILLI = 17,  /* BARNES_HUT adaptive: beta_max x 1000, 500..1e6 (default
                                     10000) */
  LK_OPT_BH_TARGET_PPM = 18,      /* BARNES_HUT adaptive: E_target in millionths, 1..1e6
                                     (default 200000 = 0.2) */
  LK_OPT_PAIR_SEARCH = 19         /* lk_build_pairs: 0 = grid from 2,048 loops on (default),
                                     1 = test all box pairs, 2 = grid always */
};

/* Set an option; returns LK_EINVAL for an unknown key or a bad value. */
lk_status lk_set_option(lk_ctx* ctx, int key, int64_t value);

/* View direction of the CROSSINGS mode (Sec. 2.1: the projection must be
 * regular, and a random frame makes that almost certain, Alg. 4).  dir is a
 * host array of 3 finite values, not all zero; it is scaled so that its
 * largest magnitude is 1 and rounded to FP32.  The sign of each crossing does
 * not depend on which way along the line one looks.  Default: a fixed generic
 * direction.  lk_get_view_direction returns the direction in use (host). */
lk_status lk_set_view_direction(lk_ctx* ctx, const double* dir);
lk_status lk_get_view_direction(const lk_ctx* ctx, double* dir);

typedef struct {
  int64_t refits;         /* pairs recomputed in FP64 by the last MIXED or CROSSINGS call */
  double kernel_ms;       /* mean main-kernel time over the timed calls in the ring */
  double refit_kernel_ms; /* mean refit-kernel time over the same calls (MIXED) */
  int32_t timed_calls;    /* number of calls those means cover */
  int32_t graph_replayed; /* 1 if the last call replayed a captured graph */
  int32_t tile_a, chunk_a, waves_per_cu, atan_form, segs_per_lane; /* configuration used
                            (atan_form 3: the crossing count) */
  int64_t refits_direct_sum; /* CROSSINGS: pairs the FP64 crossing count could not decide
                                either, computed by the FP64 direct sum */
  int64_t bh_list_peak;      /* BARNES_HUT: most node pairs in one traversal step */
  int64_t bh_near_pairs;     /* BARNES_HUT: leaf pairs summed directly */
  int64_t bh_list_cap;       /* BARNES_HUT: capacity of a step's list (pairs beyond it are
                                refitted) */
  int64_t bh_reruns;         /* BARNES_HUT with adaptive beta: pairs evaluated again at a
                                larger beta */
} lk_stats;

/* ------------------------------------------------------------ autotuner */
typedef struct {
  int32_t segs_per_lane;     /* FP32 kernel: segments of loop B per lane */
  int32_t segs_per_lane_f64; /* FP64 kernel: segments of loop B per lane */
  int32_t tile_a;            /* LDS tile of loop A (vertices) */
  int32_t chunk_a;           /* vertices of loop A per work item */
  int32_t small_batch;       /* small pairs per work-counter step */
  int32_t waves_per_cu;      /* persistent waves per CU (0 = occupancy limit) */
  int32_t evaluated;         /* configurations timed (0 when read from the cache) */
  int32_t from_cache;        /* 1 if the configuration came from the cache file */
  double best_ms;            /* main-kernel time of the chosen configuration */
  double start_ms;           /* main-kernel time of the configuration tuning started from */
  int32_t atan_form;         /* FP32 arctangent form (LK_OPT_ATAN) */
  int32_t reserved;
} lk_tuning;

/* Choose the kernel configuration (work split and tile shapes) for a
 * workload: times the main direct-sum kernel of this exact call (eager, HIP
 * events, on `stream`) over a coordinate-descent search of segments per lane,
 * arctangent form, small-pair batch, LDS tile, A chunk and waves per CU, applies the fastest to
 * the context (as if set with lk_set_option) and returns it in *out (host).
 * cache_path (host string, may be NULL): a text file of earlier results keyed
 * by GPU architecture, mode, dtype and the workload's size profile; a hit is
 * applied without timing, a new result is appended.  Synchronises; the
 * output arrays of the call are used as scratch (their contents afterwards
 * are those of a valid lk_direct_sum). */
lk_status lk_autotune(lk_ctx* ctx, const void* xyz, int dtype, const int64_t* loop_offsets,
                      int32_t n_loops, const int32_t* pairs, int64_t n_pairs, int mode,
                      double* lk_real, int32_t* lk_int, uint32_t* flags, const char* cache_path,
                      lk_tuning* out /* host */, void* stream);

/* Reserve workspace for calls of up to max_loops loops, max_pairs pairs and
 * max_verify verify entries (n + n_exp), so that later calls within those
 * sizes never allocate device memory or synchronise the device for growth. */
lk_status lk_reserve(lk_ctx* ctx, int32_t max_loops, int64_t max_pairs, int64_t max_verify);

/* -------------------------------------------------------------- serving */
/* A verification server for streams of timesteps (the per-frame use of
 * Sec. 3.1's certificate comparison: compute the linking matrix of a new
 * state and compare it with the stored one).  Requests are queued, admitted
 * in arrival order when a slot is free and the device-memory budget allows,
 * and run concurrently on the slots (one context, HIP stream and host thread
 * each), so work of requests that arrive while others run overlaps on the
 * device.  Each request runs lk_build_pairs, lk_direct_sum and lk_verify
 * against its session's expected matrix.  A request's results do not depend
 * on what else runs (fixed configuration, fixed-point pair sums). */
typedef struct lk_server lk_server;

enum { LK_MEM_HOST = 0, LK_MEM_DEVICE = 1 };

typedef struct {
  int64_t id;          /* request id */
  int32_t status;      /* lk_status of the request's calls */
  int32_t slot;        /* slot that ran it */
  int64_t n_pairs;     /* candidate pairs found */
  int64_t n_mismatch;  /* pairs whose integer differs from the session's expectation */
  int64_t n_flagged;   /* pairs with NONFINITE, BADPAIR, BADLOOP or AMBIGUOUS set */
  int64_t refits;      /* pairs recomputed in FP64 */
  double terms;        /* segment-pair terms evaluated */
  int64_t bytes;       /* device bytes of its own buffers charged while it ran */
  double t_submit;     /* seconds (server clock) when submitted */
  double t_admit;      /* ... when admitted to a slot */
  double t_done;       /* ... when its results were on the host */
} lk_result;

/* Create a server on `device` with `slots` concurrent slots (1..8), a device
 * memory budget in bytes (0 = 80% of free memory), the direct-sum mode of
 * every request, and per-slot workspace reserved for up to max_loops loops
 * and max_pairs candidate pairs per request.  The budget covers sessions,
 * each running request's buffers (charged for a first guess of its pair
 * count, corrected once the pairs are counted; a request whose charge grows
 * waits for memory unless nothing else could free it) and the growth of a
 * slot's workspace beyond the reservation made here (the Barnes-Hut trees and
 * lists, about 150 bytes per vertex, and the crossing-count boxes are sized
 * per request).  A request is admitted over the budget only when nothing else
 * runs. */
lk_status lk_server_create(lk_server** out, int device, int32_t slots, int64_t mem_budget,
                           int mode, int32_t max_loops, int64_t max_pairs);
/* Stop accepting, finish queued and running requests, free everything. */
void lk_server_destroy(lk_server* srv);
const char* lk_server_last_error(const lk_server* srv);

/* A session: the loop structure (offsets, host) and the expected sparse
 * linking matrix (sorted pairs and values, host) of one simulated object stay
 * resident on the device for all its timesteps.  Its bytes count against the
 * budget until it is closed. */
lk_status lk_server_open_session(lk_server* srv, const int64_t* loop_offsets, int32_t n_loops,
                                 const int32_t* exp_pairs, const int32_t* exp_lk, int64_t n_exp,
                                 int64_t* session /* host */);
lk_status lk_server_close_session(lk_server* srv, int64_t session);

/* Queue one timestep of a session: xyz [V][3] (V = the session's vertex
 * count) of `dtype`, in host memory (copied to the device when the request
 * runs) or device memory (used in place).  The caller keeps xyz valid until
 * the request is done.  Returns immediately with the request id; LK_ECAPACITY
 * if the request can never fit the budget. */
lk_status lk_server_submit(lk_server* srv, int64_t session, const void* xyz, int dtype,
                           int where, int64_t* request_id /* host */);

/* Wait up to timeout_ms (< 0: forever) for a request; LK_EBUSY on timeout.
 * Fills *res; optionally copies up to `cap` of its pairs, integers, reals and
 * (up to cap) mismatch records (i, j, got, expected) into host buffers (any
 * may be NULL).  A request's results can be fetched once. */
lk_status lk_server_wait(lk_server* srv, int64_t request_id, int32_t timeout_ms, lk_result* res,
                         int32_t* pairs_out, int32_t* lk_out, double* real_out,
                         int32_t* mismatches_out, int64_t cap);

/* Statistics of the last lk_direct_sum on this context.  Reading refits and
 * the timings synchronises the stream of that call; the timed calls must all
 * have been issued on that stream. */
lk_status lk_get_stats(lk_ctx* ctx, lk_stats* out /* host */);

#ifdef __cplusplus
}
#endif
#endif /* LK_H_ */
