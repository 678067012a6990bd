/*
 * hd.h -- certified one-sided Pompeiu-Hausdorff bounds between triangle soups
 * on AMD Instinct MI355X (gfx950).
 *
 * The library computes an interval [L, U] with L <= h(A,B) <= U and
 * U - L <= eps, where h(A,B) = max over p in A of the distance from p to B.
 * The paper states the tolerance relative to dA, the length of the diagonal
 * of the bounding box of A's (referenced) vertices: eps = epsilon * dA. This
 * is the problem statement and output contract
 * of Sacht & Jacobson, "Cascading upper bounds for triangle soup
 * Pompeiu-Hausdorff distance" (Method section: eq. hausdorff_distance and
 * eq. output_bounds). The method is that paper's branch and bound with its
 * exact same-triangle bound and four cascading upper bounds, run as
 * breadth-first rounds of data-parallel HIP kernels.
 *
 * Conventions for every entry point:
 *  - Mesh arrays are DEVICE pointers owned by the caller: V is m x 3 doubles,
 *    row-major; F is n x 3 int32, 0-based. They must stay valid and unmodified
 *    until the stream passes the call. The library never frees caller memory.
 *  - Vertices that no face references are ignored (Limitations subsection: an
 *    unreferenced vertex would make the lower bound wrong).
 *  - Work is enqueued on the given stream; entry points that return numbers
 *    to the host synchronise that stream before returning.
 *  - Errors are returned as hd_status; no C++ exception crosses the ABI. On
 *    any error LU_out receives {NaN, NaN}.
 */
#ifndef HD_H
#define HD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hd_stream_t;

#define HD_QUERY_SHAPES 9 /* launch shapes of the query kernel (hd_options.query_shape) */ /* hipStream_t; NULL = default stream */

typedef enum {
    HD_OK = 0,
    HD_E_INVALID = 1,  /* bad argument: eps <= 0, empty mesh, index out of range, non-finite coordinate */
    HD_E_CAPACITY = 2, /* face budget m * nA exceeded, or frontier workspace / subdivision depth exhausted */
    HD_E_NOMEM = 3,    /* device allocation failed */
    HD_E_DEVICE = 4,   /* a HIP runtime call failed */
    HD_E_INTERNAL = 5  /* an invariant failed (e.g. the frontier emptied while the tolerance did not hold) */
} hd_status;

/* Arithmetic of the branch-and-bound rounds. The final [L, U] is always
 * evaluated in FP64. */
enum { HD_PREC_FP64 = 0, HD_PREC_FP32 = 1, HD_PREC_FP32_RECHECK = 2 };

typedef struct hd_bvh_s *hd_bvh; /* opaque; owns library-allocated device memory */

typedef struct {
    int32_t precision;   /* HD_PREC_*; default HD_PREC_FP32_RECHECK */
    int32_t order;       /* cascade order as decimal digits, e.g. 1234 (default) or 2314;
                            any non-empty subset of {1,2,3,4,5} without repeats. 5 is the bound
                            of Zheng et al. that the paper quotes in its fourth-bound subsection
                            (min over the vertices' and the barycenter's closest B triangles of
                            the largest vertex distance to it); it costs one point query per
                            triangle that reaches it. A single digit is a single-bound cascade. */
    double budget_m;     /* the paper's m: at most m * nA faces may be processed (Implementation
                            section); <= 0 means 1e7 */
    int64_t capacity;    /* frontier capacity in triangles; 0 = automatic */
    int32_t max_rounds;  /* 0 = unlimited */
    int32_t stack_depth; /* test hook: 1..15 runs the query kernel with a one-entry LDS
                            stack per lane (restarts, then the deep-stack fallback); 0 = default */
    int32_t subbatch;    /* > 0: subdivide about this many triangles per round, highest upper
                            bound first (approximates the paper's best-first queue). The device
                            selects them (a radix select on the key; the last key bin is taken
                            whole, so a round may split a few more); triangles whose bound fell
                            below L are dropped and those within eps of L parked first. */
    int32_t profile;     /* 1: time the query and cascade kernels with HIP events on the
                            call's stream (fills the ms_* kernel fields of hd_stats); 2: the
                            query kernels only (every event record costs the stream a few
                            microseconds) */
    int32_t learned;     /* learned proposal (not in the paper): 0 off; 1 the sub-batch is
                            taken in order of the network's predicted maximum distance
                            instead of the upper bound; 2 also let the network skip u3 and u4
                            for triangles it predicts to stay active. Bounds, discards and
                            the certificate are unchanged in kind. */
    int32_t log_frontier;      /* 1: log every subdivided parent's features and label */
    const float *mlp_params;   /* device, hd_mlp_nparams() FP32 values; needed when learned > 0 */
    float *log_out;            /* device, log_cap rows of 17 FP32: the 16 features (as the
                                  network takes them) and the label (max over the resolution-4
                                  barycentric lattice of d(p, B) - max vertex distance) /
                                  longest edge; rows of parents deeper than level 28 are NaN */
    int64_t log_cap;
    int32_t autotune;          /* 1: on the first call on a device (per arithmetic), time the
                                  query kernel's launch shapes (block size, LDS stack depth) on
                                  this call's vertex queries and keep the fastest for later
                                  calls; 2: retune on this call; 0: use the kept choice */
    int32_t query_lanes;       /* lanes per point query: 0 automatic (a quad of four lanes per
                                  query in query launches of at most 32768 queries, where one
                                  lane per query leaves the GPU latency-bound; above, one query
                                  per lane); 1 always one lane per query; 4 always a quad.
                                  Results do not depend on it. */
    int32_t eps_relative;      /* 0 (default): eps is the absolute tolerance, U - L <= eps;
                                  1: eps is the paper's relative tolerance (eq. output_bounds),
                                  U - L <= eps * dA, dA computed on the device from A */
    int32_t query_shape;       /* 0: the query kernel's kept launch shape (the autotuner's
                                  choice, else the default); k in 1..HD_QUERY_SHAPES: shape k-1
                                  of the kernel's list (block size, LDS stack entries per lane)
                                  for this call only, reported in hd_stats query_block and
                                  query_stack. Results do not depend on it. */
    const char *tuner_cache;   /* autotune != 0: path of a JSON file that keeps the autotuner's
                                  choice per (device, arithmetic, kernel-source hash) across
                                  processes: a kept choice is used without tuning, a new one is
                                  added to the file; NULL: the choice lives in process memory */
    struct hd_round_record *round_log; /* HOST array of round_log_cap records, one per round
                                  (round 0 = the vertex round), or NULL. Logging runs the rounds
                                  host-driven (one report and one extra reduction per round). */
    int64_t round_log_cap;
    double test_bound_shift;   /* test hook, 0 normally: subtracted from every upper bound of the
                                  FP32/FP64 cascade stages. A shift that makes a bound smaller than
                                  the largest vertex distance of its triangle (no valid bound is)
                                  must end the call with HD_E_INTERNAL. */
    int32_t split_levels;      /* 0 (default): a breadth-first round that splits at most 8192
                                  triangles splits each of them two levels deep at once (its 16
                                  grandchildren, every one bounded), and one of at most 64
                                  triangles four levels deep (256 descendants), so that the few
                                  last rounds, bound by kernel latency rather than work, take
                                  fewer launches; 1: every round splits one level (1 -> 4); 2: at
                                  most two levels; k >= 3: rounds of at most k triangles split two
                                  levels (and of at most 64, four). A sub-batched round goes
                                  deeper only when it splits every live record; host-driven
                                  rounds always split one level. Negative: HD_E_INVALID. */
    int32_t pad_opt;
} hd_options;

/* One record of hd_options.round_log: the state after a round. */
typedef struct hd_round_record {
    int32_t round;             /* 0: the vertex round */
    int32_t pad;
    int64_t split;             /* triangles split 1 -> 4 in this round */
    int64_t active, parked;    /* list sizes after the round */
    int64_t bounded;           /* triangles bounded so far */
    int64_t discards[5];       /* triangles discarded so far by uexact, u1, u2, u3, u4 */
    double L;                  /* pair 0: lower bound after the round */
    double U;                  /* pair 0: largest upper bound (margin included) of a live
                                  triangle after the round, or L if none is left */
    double ms;                 /* host time from the start of the call to the round's report */
} hd_round_record;

typedef struct {
    int32_t rounds;            /* rounds after round 0 */
    int32_t status;            /* hd_status of the call */
    int64_t nodes_bounded;     /* frontier triangles whose upper bound was computed */
    int64_t subdivided;        /* triangles split 1 -> 4 */
    int64_t queries;           /* point -> B distance queries */
    int64_t pt_tri_evals;      /* point-triangle closest-point evaluations (traversal leaves
                                  and the third bound's fixed-triangle evaluations) */
    int64_t box_tests;         /* BVH box tests */
    int64_t discards[5];       /* triangles discarded by uexact, u1, u2, u3, u4 */
    int64_t rechecked64;       /* triangles re-bounded in FP64 inside the ambiguity band */
    int64_t parked_final;      /* triangles left within eps of L at the end */
    int64_t max_frontier;      /* peak live frontier size */
    int64_t stack_overflows;   /* traversals that fell back to the deep-stack path */
    double dA, eps_abs;        /* bbox diagonal of A and eps * dA */
    double L_rounds, U_rounds; /* interval reached by the rounds, before the FP64 final step */
    double mu_coef_d, mu_coef_0; /* FP32 margin: mu(d) = mu_coef_d * d + mu_coef_0 */
    double ms_total;           /* wall time of the hd_bound call */
    double ms_query_kernels;   /* profile > 0: summed duration of the point-query kernels */
    double ms_cascade_kernels; /* profile = 1: summed duration of the bound/classify kernels */
    int64_t query_launches, cascade_launches;
    int64_t query_leaf_evals;  /* closest-point evaluations inside the query kernels */
    int64_t query_box_tests;   /* box tests inside the query kernels */
    int64_t logged;            /* log_frontier: rows written to log_out (<= log_cap) */
    int64_t learned_skips;     /* learned = 2: triangles whose u3 and u4 were skipped */
    int32_t query_block;       /* launch shape of this call's query kernel: block size */
    int32_t query_stack;       /* and LDS stack entries per query */
    int32_t query_lanes;       /* the call's query_lanes option */
    int32_t query_quad_max;    /* launches of at most this many queries ran a quad per query
                                  (0: none did; -1: all did) */
    int64_t round_records;     /* records written to hd_options.round_log */
    int32_t tuned;             /* where the query launch shape came from: 0 kept in memory or the
                                  default, 1 tuned by this call, 2 read from tuner_cache */
    int32_t pad1;
    int64_t stale;             /* sub-batches: active triangles dropped before being split because
                                  L had risen above their bound (the paper's stale queue entries) */
    int64_t discards_u5;       /* triangles discarded by the fifth bound (order digit 5) */
    int32_t device_flag;       /* what the device found wrong (0 nothing): 2 a traversal deeper than the
                                  fallback stack, 3 the subdivision depth limit, 4 an upper bound below a
                                  vertex distance of its triangle, 5 plain FP32 with a tolerance below
                                  its margin */
    int32_t pad2;
} hd_stats;

/* Build the LBVH over soup B (device-built: Morton codes of triangle
 * centroids, radix sort, Karras hierarchy, outward-rounded refit) together
 * with per-triangle frames used by the closest-point evaluation. The paper
 * builds an AABB tree over B before any query (Implementation section).
 * Returns HD_E_INVALID for nB <= 0, mB <= 0, an out-of-range index or a
 * non-finite coordinate. The handle is usable once the stream reaches it. */
hd_status hd_build_bvh(const double *VB, int64_t mB, const int32_t *FB, int64_t nB,
                       hd_stream_t stream, hd_bvh *out);

/* One BVH over npairs soups B_p (host arrays of npairs device pointers and
 * sizes): keys (pair id, Morton code) give every pair its own subtree, and
 * the returned handle serves hd_bound_batched with the same pair order. The
 * per-pair original face index is what the queries report. */
hd_status hd_build_bvh_batched(int32_t npairs, const double *const *VB, const int64_t *mB,
                               const int32_t *const *FB, const int64_t *nB, hd_stream_t stream,
                               hd_bvh *out);

/* Release a handle from hd_build_bvh or hd_build_bvh_batched (NULL is allowed).
 * Waits for the device to go idle (work on any stream may still read the
 * BVH). The library may keep the handle's device buffers for a later build on
 * the same device instead of freeing them. */
void hd_free_bvh(hd_bvh bvh);

/* Whether hd_build_bvh / hd_build_bvh_batched run the build as a HIP graph
 * (default 1): the build's copies and kernels depend only on the soup sizes
 * and the buffers, so they are captured once per (sizes, buffers) and
 * replayed by later builds, one graph launch instead of about 20 kernel
 * launches and copies (a few graphs are kept per device). 0 launches every kernel
 * directly. The result is the same either way. Returns the previous
 * setting; the setting is process-wide. */
int32_t hd_build_graphs(int32_t enable);

/* Certified [L, U] for h(A, B), B given by its BVH: on success
 * L <= h(A,B) <= U and U - L <= eps, eps the absolute tolerance (the paper's
 * relative tolerance times dA, eq. output_bounds; hd_options.eps_relative = 1
 * takes the relative form and computes dA on the device).
 * opt may be NULL (defaults). LU_out is a HOST array of 2 doubles; stats is a
 * host struct or NULL. The stream is synchronised before return.
 * HD_E_INVALID for nA <= 0, mA <= 0, eps <= 0, a bad option, or an
 * out-of-range index or non-finite coordinate in A. The device finds the
 * latter while ingesting A, so the call returns it at its first report, after
 * the work already enqueued has drained. That work runs on sanitised copies:
 * indices are replaced and values zeroed.
 * With HD_PREC_FP32 (no FP64 recheck) the tolerance must exceed the FP32
 * margin at the lower bound (mu_coef_d * L + mu_coef_0 in hd_stats): no FP32
 * bound can then park the triangle that holds the maximum, so the call
 * returns HD_E_INVALID after the vertex round instead of subdividing to the
 * depth limit (use HD_PREC_FP32_RECHECK or HD_PREC_FP64 there). */
hd_status hd_bound(const double *VA, int64_t mA, const int32_t *FA, int64_t nA, hd_bvh B,
                   double eps, const hd_options *opt, hd_stream_t stream, double LU_out[2],
                   hd_stats *stats);

/* Certified [L_p, U_p] for npairs independent pairs (A_p, B_p) in one call:
 * the pairs share every kernel launch of every round (records carry their
 * pair id; L, U, eps and the margins are per pair). A_p is given as host
 * arrays of device pointers and sizes; B is a handle from
 * hd_build_bvh_batched over the B_p in the same order. eps is a host array
 * of npairs tolerances when eps_per_pair != 0, else one value (absolute, or
 * relative to each pair's dA with hd_options.eps_relative = 1).
 * LU_out is a host array of 2 * npairs doubles (L_0, U_0, L_1, U_1, ...);
 * stats (host, nullable) sums the counters over pairs and reports pair 0's
 * dA and eps_abs. A pair whose vertices are all referenced by no face is
 * HD_E_INVALID like an empty mesh. */
hd_status hd_bound_batched(int32_t npairs, const double *const *VA, const int64_t *mA,
                           const int32_t *const *FA, const int64_t *nA, hd_bvh B, const double *eps,
                           int32_t eps_per_pair, const hd_options *opt, hd_stream_t stream,
                           double *LU_out, hd_stats *stats);

/* Certified [L, U] for the two-sided distance H(A,B) = max{h(A,B), h(B,A)}
 * (Conclusion and future work: the symmetric distance, with the lower bound of
 * one direction reused by the other). Both directions run as one two-pair
 * call over one BVH of both soups (built inside the call), and their
 * decisions share one lower bound, the larger of the two: a triangle of
 * either direction bounded below it cannot raise H. On success
 * L <= H(A,B) <= U and U - L <= eps (absolute; with hd_options.eps_relative = 1
 * relative to the larger of the two soups' bounding-box diagonals).
 * LU_out: HOST array of 2 doubles. LU_dir (host, 4 doubles, nullable):
 * [L, U] of h(A,B), then of h(B,A); each contains its distance but may be
 * wider than eps (the direction whose distance is the smaller one stops as
 * soon as it cannot exceed the other). Soups are device arrays as for
 * hd_bound; stats (nullable) sums both directions. Errors as for hd_bound. */
hd_status hd_hausdorff(const double *VA, int64_t mA, const int32_t *FA, int64_t nA, const double *VB, int64_t mB,
                       const int32_t *FB, int64_t nB, double eps, const hd_options *opt, hd_stream_t stream,
                       double LU_out[2], double LU_dir[4], hd_stats *stats);

/* Distances from nP points P (device, nP x 3 doubles) to B: d (device, nP
 * doubles), closest face of B as its original index (device, nP int32) and
 * closest points (device, nP x 3 doubles; may be NULL). precision selects
 * FP64 or FP32 arithmetic (HD_PREC_FP32 and HD_PREC_FP32_RECHECK both mean
 * FP32 here). lanes (0 or 1: one lane per point; 4: a quad of lanes per
 * point) selects the query kernel; the results do not depend on it. This is
 * the per-vertex query of the Implementation section, exposed for testing
 * and reuse. HD_E_INVALID for other values of lanes. */
hd_status hd_point_distances(const double *P, int64_t nP, hd_bvh B, int32_t precision, int32_t lanes,
                             double *d, int32_t *I, double *Q, hd_stream_t stream);

/* hd_point_distances for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same query kernels and results, with every piece of scratch
 * (control block, pair table, overflow list, deep stack, query results) in a
 * static device array of about 5 MB per GPU, held until the process ends.
 * Nothing is allocated, nothing is copied to the host and the stream is not
 * synchronised: the call only enqueues work on `stream`. *err (a DEVICE
 * int32) receives HD_OK, or HD_E_INTERNAL when a traversal exceeded the deep
 * fallback stack, once the stream reaches the end of the call.
 * At most HD_NOALLOC_MAX_POINTS points per call: more returns HD_E_CAPACITY
 * before anything is enqueued. HD_E_INVALID for a NULL err or bad arguments.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU
 * (other streams, other host threads) race and must be serialised by the
 * caller; consecutive calls on one stream are safe. */
#define HD_NOALLOC_MAX_POINTS 65536
hd_status hd_point_distances_noalloc(const double *P, int64_t nP, hd_bvh B, int32_t precision, int32_t lanes,
                                     double *d, int32_t *I, double *Q, int32_t *err, hd_stream_t stream);

/* All five bounds of n given triangles against B, for testing the bound
 * kernels in isolation ("Upper bounds" subsection). Device arrays: v (n x 9
 * doubles: three vertices), d (n x 3 vertex distances), I (n x 3 closest faces
 * of B, original indices), q (n x 9 closest points). out (device, n x 5
 * doubles) receives uexact (NaN unless the three faces coincide), u1, u2, u3,
 * u4 without rounding margins; u3_case (device, n int32) receives 1 or 2.
 * precision is HD_PREC_FP64 or HD_PREC_FP32. */
hd_status hd_eval_bounds(const double *v, const double *d, const int32_t *I, const double *q, int64_t n,
                         hd_bvh B, int32_t precision, double *out, int32_t *u3_case, hd_stream_t stream);

/* The fifth bound (order digit 5) of n given triangles, for testing it in
 * isolation: v (device, n x 9 doubles), d (n x 3 vertex distances), I (n x 3
 * closest faces of B, original indices); the closest face of each
 * triangle's barycenter comes from a point query and is written to Sb
 * (device, n int32, original index), the bound (no margin) to out (device, n
 * doubles). precision is HD_PREC_FP64 or HD_PREC_FP32. */
hd_status hd_eval_bound_u5(const double *v, const double *d, const int32_t *I, int64_t n, hd_bvh B,
                           int32_t precision, double *out, int32_t *Sb, hd_stream_t stream);

/* ---- learned proposal: the network ---------------------------------------
 * Not part of the paper's method. A 16 -> 64 -> 64 -> 1 ReLU network predicts,
 * for a frontier triangle, (max over the triangle of d(p, B) - largest vertex
 * distance) / longest edge from 16 features; the prediction only orders work
 * and picks which bounds to evaluate, never a discard or a certificate.
 * Parameters: one FP32 vector of hd_mlp_nparams() = 5313 values, W1 [16][64]
 * (input-major), b1 [64], W2 [64][64], b2 [64], w3 [64], b3. The hidden layers
 * run as BF16 x BF16 matrix products with FP32 accumulation, the output layer
 * as an FP32 dot product with BF16-rounded weights. All pointers are device
 * pointers; the calls are asynchronous on `stream`. */
int32_t hd_mlp_nparams(void);

/* y[i] = network(X[i, 0..15]) for i < n (X row-major FP32, 16-byte aligned). */
hd_status hd_mlp_forward(const float *X, int64_t n, const float *params, float *y, hd_stream_t stream);

/* Gradient of the mean squared error (1/n) sum_i (y_i - t_i)^2 with respect to
 * the parameters, into grad[5313]; *loss (device, may be NULL) receives the
 * loss. One workgroup; intended for checks and small batches. */
hd_status hd_mlp_grad(const float *X, const float *t, int64_t n, const float *params, float *grad, float *loss,
                      hd_stream_t stream);

/* nsteps Adam steps (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) on
 * the mean squared error; step s uses rows rows[s*batch .. s*batch+batch-1] of
 * (X, t). params, adam_m and adam_v (5313 each) are updated in place; step0 is
 * the number of steps already taken (for the bias correction). loss (device,
 * may be NULL) receives nsteps minibatch losses. Runs in one workgroup. */
hd_status hd_mlp_train(const float *X, const float *t, const int32_t *rows, int64_t nsteps, int32_t batch,
                       float *params, float *adam_m, float *adam_v, int64_t step0, float lr, float *loss,
                       hd_stream_t stream);

/* Test entry: the 16 features of n triangles of a single-pair B (layout as in
 * hd_eval_bounds: v, q n x 9, d, I n x 3 with ORIGINAL face indices), given
 * the running lower bound L and the tolerance scale dA, in FP32 arithmetic,
 * into X (n x 16, device). Out-of-range face indices give NaN rows. */
hd_status hd_frontier_features(const double *v, const double *d, const int32_t *I, const double *q, int64_t n,
                               hd_bvh B, double L, double dA, float *X, hd_stream_t stream);

/* Human-readable name of a status code (static string). */
const char *hd_status_str(hd_status s);

/* Default options (precision FP32 + FP64 recheck, order 1234, m = 1e7). */
void hd_default_options(hd_options *opt);

#ifdef __cplusplus
}
#endif
#endif /* HD_H */
