/*
 * hdo -- FP64 CPU oracle for certified one-sided Pompeiu-Hausdorff bounds.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, plain reference that the
 * HIP library is checked against. Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it. It shares no code, header,
 * table or helper with the GPU library.
 *
 * Everything is double precision and single-threaded; FP64 rounding is treated
 * as exact. Meshes are vertex arrays V (m x 3, row-major) and 0-based face
 * arrays F (n x 3).
 */
#ifndef HDO_H
#define HDO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { HDO_OK = 0, HDO_E_INVALID = 1, HDO_E_CAPACITY = 2, HDO_E_NOMEM = 3, HDO_E_INTERNAL = 5 };

/* Bound identifiers used in the order array and the discard counters. */
enum { HDO_UEXACT = 0, HDO_U1 = 1, HDO_U2 = 2, HDO_U3 = 3, HDO_U4 = 4, HDO_U5 = 5 /* Zheng et al. */ };

typedef struct {
    double L, U;             /* certified interval, L <= h(A,B) <= U */
    double dA;               /* bbox diagonal of the referenced A vertices */
    double eps_abs;          /* eps_rel * dA */
    int64_t subdivided;      /* popped triangles that were split 1->4 */
    int64_t bounded;         /* triangles whose upper bound was computed */
    int64_t queries;         /* point -> B distance queries */
    int64_t evals;           /* point-triangle closest-point evaluations */
    int64_t pushes;          /* triangles pushed into the priority queue */
    int64_t stale;           /* popped triangles already below the lower bound */
    int64_t discards[6];     /* triangles discarded by uexact, u1, u2, u3, u4, u5 */
    int64_t max_queue;       /* peak priority-queue length */
    int32_t status;          /* HDO_* */
    int32_t empty_queue;     /* 1 if the queue emptied before the tolerance held */
    double argmax[3];        /* vertex that attains L */
} hdo_result;

/* Closest point on triangle (a,b,c) to p; returns the squared distance and
 * writes the closest point to q. Degenerate triangles are allowed. */
double hdo_closest_point(const double p[3], const double a[3], const double b[3],
                         const double c[3], double q[3]);

/* Brute-force distance from p to the soup (VB,FB): returns d and writes the
 * closest triangle (smallest index among exact ties) and the closest point. */
double hdo_point_soup(const double p[3], const double *VB, const int32_t *FB, int64_t nB,
                      int32_t *I, double q[3]);

/* hdo_point_soup for n points P (n x 3); writes d[n] (and I[n] if non-NULL). */
void hdo_points_soup(const double *P, int64_t n, const double *VB, const int32_t *FB, int64_t nB,
                     double *d, int32_t *I);

/* Median-split AABB tree over the soup, for workloads too large to query by
 * brute force. Same answers as hdo_point_soup, including the tie rule. */
typedef struct hdo_tree_s *hdo_tree;
hdo_tree hdo_tree_build(const double *VB, int64_t mB, const int32_t *FB, int64_t nB);
double hdo_tree_query(hdo_tree t, const double p[3], int32_t *I, double q[3], int64_t *evals);
void hdo_tree_free(hdo_tree t);

/* All five bounds of one triangle T = (v1,v2,v3) (v: 9 doubles) whose vertices
 * have distances d, closest triangles I and closest points q. out[0] = uexact
 * (NaN unless I1 = I2 = I3), out[1..4] = u1..u4. u3_case receives 1 or 2. */
void hdo_bounds(const double v[9], const double d[3], const int32_t I[3], const double q[9],
                const double *VB, const int32_t *FB, int64_t nB, double out[5],
                int32_t *u3_case);

/* The bound of Zheng et al. quoted in the paper's fourth-bound subsection,
 * min over S in {S1, S2, S3, S_b} of the largest vertex distance of T to S,
 * S_b the triangle of B closest to T's barycenter (found by brute force here;
 * written to *Sb). */
double hdo_bound_u5(const double v[9], const double d[3], const int32_t I[3], const double *VB,
                    const int32_t *FB, int64_t nB, int32_t *Sb);

/* The branch-and-bound. eps_rel is the paper's epsilon (relative to dA);
 * budget_m is the paper's m (the queue may process at most m * nA faces);
 * order lists the bounds to try (values 1..4, and 5 for the bound of Zheng
 * et al., which makes one point query per evaluation), norder of them;
 * backend 0 = brute force, 1 = AABB tree. Returns the status, also stored in
 * res. */
int32_t hdo_bound(const double *VA, int64_t mA, const int32_t *FA, int64_t nA,
                  const double *VB, int64_t mB, const int32_t *FB, int64_t nB,
                  double eps_rel, double budget_m, const int32_t *order, int32_t norder,
                  int32_t backend, hdo_result *res);

/* Threads for the vertex-query phase of hdo_bound (default 1, the plain
 * single-threaded oracle). Only that phase is split; results are identical. */
void hdo_set_threads(int32_t n);

#ifdef __cplusplus
}
#endif
#endif
