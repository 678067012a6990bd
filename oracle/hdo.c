/*
 * hdo.c -- FP64 CPU oracle (test infrastructure only; see hdo.h).
 *
 * Follows Sacht & Jacobson, "Cascading upper bounds for triangle soup
 * Pompeiu-Hausdorff distance": the branch and bound of the "Branch and bound"
 * subsection, the exact same-triangle bound and the four upper bounds of the
 * "Upper bounds" subsection, and the main loop of the "Implementation"
 * section (bbox diagonal, per-vertex queries, initial lower bound, priority
 * queue keyed by upper bound, 1->4 midpoint subdivision, face budget m * nA).
 *
 * Written for clarity, not speed: no blocking, fusion or reordering beyond
 * what those passages state. FP64 rounding is treated as exact.
 */
#include "hdo.h"

#include <math.h>
#include <stdlib.h>
#include <pthread.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* small vector helpers                                                     */
/* ------------------------------------------------------------------------ */

static void sub3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2];
}
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double a[3], const double b[3], double r[3]) {
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
static double dist3(const double a[3], const double b[3]) {
    double r[3];
    sub3(a, b, r);
    return sqrt(dot3(r, r));
}
static void mid3(const double a[3], const double b[3], double r[3]) {
    r[0] = 0.5 * (a[0] + b[0]); r[1] = 0.5 * (a[1] + b[1]); r[2] = 0.5 * (a[2] + b[2]);
}
static void copy3(const double a[3], double r[3]) { r[0] = a[0]; r[1] = a[1]; r[2] = a[2]; }
static double max2(double a, double b) { return a > b ? a : b; }
static double min2(double a, double b) { return a < b ? a : b; }
static double max3(double a, double b, double c) { return max2(a, max2(b, c)); }

static void vtx(const double *V, int32_t i, double r[3]) {
    r[0] = V[3 * (int64_t)i]; r[1] = V[3 * (int64_t)i + 1]; r[2] = V[3 * (int64_t)i + 2];
}

/* ------------------------------------------------------------------------ */
/* point to triangle: the closest point of a convex set is either the       */
/* orthogonal projection onto its plane (when that lies inside) or a point  */
/* of its boundary; every candidate below lies in the triangle, so the      */
/* smallest candidate distance is the distance.                             */
/* ------------------------------------------------------------------------ */

static double closest_on_segment(const double p[3], const double a[3], const double b[3],
                                 double q[3]) {
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double len2 = dot3(ab, ab);
    double t = 0.0;
    if (len2 > 0.0) {
        t = dot3(ap, ab) / len2;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    q[0] = a[0] + t * ab[0]; q[1] = a[1] + t * ab[1]; q[2] = a[2] + t * ab[2];
    double r[3];
    sub3(p, q, r);
    return dot3(r, r);
}

double hdo_closest_point(const double p[3], const double a[3], const double b[3],
                         const double c[3], double q[3]) {
    double best = INFINITY, cand[3], d2;
    /* interior candidate: projection onto the plane, if its barycentric
     * coordinates are all non-negative */
    double e1[3], e2[3], n[3], ap[3];
    sub3(b, a, e1);
    sub3(c, a, e2);
    cross3(e1, e2, n);
    double nn = dot3(n, n);
    if (nn > 0.0) {
        sub3(p, a, ap);
        double s = dot3(ap, n) / nn;
        double x[3] = {p[0] - s * n[0], p[1] - s * n[1], p[2] - s * n[2]};
        double xa[3], t1[3], t2[3];
        sub3(x, a, xa);
        cross3(xa, e2, t1);
        cross3(e1, xa, t2);
        double beta = dot3(t1, n) / nn;
        double gamma = dot3(t2, n) / nn;
        double alpha = 1.0 - beta - gamma;
        if (alpha >= 0.0 && beta >= 0.0 && gamma >= 0.0) {
            cand[0] = a[0] + beta * e1[0] + gamma * e2[0];
            cand[1] = a[1] + beta * e1[1] + gamma * e2[1];
            cand[2] = a[2] + beta * e1[2] + gamma * e2[2];
            double r[3];
            sub3(p, cand, r);
            best = dot3(r, r);
            copy3(cand, q);
        }
    }
    /* boundary candidates */
    d2 = closest_on_segment(p, a, b, cand);
    if (d2 < best) { best = d2; copy3(cand, q); }
    d2 = closest_on_segment(p, b, c, cand);
    if (d2 < best) { best = d2; copy3(cand, q); }
    d2 = closest_on_segment(p, c, a, cand);
    if (d2 < best) { best = d2; copy3(cand, q); }
    return best;
}

static double closest_on_face(const double p[3], const double *VB, const int32_t *FB,
                              int32_t f, double q[3]) {
    double a[3], b[3], c[3];
    vtx(VB, FB[3 * (int64_t)f], a);
    vtx(VB, FB[3 * (int64_t)f + 1], b);
    vtx(VB, FB[3 * (int64_t)f + 2], c);
    return hdo_closest_point(p, a, b, c, q);
}

double hdo_point_soup(const double p[3], const double *VB, const int32_t *FB, int64_t nB,
                      int32_t *I, double q[3]) {
    double best = INFINITY, cand[3];
    int32_t bi = -1;
    for (int64_t f = 0; f < nB; ++f) {
        double d2 = closest_on_face(p, VB, FB, (int32_t)f, cand);
        if (d2 < best) { /* strict: exact ties keep the smallest index */
            best = d2;
            bi = (int32_t)f;
            copy3(cand, q);
        }
    }
    *I = bi;
    return sqrt(best);
}

void hdo_points_soup(const double *P, int64_t n, const double *VB, const int32_t *FB, int64_t nB,
                     double *d, int32_t *I) {
    for (int64_t i = 0; i < n; ++i) {
        int32_t bi;
        double q[3];
        d[i] = hdo_point_soup(P + 3 * i, VB, FB, nB, &bi, q);
        if (I) I[i] = bi;
    }
}

/* ------------------------------------------------------------------------ */
/* AABB tree (median split), an independent stand-in for brute force on     */
/* large soups                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    double lo[3], hi[3];
    int64_t left, right;  /* children, or -1 for a leaf */
    int64_t start, count; /* leaf range in tri[] */
} tnode;

struct hdo_tree_s {
    const double *VB;
    const int32_t *FB;
    int64_t nB;
    int32_t *tri;
    double *cen;
    tnode *nodes;
    int64_t nnodes, cap;
};

static int g_sort_axis;
static const double *g_sort_cen;
static int cmp_centroid(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    double ca = g_sort_cen[3 * (int64_t)a + g_sort_axis], cb = g_sort_cen[3 * (int64_t)b + g_sort_axis];
    if (ca < cb) return -1;
    if (ca > cb) return 1;
    return (a > b) - (a < b);
}

static int64_t tree_new_node(struct hdo_tree_s *t) {
    if (t->nnodes == t->cap) {
        t->cap = t->cap ? 2 * t->cap : 1024;
        t->nodes = (tnode *)realloc(t->nodes, (size_t)t->cap * sizeof(tnode));
    }
    return t->nnodes++;
}

static int64_t tree_build_rec(struct hdo_tree_s *t, int64_t start, int64_t count) {
    int64_t id = tree_new_node(t);
    tnode nd;
    for (int k = 0; k < 3; ++k) { nd.lo[k] = INFINITY; nd.hi[k] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = start; i < start + count; ++i) {
        int32_t f = t->tri[i];
        for (int j = 0; j < 3; ++j) {
            double v[3];
            vtx(t->VB, t->FB[3 * (int64_t)f + j], v);
            for (int k = 0; k < 3; ++k) {
                nd.lo[k] = min2(nd.lo[k], v[k]);
                nd.hi[k] = max2(nd.hi[k], v[k]);
            }
        }
        for (int k = 0; k < 3; ++k) {
            clo[k] = min2(clo[k], t->cen[3 * (int64_t)f + k]);
            chi[k] = max2(chi[k], t->cen[3 * (int64_t)f + k]);
        }
    }
    nd.start = start;
    nd.count = count;
    nd.left = nd.right = -1;
    if (count > 4) {
        int axis = 0;
        for (int k = 1; k < 3; ++k)
            if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
        g_sort_axis = axis;
        g_sort_cen = t->cen;
        qsort(t->tri + start, (size_t)count, sizeof(int32_t), cmp_centroid);
        int64_t half = count / 2;
        int64_t l = tree_build_rec(t, start, half);
        int64_t r = tree_build_rec(t, start + half, count - half);
        nd.left = l;
        nd.right = r;
    }
    t->nodes[id] = nd;
    return id;
}

hdo_tree hdo_tree_build(const double *VB, int64_t mB, const int32_t *FB, int64_t nB) {
    (void)mB;
    struct hdo_tree_s *t = (struct hdo_tree_s *)calloc(1, sizeof(*t));
    t->VB = VB;
    t->FB = FB;
    t->nB = nB;
    t->tri = (int32_t *)malloc((size_t)nB * sizeof(int32_t));
    t->cen = (double *)malloc((size_t)nB * 3 * sizeof(double));
    for (int64_t f = 0; f < nB; ++f) {
        t->tri[f] = (int32_t)f;
        double a[3], b[3], c[3];
        vtx(VB, FB[3 * f], a);
        vtx(VB, FB[3 * f + 1], b);
        vtx(VB, FB[3 * f + 2], c);
        for (int k = 0; k < 3; ++k) t->cen[3 * f + k] = (a[k] + b[k] + c[k]) / 3.0;
    }
    tree_build_rec(t, 0, nB);
    return t;
}

void hdo_tree_free(hdo_tree t) {
    if (!t) return;
    free(t->tri);
    free(t->cen);
    free(t->nodes);
    free(t);
}

static double box_dist2(const tnode *nd, const double p[3]) {
    double s = 0.0;
    for (int k = 0; k < 3; ++k) {
        double e = 0.0;
        if (p[k] < nd->lo[k]) e = nd->lo[k] - p[k];
        else if (p[k] > nd->hi[k]) e = p[k] - nd->hi[k];
        s += e * e;
    }
    return s;
}

typedef struct { double best; int32_t I; double q[3]; int64_t evals; } tquery;

static void tree_query_rec(const struct hdo_tree_s *t, int64_t id, const double p[3], tquery *st) {
    const tnode *nd = &t->nodes[id];
    /* a box strictly farther than the best so far cannot hold a closer or an
     * equally close triangle */
    if (box_dist2(nd, p) > st->best) return;
    if (nd->left < 0) {
        for (int64_t i = nd->start; i < nd->start + nd->count; ++i) {
            int32_t f = t->tri[i];
            double cand[3];
            double d2 = closest_on_face(p, t->VB, t->FB, f, cand);
            st->evals++;
            if (d2 < st->best || (d2 == st->best && f < st->I)) {
                st->best = d2;
                st->I = f;
                copy3(cand, st->q);
            }
        }
        return;
    }
    double dl = box_dist2(&t->nodes[nd->left], p);
    double dr = box_dist2(&t->nodes[nd->right], p);
    if (dl <= dr) {
        tree_query_rec(t, nd->left, p, st);
        tree_query_rec(t, nd->right, p, st);
    } else {
        tree_query_rec(t, nd->right, p, st);
        tree_query_rec(t, nd->left, p, st);
    }
}

double hdo_tree_query(hdo_tree t, const double p[3], int32_t *I, double q[3], int64_t *evals) {
    tquery st;
    st.best = INFINITY;
    st.I = -1;
    st.evals = 0;
    tree_query_rec(t, 0, p, &st);
    *I = st.I;
    copy3(st.q, q);
    if (evals) *evals += st.evals;
    return sqrt(st.best);
}

/* ------------------------------------------------------------------------ */
/* Upper bounds ("Upper bounds" subsection)                                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double v[3][3];  /* vertices v1, v2, v3 */
    double d[3];     /* distances to B */
    int32_t I[3];    /* closest B triangle */
    double q[3][3];  /* closest points on B */
} otri;

typedef struct {
    const double *VB;
    const int32_t *FB;
    int64_t nB;
    int64_t *evals;
    hdo_tree tree;     /* for the point queries a bound makes (NULL: brute force) */
    int64_t *queries;  /* counter of those queries (may be NULL) */
} soupref;

/* distance from x to one triangle S of B */
static double dist_to_face(const soupref *B, const double x[3], int32_t f) {
    double q[3];
    (*B->evals)++;
    return sqrt(closest_on_face(x, B->VB, B->FB, f, q));
}

/* eq. uexact: all three closest points on the same triangle of B */
static double bound_uexact(const otri *T) { return max3(T->d[0], T->d[1], T->d[2]); }

/* eq. u1: the best vertex, plus the longer of its two incident edges */
static double bound_u1(const otri *T) {
    double e12 = dist3(T->v[0], T->v[1]);
    double e23 = dist3(T->v[1], T->v[2]);
    double e31 = dist3(T->v[2], T->v[0]);
    double b1 = max2(e12, e31) + T->d[0];
    double b2 = max2(e12, e23) + T->d[1];
    double b3 = max2(e23, e31) + T->d[2];
    return min2(b1, min2(b2, b3));
}

/* g of eq. u2: the circumradius R when s - r > 2R (acute), else half the
 * longest edge. Zero area falls to the half-longest-edge branch. */
static double u2_g(const double v[3][3]) {
    double e1 = dist3(v[0], v[1]);
    double e2 = dist3(v[1], v[2]);
    double e3 = dist3(v[2], v[0]);
    double ab[3], ac[3], n[3];
    sub3(v[1], v[0], ab);
    sub3(v[2], v[0], ac);
    cross3(ab, ac, n);
    double area = 0.5 * sqrt(dot3(n, n));
    double emax = max3(e1, e2, e3);
    if (area > 0.0) {
        double R = e1 * e2 * e3 / (4.0 * area);
        double s = 0.5 * (e1 + e2 + e3);
        double r = area / s;
        if (s - r > 2.0 * R) return R;
    }
    return 0.5 * emax;
}

/* eq. u2 */
static double bound_u2(const otri *T) {
    return u2_g(T->v) + max3(T->d[0], T->d[1], T->d[2]);
}

/* Two faces of B share an edge when they have at least two vertex indices in
 * common (the soup has no other adjacency information). On success writes
 * the shared edge endpoints' vertex ids. */
static int faces_share_edge(const soupref *B, int32_t f, int32_t g, int32_t *ea, int32_t *eb) {
    const int32_t *F = B->FB;
    int32_t common[3];
    int nc = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (F[3 * (int64_t)f + i] == F[3 * (int64_t)g + j]) {
                int dup = 0;
                for (int k = 0; k < nc; ++k) dup |= common[k] == F[3 * (int64_t)f + i];
                if (!dup) common[nc++] = F[3 * (int64_t)f + i];
            }
    if (nc < 2) return 0;
    *ea = common[0];
    *eb = common[1];
    return 1;
}

/* unit vector in the plane of face f, perpendicular to edge (a,b), pointing
 * towards the face's third vertex; returns 0 when undefined */
static int inplane_normal(const soupref *B, int32_t f, int32_t ia, int32_t ib, double t[3]) {
    int32_t ic = -1;
    for (int i = 0; i < 3; ++i) {
        int32_t x = B->FB[3 * (int64_t)f + i];
        if (x != ia && x != ib) ic = x;
    }
    if (ic < 0) return 0;
    double a[3], b[3], c[3], e[3], w[3];
    vtx(B->VB, ia, a);
    vtx(B->VB, ib, b);
    vtx(B->VB, ic, c);
    sub3(b, a, e);
    sub3(c, a, w);
    double ee = dot3(e, e);
    if (!(ee > 0.0)) return 0;
    double s = dot3(w, e) / ee;
    for (int k = 0; k < 3; ++k) t[k] = w[k] - s * e[k];
    double tn = sqrt(dot3(t, t));
    if (!(tn > 0.0)) return 0;
    for (int k = 0; k < 3; ++k) t[k] /= tn;
    return 1;
}

/* eq. Kang2018_case1: v[i1] projects to S1, the other two vertices to S2,
 * S1 and S2 adjacent through the edge (ea, eb). */
static double bound_u3_case1(const otri *T, const soupref *B, int i1, int32_t S1, int32_t S2,
                             int32_t ea, int32_t eb) {
    int i2 = (i1 + 1) % 3, i3 = (i1 + 2) % 3;
    const double *v1 = T->v[i1], *v2 = T->v[i2], *v3 = T->v[i3];
    double b1[3], b2[3];
    int found = 0;
    double t1[3], t2[3];
    if (inplane_normal(B, S1, ea, eb, t1) && inplane_normal(B, S2, ea, eb, t2)) {
        double nu[3] = {t1[0] - t2[0], t1[1] - t2[1], t1[2] - t2[2]};
        if (dot3(nu, nu) > 0.0) {
            double a[3];
            vtx(B->VB, ea, a);
            double x[3];
            sub3(v1, a, x); double f1 = dot3(x, nu);
            sub3(v2, a, x); double f2 = dot3(x, nu);
            sub3(v3, a, x); double f3 = dot3(x, nu);
            /* the bisecting plane must cut both edges v1v2 and v1v3 */
            if (f1 != f2 && f1 != f3) {
                double s12 = f1 / (f1 - f2), s13 = f1 / (f1 - f3);
                if (s12 >= 0.0 && s12 <= 1.0 && s13 >= 0.0 && s13 <= 1.0) {
                    for (int k = 0; k < 3; ++k) {
                        b1[k] = v1[k] + s12 * (v2[k] - v1[k]);
                        b2[k] = v1[k] + s13 * (v3[k] - v1[k]);
                    }
                    found = 1;
                }
            }
        }
    }
    if (!found) {
        mid3(v1, v2, b1);
        mid3(v1, v3, b2);
    }
    /* h(R,S1) over R = (v1,b1,b2); h(Q,S2) over Q = (v3,b2,b1,v2) */
    double hR = max3(T->d[i1], dist_to_face(B, b1, S1), dist_to_face(B, b2, S1));
    double hQ = max2(max2(T->d[i2], T->d[i3]),
                     max2(dist_to_face(B, b1, S2), dist_to_face(B, b2, S2)));
    return max2(hR, hQ);
}

/* eq. Kang2018_case2_partial and eq. Kang2018_case2 */
static double bound_u3_case2(const otri *T, const soupref *B) {
    const double *v1 = T->v[0], *v2 = T->v[1], *v3 = T->v[2];
    double m1[3], m2[3], m3[3], b[3];
    mid3(v1, v2, m1);
    mid3(v2, v3, m2);
    mid3(v3, v1, m3);
    for (int k = 0; k < 3; ++k) b[k] = (v1[k] + v2[k] + v3[k]) / 3.0;
    int32_t S1 = T->I[0], S2 = T->I[1], S3 = T->I[2];
    /* Q1 = (v1,m1,b,m3) to S1, Q2 = (v2,m2,b,m1) to S2, Q3 = (v3,m3,b,m2) to S3 */
    double h1 = max2(max2(T->d[0], dist_to_face(B, m1, S1)),
                     max2(dist_to_face(B, b, S1), dist_to_face(B, m3, S1)));
    double h2 = max2(max2(T->d[1], dist_to_face(B, m2, S2)),
                     max2(dist_to_face(B, b, S2), dist_to_face(B, m1, S2)));
    double h3 = max2(max2(T->d[2], dist_to_face(B, m3, S3)),
                     max2(dist_to_face(B, b, S3), dist_to_face(B, m2, S3)));
    double partial = max3(h1, h2, h3);
    /* h(T,S_i) = max over the three vertices of their distance to S_i */
    double best = partial;
    for (int i = 0; i < 3; ++i) {
        double h = 0.0;
        for (int j = 0; j < 3; ++j) {
            double dj = (j == i) ? T->d[i] : dist_to_face(B, T->v[j], T->I[i]);
            h = max2(h, dj);
        }
        best = min2(best, h);
    }
    return best;
}

/* Third bound: case 1 when exactly two distinct closest triangles that share
 * an edge, otherwise case 2. */
static double bound_u3(const otri *T, const soupref *B, int32_t *which_case) {
    int32_t I1 = T->I[0], I2 = T->I[1], I3 = T->I[2];
    int odd = -1; /* the vertex whose closest triangle differs from the others */
    if (I1 != I2 && I2 == I3) odd = 0;
    else if (I2 != I1 && I1 == I3) odd = 1;
    else if (I3 != I1 && I1 == I2) odd = 2;
    if (odd >= 0) {
        int32_t S1 = T->I[odd], S2 = T->I[(odd + 1) % 3];
        int32_t ea, eb;
        if (faces_share_edge(B, S1, S2, &ea, &eb)) {
            if (which_case) *which_case = 1;
            return bound_u3_case1(T, B, odd, S1, S2, ea, eb);
        }
    }
    if (which_case) *which_case = 2;
    return bound_u3_case2(T, B);
}

/* h(T, {x, y}): the maximum of min(|p-x|, |p-y|) over T is reached at a vertex
 * of T or where an edge of T crosses the bisector plane of x and y. */
static double h_tri_two_points(const otri *T, const double x[3], const double y[3]) {
    double h = 0.0;
    for (int j = 0; j < 3; ++j)
        h = max2(h, min2(dist3(T->v[j], x), dist3(T->v[j], y)));
    double w[3], m[3];
    sub3(y, x, w);
    if (dot3(w, w) == 0.0) return h;
    mid3(x, y, m);
    double f[3];
    for (int j = 0; j < 3; ++j) {
        double r[3];
        sub3(T->v[j], m, r);
        f[j] = dot3(r, w);
    }
    for (int j = 0; j < 3; ++j) {
        int k = (j + 1) % 3;
        if (f[j] * f[k] < 0.0) {
            double t = f[j] / (f[j] - f[k]);
            double p[3];
            for (int c = 0; c < 3; ++c) p[c] = T->v[j][c] + t * (T->v[k][c] - T->v[j][c]);
            h = max2(h, dist3(p, x));
        }
    }
    return h;
}

/* eq. bound_u4: q2, q3 are the footpoints of the shortest edge's endpoints,
 * q1 the footpoint of the remaining vertex */
static double bound_u4(const otri *T) {
    double e[3] = {dist3(T->v[0], T->v[1]), dist3(T->v[1], T->v[2]), dist3(T->v[2], T->v[0])};
    int s = 0;
    if (e[1] < e[s]) s = 1;
    if (e[2] < e[s]) s = 2;
    int a = s, b = (s + 1) % 3, c = (s + 2) % 3;
    const double *q1 = T->q[c], *q2 = T->q[a], *q3 = T->q[b];
    return min2(h_tri_two_points(T, q1, q2), h_tri_two_points(T, q1, q3));
}

/* The bound of Zheng et al. that the paper quotes in its fourth-bound
 * subsection: min over S in {S1, S2, S3, S_b} of h(T, S), where S_b is the
 * triangle of B closest to the barycenter b of T (one more point query), and
 * h(T, S), the distance from the triangle T to the triangle S, is the largest
 * distance of a vertex of T to S (the distance to a convex set is a convex
 * function, so its maximum over T is reached at a vertex). *Sb_out (may be
 * NULL) receives S_b. */
static double bound_u5(const otri *T, const soupref *B, int32_t *Sb_out) {
    double b[3], qb[3];
    for (int k = 0; k < 3; ++k) b[k] = (T->v[0][k] + T->v[1][k] + T->v[2][k]) / 3.0;
    int32_t Sb = -1;
    if (B->queries) (*B->queries)++;
    if (B->tree) {
        hdo_tree_query(B->tree, b, &Sb, qb, B->evals);
    } else {
        *B->evals += B->nB;
        hdo_point_soup(b, B->VB, B->FB, B->nB, &Sb, qb);
    }
    if (Sb_out) *Sb_out = Sb;
    const int32_t S[4] = {T->I[0], T->I[1], T->I[2], Sb};
    double best = INFINITY;
    for (int i = 0; i < 4; ++i) {
        double h = 0.0;
        for (int j = 0; j < 3; ++j) {
            /* vertex i's distance to its own closest triangle is known */
            const double dj = (i < 3 && j == i) ? T->d[i] : dist_to_face(B, T->v[j], S[i]);
            h = max2(h, dj);
        }
        best = min2(best, h);
    }
    return best;
}

static double bound_k(int k, const otri *T, const soupref *B) {
    switch (k) {
    case 1: return bound_u1(T);
    case 2: return bound_u2(T);
    case 3: return bound_u3(T, B, NULL);
    case 4: return bound_u4(T);
    case 5: return bound_u5(T, B, NULL);
    }
    return INFINITY;
}

void hdo_bounds(const double v[9], const double d[3], const int32_t I[3], const double q[9],
                const double *VB, const int32_t *FB, int64_t nB, double out[5],
                int32_t *u3_case) {
    otri T;
    for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < 3; ++k) {
            T.v[i][k] = v[3 * i + k];
            T.q[i][k] = q[3 * i + k];
        }
        T.d[i] = d[i];
        T.I[i] = I[i];
    }
    int64_t evals = 0;
    soupref B = {VB, FB, nB, &evals, NULL, NULL};
    out[0] = (I[0] == I[1] && I[1] == I[2]) ? bound_uexact(&T) : NAN;
    out[1] = bound_u1(&T);
    out[2] = bound_u2(&T);
    out[3] = bound_u3(&T, &B, u3_case);
    out[4] = bound_u4(&T);
}

double hdo_bound_u5(const double v[9], const double d[3], const int32_t I[3], const double *VB,
                    const int32_t *FB, int64_t nB, int32_t *Sb) {
    otri T;
    for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < 3; ++k) {
            T.v[i][k] = v[3 * i + k];
            T.q[i][k] = 0.0;
        }
        T.d[i] = d[i];
        T.I[i] = I[i];
    }
    int64_t evals = 0;
    soupref B = {VB, FB, nB, &evals, NULL, NULL};
    return bound_u5(&T, &B, Sb);
}

/* UpperBound: the exact bound when all closest points share a triangle of B;
 * otherwise the bounds in the given order, stopping at the first one below
 * the lower bound l (the triangle is then discarded); if none is below l,
 * the minimum of all of them. *decider gets the bound that decided. */
static double upper_bound(const otri *T, double l, const int32_t *order, int norder,
                          const soupref *B, int *decider) {
    if (T->I[0] == T->I[1] && T->I[1] == T->I[2]) {
        *decider = HDO_UEXACT;
        return bound_uexact(T);
    }
    double best = INFINITY;
    *decider = order[norder - 1];
    for (int i = 0; i < norder; ++i) {
        double u = bound_k(order[i], T, B);
        if (u < l) {
            *decider = order[i];
            return u;
        }
        if (u < best) {
            best = u;
            *decider = order[i];
        }
    }
    return best;
}

/* ------------------------------------------------------------------------ */
/* max-heap on (ub desc, insertion sequence asc)                            */
/* ------------------------------------------------------------------------ */

typedef struct { double ub; int64_t seq; int64_t tri; } hentry;
typedef struct { hentry *a; int64_t n, cap; } heap;

static int h_before(const hentry *x, const hentry *y) {
    if (x->ub != y->ub) return x->ub > y->ub;
    return x->seq < y->seq;
}

static int heap_push(heap *h, hentry e) {
    if (h->n == h->cap) {
        int64_t nc = h->cap ? 2 * h->cap : 1024;
        hentry *na = (hentry *)realloc(h->a, (size_t)nc * sizeof(hentry));
        if (!na) return 0;
        h->a = na;
        h->cap = nc;
    }
    int64_t i = h->n++;
    h->a[i] = e;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!h_before(&h->a[i], &h->a[p])) break;
        hentry t = h->a[i]; h->a[i] = h->a[p]; h->a[p] = t;
        i = p;
    }
    return 1;
}

static hentry heap_pop(heap *h) {
    hentry top = h->a[0];
    h->a[0] = h->a[--h->n];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->n && h_before(&h->a[l], &h->a[m])) m = l;
        if (r < h->n && h_before(&h->a[r], &h->a[m])) m = r;
        if (m == i) break;
        hentry t = h->a[i]; h->a[i] = h->a[m]; h->a[m] = t;
        i = m;
    }
    return top;
}

/* ------------------------------------------------------------------------ */
/* the branch and bound                                                     */
/* ------------------------------------------------------------------------ */

typedef struct { otri *a; int64_t n, cap; } tripool;

static int64_t pool_add(tripool *p, const otri *t) {
    if (p->n == p->cap) {
        int64_t nc = p->cap ? 2 * p->cap : 1024;
        otri *na = (otri *)realloc(p->a, (size_t)nc * sizeof(otri));
        if (!na) return -1;
        p->a = na;
        p->cap = nc;
    }
    p->a[p->n] = *t;
    return p->n++;
}

typedef struct {
    const double *VB;
    const int32_t *FB;
    int64_t nB;
    hdo_tree tree;
    hdo_result *res;
} qctx;

static double query_point(qctx *c, const double p[3], int32_t *I, double q[3]) {
    c->res->queries++;
    if (c->tree) return hdo_tree_query(c->tree, p, I, q, &c->res->evals);
    c->res->evals += c->nB;
    return hdo_point_soup(p, c->VB, c->FB, c->nB, I, q);
}

/* Threads of the vertex-query phase (1 = the plain single-threaded oracle).
 * The phase computes D_A, I_A and C_A for every referenced vertex: each
 * query is independent, so threads take contiguous vertex ranges with their
 * own counters; the lower bound and its argmax are then taken in vertex
 * order, as in the single-threaded run. Results are identical. */
static int g_threads = 1;
void hdo_set_threads(int32_t n) { g_threads = n < 1 ? 1 : (n > 256 ? 256 : n); }

typedef struct {
    const qctx *c;
    const double *VA;
    const unsigned char *ref;
    int64_t lo, hi;
    double *DA, *CA;
    int32_t *IA;
    hdo_result counters;
} vq_job;

static void *vq_run(void *arg) {
    vq_job *j = (vq_job *)arg;
    qctx c = *j->c;
    c.res = &j->counters;
    for (int64_t i = j->lo; i < j->hi; ++i)
        if (j->ref[i]) j->DA[i] = query_point(&c, j->VA + 3 * i, &j->IA[i], j->CA + 3 * i);
    return NULL;
}

static void query_vertices(qctx *c, const double *VA, int64_t mA, const unsigned char *ref, double *DA,
                           int32_t *IA, double *CA) {
    int nt = g_threads;
    if (nt > mA) nt = (int)mA;
    vq_job jobs[256];
    pthread_t th[256];
    int started[256];
    for (int t = 0; t < nt; ++t) {
        memset(&jobs[t], 0, sizeof(jobs[t]));
        jobs[t].c = c;
        jobs[t].VA = VA;
        jobs[t].ref = ref;
        jobs[t].lo = mA * t / nt;
        jobs[t].hi = mA * (t + 1) / nt;
        jobs[t].DA = DA;
        jobs[t].IA = IA;
        jobs[t].CA = CA;
        started[t] = nt > 1 && pthread_create(&th[t], NULL, vq_run, &jobs[t]) == 0;
        if (!started[t]) vq_run(&jobs[t]);
    }
    for (int t = 0; t < nt; ++t) {
        if (started[t]) pthread_join(th[t], NULL);
        c->res->queries += jobs[t].counters.queries;
        c->res->evals += jobs[t].counters.evals;
    }
}

static int all_finite(const double *x, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

int32_t hdo_bound(const double *VA, int64_t mA, const int32_t *FA, int64_t nA,
                  const double *VB, int64_t mB, const int32_t *FB, int64_t nB,
                  double eps_rel, double budget_m, const int32_t *order, int32_t norder,
                  int32_t backend, hdo_result *res) {
    memset(res, 0, sizeof(*res));
    res->L = res->U = NAN;
    static const int32_t default_order[4] = {1, 2, 3, 4};
    if (!order || norder <= 0) {
        order = default_order;
        norder = 4;
    }
    /* validation */
    if (!(eps_rel > 0.0) || nA <= 0 || nB <= 0 || mA <= 0 || mB <= 0 || norder > 5) {
        res->status = HDO_E_INVALID;
        return res->status;
    }
    for (int i = 0; i < norder; ++i)
        if (order[i] < 1 || order[i] > 5) { res->status = HDO_E_INVALID; return res->status; }
    for (int64_t i = 0; i < 3 * nA; ++i)
        if (FA[i] < 0 || FA[i] >= mA) { res->status = HDO_E_INVALID; return res->status; }
    for (int64_t i = 0; i < 3 * nB; ++i)
        if (FB[i] < 0 || FB[i] >= mB) { res->status = HDO_E_INVALID; return res->status; }
    if (!all_finite(VA, 3 * mA) || !all_finite(VB, 3 * mB)) {
        res->status = HDO_E_INVALID;
        return res->status;
    }
    if (!(budget_m > 0.0)) budget_m = 1e7;

    /* only vertices referenced by a face belong to A */
    unsigned char *ref = (unsigned char *)calloc((size_t)mA, 1);
    for (int64_t i = 0; i < 3 * nA; ++i) ref[FA[i]] = 1;

    /* dA: diagonal of the bounding box of A (eq. output_bounds) */
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = 0; i < mA; ++i) {
        if (!ref[i]) continue;
        for (int k = 0; k < 3; ++k) {
            lo[k] = min2(lo[k], VA[3 * i + k]);
            hi[k] = max2(hi[k], VA[3 * i + k]);
        }
    }
    double diag[3];
    sub3(hi, lo, diag);
    res->dA = sqrt(dot3(diag, diag));
    res->eps_abs = eps_rel * res->dA;
    const double eps = res->eps_abs;

    qctx qc = {VB, FB, nB, NULL, res};
    if (backend == 1) qc.tree = hdo_tree_build(VB, mB, FB, nB);
    soupref B = {VB, FB, nB, &res->evals, qc.tree, &res->queries};

    /* distances of all referenced vertices; the initial lower bound */
    double *DA = (double *)malloc((size_t)mA * sizeof(double));
    int32_t *IA = (int32_t *)malloc((size_t)mA * sizeof(int32_t));
    double *CA = (double *)malloc((size_t)mA * 3 * sizeof(double));
    double l = 0.0;
    int have_l = 0;
    query_vertices(&qc, VA, mA, ref, DA, IA, CA);
    for (int64_t i = 0; i < mA; ++i) {
        if (!ref[i]) continue;
        if (!have_l || DA[i] > l) {
            l = DA[i];
            copy3(VA + 3 * i, res->argmax);
            have_l = 1;
        }
    }

    tripool pool = {0};
    heap Q = {0};
    int64_t seq = 0;
    int status = HDO_OK;

    /* upper bound of every face; push those not below l */
    for (int64_t f = 0; f < nA && status == HDO_OK; ++f) {
        otri T;
        for (int j = 0; j < 3; ++j) {
            int32_t vi = FA[3 * f + j];
            copy3(VA + 3 * (int64_t)vi, T.v[j]);
            T.d[j] = DA[vi];
            T.I[j] = IA[vi];
            copy3(CA + 3 * (int64_t)vi, T.q[j]);
        }
        int dec;
        double ub = upper_bound(&T, l, order, norder, &B, &dec);
        res->bounded++;
        if (ub >= l) {
            int64_t id = pool_add(&pool, &T);
            hentry e = {ub, seq++, id};
            if (id < 0 || !heap_push(&Q, e)) status = HDO_E_NOMEM;
            res->pushes++;
        } else {
            res->discards[dec]++;
        }
    }
    free(DA);
    free(IA);
    free(CA);
    free(ref);

    double U = l;
    const double budget = budget_m * (double)nA;
    double cf = (double)nA;
    while (status == HDO_OK) {
        if (Q.n > res->max_queue) res->max_queue = Q.n;
        if (Q.n == 0) {
            /* only possible with an inconsistent lower bound */
            res->empty_queue = 1;
            U = l;
            break;
        }
        U = max2(l, Q.a[0].ub);
        if (U - l <= eps) break;
        hentry top = heap_pop(&Q);
        if (top.ub < l) {
            res->stale++;
            continue;
        }
        otri P = pool.a[top.tri];
        /* 1->4 midpoint subdivision */
        double m[3][3];
        int32_t mI[3];
        double md[3], mq[3][3];
        mid3(P.v[0], P.v[1], m[0]);
        mid3(P.v[1], P.v[2], m[1]);
        mid3(P.v[2], P.v[0], m[2]);
        for (int j = 0; j < 3; ++j) {
            md[j] = query_point(&qc, m[j], &mI[j], mq[j]);
            if (md[j] > l) {
                l = md[j];
                copy3(m[j], res->argmax);
            }
        }
        res->subdivided++;
        /* children: (v1,m12,m31), (m12,v2,m23), (m31,m23,v3), (m12,m23,m31) */
        static const int kids[4][3] = {{0, 3, 5}, {3, 1, 4}, {5, 4, 2}, {3, 4, 5}};
        for (int c = 0; c < 4; ++c) {
            otri C;
            for (int j = 0; j < 3; ++j) {
                int s = kids[c][j];
                if (s < 3) {
                    copy3(P.v[s], C.v[j]);
                    C.d[j] = P.d[s];
                    C.I[j] = P.I[s];
                    copy3(P.q[s], C.q[j]);
                } else {
                    copy3(m[s - 3], C.v[j]);
                    C.d[j] = md[s - 3];
                    C.I[j] = mI[s - 3];
                    copy3(mq[s - 3], C.q[j]);
                }
            }
            int dec;
            double ub = upper_bound(&C, l, order, norder, &B, &dec);
            res->bounded++;
            if (ub >= l) {
                int64_t id = pool_add(&pool, &C);
                hentry e = {ub, seq++, id};
                if (id < 0 || !heap_push(&Q, e)) { status = HDO_E_NOMEM; break; }
                res->pushes++;
            } else {
                res->discards[dec]++;
            }
        }
        cf += 4.0;
        if (cf > budget) status = HDO_E_CAPACITY;
    }
    free(pool.a);
    free(Q.a);
    hdo_tree_free(qc.tree);
    res->status = status;
    if (status == HDO_OK) {
        res->L = l;
        res->U = U;
    }
    return status;
}
