// hd_geom.hpp -- device geometry: the per-triangle frame record of soup B,
// point-to-triangle distance in that frame, and the paper's upper bounds
// (exact same-triangle bound and u1..u4 of the "Upper bounds" subsection).
//
// Frame record. Every triangle S of B is stored as its longest edge AB
// (length Lb) along an orthonormal in-plane axis ex, a second in-plane axis
// ey pointing towards the third vertex C, and C's in-plane coordinates
// (cx, cy), cy >= 0, 0 <= cx <= Lb. The frame is computed once in FP64 when
// the BVH is built. A point p is then mapped to (x, y, z) in that frame and
// its distance to S is sqrt(z^2 + d2D^2), d2D being the planar distance from
// (x, y) to the planar triangle (0,0),(Lb,0),(cx,cy): zero if inside, else
// the nearest of the three edges. Each step is a short dot product or a
// clamped segment projection, so the rounding error is a few units of
// roundoff times (distance + triangle size + coordinate size), independently
// of how thin the triangle is.
#pragma once
#include "hd_math.hpp"

namespace hd {

template <class T> struct Frame {
    V3<T> A, ex, ey;
    T Lb, cx, cy, inv2bc, inv2ca, R;
    int orig; // original face index within its pair (ties between equal distances)
};

// device layout: float -> 4 x float4 (64 B); double -> 8 x double2 (128 B);
// the last word holds the original face index (int bits / exact double)
HD_D Frame<float> load_frame(const float4 *__restrict__ F, int64_t i) {
    float4 a = F[4 * i], b = F[4 * i + 1], c = F[4 * i + 2], d = F[4 * i + 3];
    Frame<float> f;
    f.A = {a.x, a.y, a.z};
    f.Lb = a.w;
    f.ex = {b.x, b.y, b.z};
    f.cx = b.w;
    f.ey = {c.x, c.y, c.z};
    f.cy = c.w;
    f.inv2bc = d.x;
    f.inv2ca = d.y;
    f.R = d.z;
    f.orig = __builtin_bit_cast(int, d.w);
    return f;
}
HD_D Frame<double> load_frame(const double2 *__restrict__ F, int64_t i) {
    const double2 *p = F + 8 * i;
    double2 a = p[0], b = p[1], c = p[2], d = p[3], e = p[4], g = p[5], h = p[6], k = p[7];
    Frame<double> f;
    f.A = {a.x, a.y, b.x};
    f.Lb = b.y;
    f.ex = {c.x, c.y, d.x};
    f.cx = d.y;
    f.ey = {e.x, e.y, g.x};
    f.cy = g.y;
    f.inv2bc = h.x;
    f.inv2ca = h.y;
    f.R = k.x;
    f.orig = (int)k.y;
    return f;
}

template <class T> HD_HD V3<T> frame_vertex(const Frame<T> &f, int k) {
    if (k == 0) return f.A;
    if (k == 1) return f.A + f.Lb * f.ex;
    return f.A + f.cx * f.ex + f.cy * f.ey;
}

// Squared distance from p to the frame triangle; optionally the closest
// point. Branch-free apart from the final selection.
template <class T, bool WANT_Q>
HD_D T frame_dist2(const Frame<T> &f, const V3<T> &p, V3<T> *q) {
    V3<T> r = p - f.A;
    T x = dot(r, f.ex);
    T y = dot(r, f.ey);
    V3<T> n = cross(f.ex, f.ey);
    T z = dot(r, n);
    T xb = x - f.Lb;
    T bcx = f.cx - f.Lb;
    // planar edge functions of the counter-clockwise triangle (0,0),(Lb,0),(cx,cy)
    T eBC = bcx * y - f.cy * xb;
    T eCA = f.cy * x - f.cx * y;
    bool inside = (y >= T(0)) & (eBC >= T(0)) & (eCA >= T(0)) & (f.cy > T(0));
    // edge AB lies on the x axis from 0 to Lb
    T Xab = clampab(x, T(0), f.Lb);
    T dxa = x - Xab;
    T dAB = dxa * dxa + y * y;
    // edge CA from (0,0) to (cx,cy)
    T tca = clamp01((x * f.cx + y * f.cy) * f.inv2ca);
    T dxc = x - tca * f.cx, dyc = y - tca * f.cy;
    T dCA = dxc * dxc + dyc * dyc;
    // edge BC from (Lb,0) to (cx,cy)
    T tbc = clamp01((xb * bcx + y * f.cy) * f.inv2bc);
    T dxq = xb - tbc * bcx, dyq = y - tbc * f.cy;
    T dBC = dxq * dxq + dyq * dyq;
    T d2 = hmin(dAB, hmin(dCA, dBC));
    d2 = inside ? T(0) : d2;
    if constexpr (WANT_Q) {
        T X, Y;
        if (inside) {
            X = x;
            Y = y;
        } else if (dAB <= dCA && dAB <= dBC) {
            X = Xab;
            Y = T(0);
        } else if (dCA <= dBC) {
            X = tca * f.cx;
            Y = tca * f.cy;
        } else {
            X = f.Lb + tbc * bcx;
            Y = tbc * f.cy;
        }
        *q = f.A + X * f.ex + Y * f.ey;
    }
    return z * z + d2;
}

// Distance of the point x to the triangle s (sorted index) of B.
template <class T> struct BView;
template <> struct BView<float> {
    const float4 *frames;
};
template <> struct BView<double> {
    const double2 *frames;
};

template <class T> HD_D T dist_to(const BView<T> &b, int s, const V3<T> &x) {
    Frame<T> f = load_frame(b.frames, s);
    return hsqrt(frame_dist2<T, false>(f, x, nullptr));
}

// ---------------------------------------------------------------------------
// The bounds. A frontier triangle T has vertices v[i], distances d[i] to B,
// closest triangles S_i = I[i] (sorted index into B) and closest points q[i].
// All bounds below are computed without rounding margins; callers add them.
// ---------------------------------------------------------------------------

template <class T> struct Tri {
    V3<T> v[3];
    T d[3];
    int I[3];
    V3<T> q[3];
};

// eq. u1: the best vertex plus the longer of its two incident edges
template <class T> HD_D T bound_u1(const Tri<T> &t) {
    T e12 = hsqrt(norm2(t.v[0] - t.v[1]));
    T e23 = hsqrt(norm2(t.v[1] - t.v[2]));
    T e31 = hsqrt(norm2(t.v[2] - t.v[0]));
    T b1 = hmax(e12, e31) + t.d[0];
    T b2 = hmax(e12, e23) + t.d[1];
    T b3 = hmax(e23, e31) + t.d[2];
    return hmin(b1, hmin(b2, b3));
}

// g of eq. u2: circumradius if the triangle is acute (the paper's s - r > 2R
// test is the classical acute criterion), half the longest edge otherwise.
// Near-right triangles are sent to the circumradius branch, which is never
// smaller (R >= longest edge / 2 for every triangle). The area comes from the
// two shorter edges, which meet at the largest angle (>= 60 degrees), so it
// is accurate whenever R is used.
template <class T> HD_D T u2_g(const Tri<T> &t) {
    V3<T> e[3] = {t.v[1] - t.v[0], t.v[2] - t.v[1], t.v[0] - t.v[2]};
    T l2[3] = {norm2(e[0]), norm2(e[1]), norm2(e[2])};
    int k = 0;
    if (l2[1] > l2[k]) k = 1;
    if (l2[2] > l2[k]) k = 2;
    int a = (k + 1) % 3, b = (k + 2) % 3;
    const T lk = pick3(l2[0], l2[1], l2[2], k);
    T lmax = hsqrt(lk);
    const T slack = T(1) + T(8 * Prec<T>::u);
    if (lk < (pick3(l2[0], l2[1], l2[2], a) + pick3(l2[0], l2[1], l2[2], b)) * slack) {
        V3<T> c = cross(pick3(e[0], e[1], e[2], a), pick3(e[0], e[1], e[2], b));
        T twice_area = hsqrt(norm2(c));
        if (twice_area > T(0)) {
            T R = hsqrt(l2[0]) * hsqrt(l2[1]) * hsqrt(l2[2]) / (T(2) * twice_area);
            return hmax(R, T(0.5) * lmax);
        }
    }
    return T(0.5) * lmax;
}

template <class T> HD_D T bound_u2(const Tri<T> &t) {
    return u2_g(t) + hmax(t.d[0], hmax(t.d[1], t.d[2]));
}

// unit vector in the plane of triangle s (positions P[3] with vertex ids
// id[3]) perpendicular to the edge (a,b), pointing to the third vertex
template <class T>
HD_D bool inplane_dir(const V3<T> P[3], const int id[3], int ia, int ib, V3<T> &out) {
    bool ha = false, hb = false, hc = false;
    V3<T> pa = P[0], pb = P[0], pc = P[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (id[k] == ia && !ha) {
            ha = true;
            pa = P[k];
        } else if (id[k] == ib && !hb) {
            hb = true;
            pb = P[k];
        } else {
            hc = true;
            pc = P[k];
        }
    }
    if (!ha || !hb || !hc) return false;
    V3<T> e = pb - pa;
    V3<T> w = pc - pa;
    T ee = norm2(e);
    if (!(ee > T(0))) return false;
    V3<T> tt = w - (dot(w, e) / ee) * e;
    T tn = hsqrt(norm2(tt));
    if (!(tn > T(0))) return false;
    out = (T(1) / tn) * tt;
    return true;
}

struct IdView {
    const int4 *ids; // per sorted triangle: vertex ids of frame corners A, B, C; original face id
};

// Which case of Kang's bound applies to closest triangles I[0..2]: the
// first (eq. Kang2018_case1) when exactly two coincide and the odd vertex's
// triangle S1 shares an edge (vertex ids c0, c1) with the others' S2, else
// the second (eq. Kang2018_case2).
struct U3Case {
    int odd;        // the vertex whose closest triangle differs (-1: none)
    int S1, S2;     // its closest triangle and the other vertices'
    int a1[3], a2[3]; // vertex ids of S1 and S2 (frame order)
    int c0, c1;     // the first two distinct ids of S1 that S2 shares (-1: none)
    HD_D bool first() const { return odd >= 0 && c1 >= 0; }
};
HD_D U3Case u3_case(int I0, int I1, int I2, const IdView &iv) {
    U3Case u;
    u.odd = -1;
    if (I0 != I1 && I1 == I2) u.odd = 0;
    else if (I1 != I0 && I0 == I2) u.odd = 1;
    else if (I2 != I0 && I0 == I1) u.odd = 2;
    u.c0 = u.c1 = -1;
    if (u.odd < 0) return u;
    u.S1 = pick3(I0, I1, I2, u.odd);
    u.S2 = pick3(I0, I1, I2, (u.odd + 1) % 3);
    const int4 i1 = iv.ids[u.S1], i2 = iv.ids[u.S2];
    u.a1[0] = i1.x, u.a1[1] = i1.y, u.a1[2] = i1.z;
    u.a2[0] = i2.x, u.a2[1] = i2.y, u.a2[2] = i2.z;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const bool shared = u.a1[i] == u.a2[0] || u.a1[i] == u.a2[1] || u.a1[i] == u.a2[2];
        if (shared && u.c0 < 0) u.c0 = u.a1[i];
        else if (shared && u.c1 < 0 && u.a1[i] != u.c0) u.c1 = u.a1[i];
    }
    return u;
}

// eq. Kang2018_case1 / eq. Kang2018_case2. *evals counts closest-point
// evaluations.
template <class T>
HD_D T bound_u3(const Tri<T> &t, const BView<T> &bv, const IdView &iv, int *which_case, int *evals) {
    const U3Case u = u3_case(t.I[0], t.I[1], t.I[2], iv);
    if (u.odd >= 0) {
        // rotate so that the odd vertex comes first (selects, not indexing)
        const int odd = u.odd, r1 = (odd + 1) % 3, r2 = (odd + 2) % 3;
        const int S1 = u.S1, S2 = u.S2;
        const int a1[3] = {u.a1[0], u.a1[1], u.a1[2]}, a2[3] = {u.a2[0], u.a2[1], u.a2[2]};
        const int c0 = u.c0, c1 = u.c1;
        if (c1 >= 0) {
            if (which_case) *which_case = 1;
            Frame<T> f1 = load_frame(bv.frames, S1), f2 = load_frame(bv.frames, S2);
            V3<T> P1[3] = {frame_vertex(f1, 0), frame_vertex(f1, 1), frame_vertex(f1, 2)};
            V3<T> P2[3] = {frame_vertex(f2, 0), frame_vertex(f2, 1), frame_vertex(f2, 2)};
            const V3<T> v1 = pick3(t.v[0], t.v[1], t.v[2], odd), v2 = pick3(t.v[0], t.v[1], t.v[2], r1),
                        v3 = pick3(t.v[0], t.v[1], t.v[2], r2);
            const T d1 = pick3(t.d[0], t.d[1], t.d[2], odd), d2 = pick3(t.d[0], t.d[1], t.d[2], r1),
                    d3 = pick3(t.d[0], t.d[1], t.d[2], r2);
            V3<T> b1 = T(0.5) * (v1 + v2), b2 = T(0.5) * (v1 + v3);
            V3<T> t1, t2;
            if (inplane_dir(P1, a1, c0, c1, t1) && inplane_dir(P2, a2, c0, c1, t2)) {
                V3<T> nu = t1 - t2;
                if (norm2(nu) > T(0)) {
                    // a point of the shared edge: the corner of S1 with id c0
                    V3<T> ea = P1[0];
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        if (a1[k] == c0) ea = P1[k];
                    T f1v = dot(v1 - ea, nu), f2v = dot(v2 - ea, nu), f3v = dot(v3 - ea, nu);
                    if (f1v != f2v && f1v != f3v) {
                        T s12 = f1v / (f1v - f2v), s13 = f1v / (f1v - f3v);
                        if (s12 >= T(0) && s12 <= T(1) && s13 >= T(0) && s13 <= T(1)) {
                            b1 = v1 + s12 * (v2 - v1);
                            b2 = v1 + s13 * (v3 - v1);
                        }
                    }
                }
            }
            T hR = hmax(d1, hmax(hsqrt(frame_dist2<T, false>(f1, b1, nullptr)),
                                 hsqrt(frame_dist2<T, false>(f1, b2, nullptr))));
            T hQ = hmax(hmax(d2, d3),
                        hmax(hsqrt(frame_dist2<T, false>(f2, b1, nullptr)),
                             hsqrt(frame_dist2<T, false>(f2, b2, nullptr))));
            if (evals) *evals += 4;
            return hmax(hR, hQ);
        }
    }
    if (which_case) *which_case = 2;
    V3<T> m1 = T(0.5) * (t.v[0] + t.v[1]);
    V3<T> m2 = T(0.5) * (t.v[1] + t.v[2]);
    V3<T> m3 = T(0.5) * (t.v[2] + t.v[0]);
    V3<T> b = T(1.0 / 3.0) * (t.v[0] + t.v[1] + t.v[2]);
    // Q1 = (v1,m1,b,m3) to S1, Q2 = (v2,m2,b,m1) to S2, Q3 = (v3,m3,b,m2) to S3;
    // alongside, h(T, S_i): the largest distance of T's vertices to S_i. One
    // frame is live at a time.
    const V3<T> *corner[3][3] = {{&m1, &b, &m3}, {&m2, &b, &m1}, {&m3, &b, &m2}};
    T part = T(0), whole = __builtin_inf();
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const Frame<T> f = load_frame(bv.frames, t.I[i]);
        T hq = t.d[i], ht = t.d[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) hq = hmax(hq, hsqrt(frame_dist2<T, false>(f, *corner[i][k], nullptr)));
#pragma unroll
        for (int j = 0; j < 3; ++j)
            if (j != i) ht = hmax(ht, hsqrt(frame_dist2<T, false>(f, t.v[j], nullptr)));
        part = hmax(part, hq);
        whole = hmin(whole, ht);
    }
    const T best = hmin(part, whole);
    if (evals) *evals += 15;
    return best;
}

// h(T, {x, y}): maximum over the vertices of T and the crossings of T's
// edges with the bisector plane of x and y (eq. bound_u4 discussion).
template <class T> HD_D T h_two_points(const Tri<T> &t, const V3<T> &x, const V3<T> &y) {
    T h = T(0);
    for (int j = 0; j < 3; ++j)
        h = hmax(h, hmin(norm2(t.v[j] - x), norm2(t.v[j] - y)));
    V3<T> w = y - x;
    if (norm2(w) > T(0)) {
        V3<T> m = T(0.5) * (x + y);
        T f[3];
        for (int j = 0; j < 3; ++j) f[j] = dot(t.v[j] - m, w);
        for (int j = 0; j < 3; ++j) {
            int k = (j + 1) % 3;
            if (f[j] * f[k] < T(0)) {
                T s = f[j] / (f[j] - f[k]);
                V3<T> p = t.v[j] + s * (t.v[k] - t.v[j]);
                h = hmax(h, norm2(p - x));
            }
        }
    }
    return hsqrt(h);
}

// eq. bound_u4: q2, q3 are the footpoints of the shortest edge's endpoints
// (first edge among v1v2, v2v3, v3v1 on ties), q1 that of the other vertex
template <class T> HD_D T bound_u4(const Tri<T> &t) {
    T e[3] = {norm2(t.v[0] - t.v[1]), norm2(t.v[1] - t.v[2]), norm2(t.v[2] - t.v[0])};
    int s = 0;
    if (e[1] < e[s]) s = 1;
    if (e[2] < e[s]) s = 2;
    V3<T> qa = t.q[0], qb = t.q[1], qc = t.q[2];
    if (s == 1) { qa = t.q[1]; qb = t.q[2]; qc = t.q[0]; }
    if (s == 2) { qa = t.q[2]; qb = t.q[0]; qc = t.q[1]; }
    return hmin(h_two_points(t, qc, qa), h_two_points(t, qc, qb));
}

// The bound of Zheng et al. that the paper quotes in its fourth-bound
// subsection: min over S in {S1, S2, S3, S_b} of the largest distance of a
// vertex of T to S (the distance to a triangle is convex, so over T it peaks
// at a vertex); S_b is the triangle of B closest to T's barycenter (sorted
// index, found by a point query). Vertex i's distance to its own S_i is known.
// One frame is live at a time; *evals counts closest-point evaluations.
template <class T> HD_D T bound_u5(const Tri<T> &t, const BView<T> &bv, int Sb, int *evals) {
    T best = __builtin_inf();
    int ev = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int S = i < 3 ? pick3(t.I[0], t.I[1], t.I[2], i) : Sb;
        // a triangle already tried gives the same term
        if (i >= 1 && S == t.I[0]) continue;
        if (i >= 2 && S == t.I[1]) continue;
        if (i == 3 && S == t.I[2]) continue;
        const Frame<T> f = load_frame(bv.frames, S);
        T h = T(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            if (i < 3 && j == i) {
                h = hmax(h, pick3(t.d[0], t.d[1], t.d[2], j));
            } else {
                h = hmax(h, hsqrt(frame_dist2<T, false>(f, pick3(t.v[0], t.v[1], t.v[2], j), nullptr)));
                ++ev;
            }
        }
        best = hmin(best, h);
    }
    if (evals) *evals += ev;
    return best;
}

} // namespace hd
