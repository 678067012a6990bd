// hd_learned.hpp -- inputs of the learned proposal: the 16 features of a
// frontier triangle. The proposal is not part of the paper's method; it only
// orders work and decides whether the third and fourth bounds are worth
// evaluating. Every discard and every certificate still comes from the
// rigorous bounds.
//
// Features (longest edge l; ratios through asinh so that deep levels stay in
// range): the three vertex distances sorted ascending / l; shortest and middle
// edge / l; twice the area / l^2; (max d - L) / l; (u1 - L) / l; (u2 - L) / l
// (both without margins); (distinct closest triangles - 1) / 2; 1 if exactly
// two distinct closest triangles share an edge; |cos| between the triangle's
// normal and each closest triangle's normal, in the order of the sorted
// distances; max |q_i - q_j| / l; log2(l / dA) / 30.
#pragma once
#include "hd_geom.hpp"

namespace hd {

template <class T> HD_D T vlen(const V3<T> &a) { return hsqrt(norm2(a)); }

// unit normal of a B triangle from its frame (ex and ey are orthonormal)
template <class T> HD_D V3<T> frame_normal(const Frame<T> &f) { return cross(f.ex, f.ey); }

template <class T>
HD_D void tri_features(const Tri<T> &t, double L, double dA, const BView<T> &bv, const IdView &iv, float out[16]) {
    const T e0 = vlen(t.v[1] - t.v[0]), e1 = vlen(t.v[2] - t.v[1]), e2 = vlen(t.v[0] - t.v[2]);
    // sorted edges
    T s0 = e0, s1 = e1, s2 = e2;
    if (s0 > s1) { T x = s0; s0 = s1; s1 = x; }
    if (s1 > s2) { T x = s1; s1 = s2; s2 = x; }
    if (s0 > s1) { T x = s0; s0 = s1; s1 = x; }
    T ell = s2;
    if (!(ell > T(0))) ell = T(1e-30);
    const T il = T(1) / ell;
    // distances sorted ascending (stable), with the vertex each came from
    T d0 = t.d[0], d1 = t.d[1], d2 = t.d[2];
    int i0 = 0, i1 = 1, i2 = 2;
    if (d0 > d1) { T x = d0; d0 = d1; d1 = x; int k = i0; i0 = i1; i1 = k; }
    if (d1 > d2) { T x = d1; d1 = d2; d2 = x; int k = i1; i1 = i2; i2 = k; }
    if (d0 > d1) { T x = d0; d0 = d1; d1 = x; int k = i0; i0 = i1; i1 = k; }
    const T dmax = d2;
    // normals
    const V3<T> nT = cross(t.v[1] - t.v[0], t.v[2] - t.v[0]);
    const T area2 = vlen(nT);
    const V3<T> nTu = area2 > T(0) ? (T(1) / area2) * nT : V3<T>{T(0), T(0), T(0)};
    T cs[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const V3<T> nS = frame_normal(load_frame(bv.frames, t.I[k]));
        const T c = dot(nS, nTu);
        cs[k] = c < T(0) ? -c : c;
    }
    const T c0 = pick3(cs[0], cs[1], cs[2], i0), c1 = pick3(cs[0], cs[1], cs[2], i1),
            c2 = pick3(cs[0], cs[1], cs[2], i2);
    // the two cheap bounds without margins
    const T u1 = hmin(hmax(e0, e2) + t.d[0], hmin(hmax(e0, e1) + t.d[1], hmax(e1, e2) + t.d[2]));
    const bool acute = s2 * s2 < s0 * s0 + s1 * s1;
    T g = T(0.5) * ell;
    if (acute && area2 > T(0)) g = hmax(e0 * e1 * e2 / (T(2) * area2), g);
    const T u2 = g + dmax;
    // closest triangles: distinct count, shared edge
    const int I0 = t.I[0], I1 = t.I[1], I2 = t.I[2];
    const int distinct = 1 + (I1 != I0) + (I2 != I0 && I2 != I1);
    float shared = 0.f;
    if (distinct == 2) {
        const int a = I0, b = I1 != I0 ? I1 : I2;
        const int4 A = iv.ids[a], B = iv.ids[b];
        const int n = (A.x == B.x || A.x == B.y || A.x == B.z) + (A.y == B.x || A.y == B.y || A.y == B.z) +
                      (A.z == B.x || A.z == B.y || A.z == B.z);
        shared = n >= 2 ? 1.f : 0.f;
    }
    const T qd = hmax(vlen(t.q[0] - t.q[1]), hmax(vlen(t.q[1] - t.q[2]), vlen(t.q[2] - t.q[0])));
    const float fl = (float)ell;
    out[0] = asinhf((float)(d0 * il));
    out[1] = asinhf((float)(d1 * il));
    out[2] = asinhf((float)(d2 * il));
    out[3] = (float)(s0 * il);
    out[4] = (float)(s1 * il);
    out[5] = (float)(area2 * il * il);
    out[6] = asinhf((float)(((double)dmax - L) / (double)fl));
    out[7] = asinhf((float)(((double)u1 - L) / (double)fl));
    out[8] = asinhf((float)(((double)u2 - L) / (double)fl));
    out[9] = 0.5f * (float)(distinct - 1);
    out[10] = shared;
    out[11] = (float)c0;
    out[12] = (float)c1;
    out[13] = (float)c2;
    out[14] = asinhf((float)(qd * il));
    out[15] = log2f((float)((double)ell / dA)) / 30.f;
}

} // namespace hd
