// hd_bvh.hip -- device-built linear BVH over soup B.
//
// Morton codes of triangle centroids (30 bits), stable radix sort, the
// binary radix tree of Karras (HPG 2012) with duplicate keys split by index,
// and a bottom-up refit whose boxes are rounded outwards from the FP64
// triangles, so that they contain both the FP64 and the FP32 geometry. Each
// internal node stores the boxes of both children (64 B), so one load per
// visited node gives the two distances a closest-first traversal needs.
// Leaves are the triangles themselves, stored in Morton order as frame
// records (see hd_geom.hpp) in FP32 and FP64.
#include "hd_geom.hpp"
#include "hd_internal.hpp"

namespace hd {

namespace {

constexpr int BLK = 256;

__device__ __forceinline__ float round_down_f(double x) {
    float f = (float)x;
    if ((double)f > x) f = next_down(f);
    return f;
}
__device__ __forceinline__ float round_up_f(double x) {
    float f = (float)x;
    if ((double)f < x) f = next_up(f);
    return f;
}

__device__ __forceinline__ void atomic_min_d(unsigned long long *a, double v) { atomicMin(a, d2ord(v)); }
__device__ __forceinline__ void atomic_max_d(unsigned long long *a, double v) { atomicMax(a, d2ord(v)); }

struct BuildState {
    unsigned long long bbox[6];  // ordered FP64 lo xyz, hi xyz of B's vertices
    unsigned long long cbox[6];  // ordered FP64 lo/hi of centroids (centred)
    unsigned long long coord_max, edge_max;
    int bad;
};

__global__ void k_init_state(BuildState *st) {
    for (int k = 0; k < 3; ++k) {
        st->bbox[k] = d2ord(__builtin_inf());
        st->bbox[3 + k] = d2ord(-__builtin_inf());
        st->cbox[k] = d2ord(__builtin_inf());
        st->cbox[3 + k] = d2ord(-__builtin_inf());
    }
    st->coord_max = d2ord(0.0);
    st->edge_max = d2ord(0.0);
    st->bad = 0;
}

// validate faces; bbox of referenced vertices (through the faces)
__global__ void k_faces_check(const double *__restrict__ V, int64_t m, const int32_t *__restrict__ F,
                              int64_t n, BuildState *st) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    for (int j = 0; j < 3; ++j) {
        int32_t v = F[3 * f + j];
        if (v < 0 || v >= m) {
            st->bad = 1;
            return;
        }
        for (int k = 0; k < 3; ++k) {
            double x = V[3 * (int64_t)v + k];
            if (!__builtin_isfinite(x)) {
                st->bad = 1;
                return;
            }
            lo[k] = fmin(lo[k], x);
            hi[k] = fmax(hi[k], x);
        }
    }
    for (int k = 0; k < 3; ++k) {
        atomic_min_d(&st->bbox[k], lo[k]);
        atomic_max_d(&st->bbox[3 + k], hi[k]);
    }
}

__global__ void k_centroids(const double *__restrict__ V, const int32_t *__restrict__ F, int64_t n,
                            double cx, double cy, double cz, double *__restrict__ cen, BuildState *st) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    double c[3] = {0, 0, 0};
    double m = 0;
    const double ctr[3] = {cx, cy, cz};
    for (int j = 0; j < 3; ++j) {
        int32_t v = F[3 * f + j];
        for (int k = 0; k < 3; ++k) {
            double x = V[3 * (int64_t)v + k] - ctr[k];
            c[k] += x;
            m = fmax(m, fabs(x));
        }
    }
    for (int k = 0; k < 3; ++k) {
        c[k] /= 3.0;
        cen[3 * f + k] = c[k];
        atomic_min_d(&st->cbox[k], c[k]);
        atomic_max_d(&st->cbox[3 + k], c[k]);
    }
    atomic_max_d(&st->coord_max, m);
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__global__ void k_morton(const double *__restrict__ cen, int64_t n, const BuildState *st,
                         uint32_t *__restrict__ keys, int32_t *__restrict__ vals) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
        double lo = ord2d(st->cbox[k]), hi = ord2d(st->cbox[3 + k]);
        double ext = hi - lo;
        double t = ext > 0 ? (cen[3 * f + k] - lo) / ext : 0.5;
        int v = (int)(t * 1023.0);
        q[k] = (uint32_t)(v < 0 ? 0 : (v > 1023 ? 1023 : v));
    }
    keys[f] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    vals[f] = (int32_t)f;
}

__device__ __forceinline__ int delta(const uint32_t *__restrict__ keys, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    uint32_t a = keys[i], b = keys[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

// Karras 2012, one thread per internal node i in [0, n-2]
__global__ void k_karras(const uint32_t *__restrict__ keys, int64_t n, int32_t *__restrict__ childL,
                         int32_t *__restrict__ childR, int32_t *__restrict__ parentN,
                         int32_t *__restrict__ parentL) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = (delta(keys, n, i, i + 1) - delta(keys, n, i, i - 1)) >= 0 ? 1 : -1;
    int dmin = delta(keys, n, i, i - d);
    int64_t lmax = 2;
    while (delta(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int64_t j = i + l * d;
    int dnode = delta(keys, n, i, j);
    int64_t s = 0;
    int64_t t = l;
    do {
        t = (t + 1) >> 1;
        if (delta(keys, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    int32_t cl, cr;
    if (lo == gamma) {
        cl = ~(int32_t)gamma;
        parentL[gamma] = (int32_t)i;
    } else {
        cl = (int32_t)gamma;
        parentN[gamma] = (int32_t)i;
    }
    if (hi == gamma + 1) {
        cr = ~(int32_t)(gamma + 1);
        parentL[gamma + 1] = (int32_t)i;
    } else {
        cr = (int32_t)(gamma + 1);
        parentN[gamma + 1] = (int32_t)i;
    }
    childL[i] = cl;
    childR[i] = cr;
}

// leaf data in sorted order: outward-rounded box, frame records, ids
__global__ void k_leaves(const double *__restrict__ V, const int32_t *__restrict__ F,
                         const int32_t *__restrict__ order, int64_t n, double ccx, double ccy,
                         double ccz, float4 *__restrict__ lbox, float4 *__restrict__ fr32,
                         double2 *__restrict__ fr64, int4 *__restrict__ ids, BuildState *st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t f = order[i];
    const double ctr[3] = {ccx, ccy, ccz};
    int32_t vid[3];
    V3<double> P[3];
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    for (int j = 0; j < 3; ++j) {
        vid[j] = F[3 * (int64_t)f + j];
        double c[3];
        for (int k = 0; k < 3; ++k) {
            c[k] = V[3 * (int64_t)vid[j] + k] - ctr[k];
            lo[k] = fmin(lo[k], c[k]);
            hi[k] = fmax(hi[k], c[k]);
        }
        P[j] = {c[0], c[1], c[2]};
    }
    lbox[2 * i] = make_float4(round_down_f(lo[0]), round_down_f(lo[1]), round_down_f(lo[2]), 0.f);
    lbox[2 * i + 1] = make_float4(round_up_f(hi[0]), round_up_f(hi[1]), round_up_f(hi[2]), 0.f);

    // frame anchored on the longest edge (P[k], P[k+1])
    double l2[3] = {norm2(P[1] - P[0]), norm2(P[2] - P[1]), norm2(P[0] - P[2])};
    int k = 0;
    if (l2[1] > l2[k]) k = 1;
    if (l2[2] > l2[k]) k = 2;
    V3<double> A = P[k], B = P[(k + 1) % 3], C = P[(k + 2) % 3];
    V3<double> e = B - A;
    double Lb = sqrt(norm2(e));
    V3<double> ex = Lb > 0 ? (1.0 / Lb) * e : mk(1.0, 0.0, 0.0);
    V3<double> fv = C - A;
    double cx = dot(fv, ex);
    V3<double> g = fv - cx * ex;
    double cy = sqrt(norm2(g));
    V3<double> ey;
    if (cy > 0) {
        ey = (1.0 / cy) * g;
    } else {
        // any unit vector perpendicular to ex
        V3<double> ax = fabs(ex.x) <= fabs(ex.y) && fabs(ex.x) <= fabs(ex.z) ? mk(1.0, 0.0, 0.0)
                        : (fabs(ex.y) <= fabs(ex.z) ? mk(0.0, 1.0, 0.0) : mk(0.0, 0.0, 1.0));
        V3<double> t = cross(ex, ax);
        ey = (1.0 / sqrt(norm2(t))) * t;
        cy = 0;
    }
    double bcx = cx - Lb;
    double nbc = bcx * bcx + cy * cy, nca = cx * cx + cy * cy;
    double ibc = nbc > 0 ? 1.0 / nbc : 0.0, ica = nca > 0 ? 1.0 / nca : 0.0;
    fr32[4 * i] = make_float4((float)A.x, (float)A.y, (float)A.z, (float)Lb);
    fr32[4 * i + 1] = make_float4((float)ex.x, (float)ex.y, (float)ex.z, (float)cx);
    fr32[4 * i + 2] = make_float4((float)ey.x, (float)ey.y, (float)ey.z, (float)cy);
    fr32[4 * i + 3] = make_float4((float)ibc, (float)ica, (float)Lb, 0.f);
    double2 *p = fr64 + 8 * i;
    p[0] = make_double2(A.x, A.y);
    p[1] = make_double2(A.z, Lb);
    p[2] = make_double2(ex.x, ex.y);
    p[3] = make_double2(ex.z, cx);
    p[4] = make_double2(ey.x, ey.y);
    p[5] = make_double2(ey.z, cy);
    p[6] = make_double2(ibc, ica);
    p[7] = make_double2(Lb, 0.0);
    ids[i] = make_int4(vid[k], vid[(k + 1) % 3], vid[(k + 2) % 3], f);
    atomic_max_d(&st->edge_max, Lb);
}

__device__ __forceinline__ void load_box(const float4 *__restrict__ nbox, const float4 *__restrict__ lbox,
                                         int32_t c, float4 &lo, float4 &hi) {
    if (c >= 0) {
        lo = nbox[2 * (int64_t)c];
        hi = nbox[2 * (int64_t)c + 1];
    } else {
        lo = lbox[2 * (int64_t)(~c)];
        hi = lbox[2 * (int64_t)(~c) + 1];
    }
}

// bottom-up union of child boxes; the second thread to reach a node builds it
__global__ void k_refit(int64_t n, const int32_t *__restrict__ childL, const int32_t *__restrict__ childR,
                        const int32_t *__restrict__ parentN, const int32_t *__restrict__ parentL,
                        const float4 *__restrict__ lbox, float4 *nbox, int32_t *counter) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t p = parentL[i];
    while (p >= 0) {
        int old = __hip_atomic_fetch_add(&counter[p], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (old == 0) return;
        float4 l0, h0, l1, h1;
        load_box(nbox, lbox, childL[p], l0, h0);
        load_box(nbox, lbox, childR[p], l1, h1);
        nbox[2 * (int64_t)p] = make_float4(fminf(l0.x, l1.x), fminf(l0.y, l1.y), fminf(l0.z, l1.z), 0.f);
        nbox[2 * (int64_t)p + 1] = make_float4(fmaxf(h0.x, h1.x), fmaxf(h0.y, h1.y), fmaxf(h0.z, h1.z), 0.f);
        if (p == 0) return;
        p = parentN[p];
    }
}

__global__ void k_node_records(int64_t ninternal, const int32_t *__restrict__ childL,
                               const int32_t *__restrict__ childR, const float4 *__restrict__ nbox,
                               const float4 *__restrict__ lbox, NodeRec *__restrict__ out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ninternal) return;
    int32_t cl = childL[i], cr = childR[i];
    float4 l0, h0, l1, h1;
    load_box(nbox, lbox, cl, l0, h0);
    load_box(nbox, lbox, cr, l1, h1);
    NodeRec r;
    r.a = make_float4(l0.x, l0.y, l0.z, __builtin_bit_cast(float, cl));
    r.b = make_float4(h0.x, h0.y, h0.z, __builtin_bit_cast(float, cr));
    r.c = make_float4(l1.x, l1.y, l1.z, 0.f);
    r.d = make_float4(h1.x, h1.y, h1.z, 0.f);
    out[i] = r;
}

// a one-triangle soup: a root whose two children are the single leaf
__global__ void k_single_root(const float4 *__restrict__ lbox, NodeRec *out) {
    float4 lo = lbox[0], hi = lbox[1];
    NodeRec r;
    int32_t c = ~0;
    r.a = make_float4(lo.x, lo.y, lo.z, __builtin_bit_cast(float, c));
    r.b = make_float4(hi.x, hi.y, hi.z, __builtin_bit_cast(float, c));
    r.c = make_float4(lo.x, lo.y, lo.z, 0.f);
    r.d = make_float4(hi.x, hi.y, hi.z, 0.f);
    out[0] = r;
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

} // namespace

Bvh *build_bvh(const double *VB, int64_t mB, const int32_t *FB, int64_t nB, hipStream_t s) {
    if (nB <= 0 || mB <= 0 || !VB || !FB) throw Error{HD_E_INVALID, "empty soup B"};
    if (nB >= (int64_t(1) << 30)) throw Error{HD_E_INVALID, "soup B too large (>= 2^30 faces)"};
    Bvh *b = new Bvh();
    try {
        HD_HIP(hipGetDevice(&b->device));
        b->nB = nB;
        b->mB = mB;
        hipEvent_t e0, e1;
        HD_HIP(hipEventCreate(&e0));
        HD_HIP(hipEventCreate(&e1));
        HD_HIP(hipEventRecord(e0, s));
        const int64_t n = nB;
        const int64_t ni = n > 1 ? n - 1 : 1;
        // scratch layout
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off += (bytes + 255) & ~size_t(255);
            return o;
        };
        size_t o_state = take(sizeof(BuildState));
        size_t o_cen = take(n * 3 * sizeof(double));
        size_t o_keys = take(n * sizeof(uint32_t));
        size_t o_vals = take(n * sizeof(int32_t));
        size_t o_keys2 = take(n * sizeof(uint32_t));
        size_t o_vals2 = take(n * sizeof(int32_t));
        size_t o_cl = take(ni * sizeof(int32_t));
        size_t o_cr = take(ni * sizeof(int32_t));
        size_t o_pn = take(ni * sizeof(int32_t));
        size_t o_pl = take(n * sizeof(int32_t));
        size_t o_cnt = take(ni * sizeof(int32_t));
        size_t o_lbox = take(n * 2 * sizeof(float4));
        size_t o_nbox = take(ni * 2 * sizeof(float4));
        b->scratch.reserve(off);
        char *base = b->scratch.as<char>();
        BuildState *st = (BuildState *)(base + o_state);
        double *cen = (double *)(base + o_cen);
        uint32_t *keys = (uint32_t *)(base + o_keys);
        int32_t *vals = (int32_t *)(base + o_vals);
        uint32_t *keys2 = (uint32_t *)(base + o_keys2);
        int32_t *vals2 = (int32_t *)(base + o_vals2);
        int32_t *cl = (int32_t *)(base + o_cl);
        int32_t *cr = (int32_t *)(base + o_cr);
        int32_t *pn = (int32_t *)(base + o_pn);
        int32_t *pl = (int32_t *)(base + o_pl);
        int32_t *cnt = (int32_t *)(base + o_cnt);
        float4 *lbox = (float4 *)(base + o_lbox);
        float4 *nbox = (float4 *)(base + o_nbox);

        k_init_state<<<1, 1, 0, s>>>(st);
        k_faces_check<<<grid_for(n, BLK), BLK, 0, s>>>(VB, mB, FB, n, st);
        HD_LAUNCH_CHECK();
        BuildState hs;
        HD_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        HD_HIP(hipStreamSynchronize(s));
        if (hs.bad) throw Error{HD_E_INVALID, "soup B has an out-of-range index or a non-finite coordinate"};
        for (int k = 0; k < 3; ++k) b->center[k] = 0.5 * (ord2d(hs.bbox[k]) + ord2d(hs.bbox[3 + k]));

        k_centroids<<<grid_for(n, BLK), BLK, 0, s>>>(VB, FB, n, b->center[0], b->center[1], b->center[2],
                                                     cen, st);
        k_morton<<<grid_for(n, BLK), BLK, 0, s>>>(cen, n, st, keys, vals);
        HD_LAUNCH_CHECK();
        DBuf sort_tmp;
        radix_sort_u32(keys, vals, keys2, vals2, n, 30, sort_tmp, s);

        b->nodes.reserve(ni * sizeof(NodeRec));
        b->frames32.reserve(n * 4 * sizeof(float4));
        b->frames64.reserve(n * 8 * sizeof(double2));
        b->ids.reserve(n * sizeof(int4));
        k_leaves<<<grid_for(n, BLK), BLK, 0, s>>>(VB, FB, vals, n, b->center[0], b->center[1], b->center[2],
                                                  lbox, b->frames32.as<float4>(), b->frames64.as<double2>(),
                                                  b->ids.as<int4>(), st);
        HD_LAUNCH_CHECK();
        if (n == 1) {
            k_single_root<<<1, 1, 0, s>>>(lbox, b->nodes.as<NodeRec>());
        } else {
            k_fill_i32<<<grid_for(ni, BLK), BLK, 0, s>>>(pn, ni, -1);
            k_fill_i32<<<grid_for(n, BLK), BLK, 0, s>>>(pl, n, -1);
            k_fill_i32<<<grid_for(ni, BLK), BLK, 0, s>>>(cnt, ni, 0);
            k_karras<<<grid_for(ni, BLK), BLK, 0, s>>>(keys, n, cl, cr, pn, pl);
            k_refit<<<grid_for(n, BLK), BLK, 0, s>>>(n, cl, cr, pn, pl, lbox, nbox, cnt);
            k_node_records<<<grid_for(ni, BLK), BLK, 0, s>>>(ni, cl, cr, nbox, lbox, b->nodes.as<NodeRec>());
        }
        HD_LAUNCH_CHECK();
        HD_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        HD_HIP(hipEventRecord(e1, s));
        HD_HIP(hipStreamSynchronize(s));
        b->coord_max = ord2d(hs.coord_max);
        b->edge_max = ord2d(hs.edge_max);
        HD_HIP(hipEventElapsedTime(&b->ms_build, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->scratch.release();
        return b;
    } catch (...) {
        delete b;
        throw;
    }
}

} // namespace hd
