// hd_bvh.hip -- device-built linear BVH over one or more soups B_p.
//
// Keys are (pair id << 32 | 30-bit Morton code of the centroid, normalised to
// the pair's own centroid box), sorted by a stable radix sort. The binary
// radix tree of Karras (HPG 2012) over the sorted keys, with duplicate keys
// split by index, then contains one subtree per pair; a pair's traversal
// starts at its subtree root. Boxes are rounded outwards from the FP64
// triangles (in the pair's centred coordinates), so they contain both the
// FP64 and the FP32 geometry. Each internal node stores the boxes of both
// children (64 B), so one load per visited node gives both distances of a
// closest-first traversal. Leaves are the triangles, stored in sorted order
// as frame records (hd_geom.hpp) in FP32 and FP64.
//
// The refit avoids device-scope synchronisation, which on a multi-XCD part
// costs an L2 write-back and invalidate per step, and any serial chain over
// the tree's height: nodes whose leaf range lies inside one 256-leaf tile are
// refit by that tile's workgroup (a bottom-up climb in LDS); every node above
// the tiles takes its box directly as the union of its leaf range, from
// prefix / suffix unions within tiles and groups of tiles and a disjoint
// sparse table over the tiles of a group (a few loads per node).
#include <atomic>
#include <memory>
#include <mutex>

#include "hd_geom.hpp"
#include "hd_internal.hpp"
#include "hd_reduce.hpp"

namespace hd {

namespace {

constexpr int BLK = 256;
constexpr int TILE = 256; // refit tile = refit workgroup

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

struct PairAcc { // per-pair accumulators, ordered-double bits
    unsigned long long bbox[6];
    unsigned long long coord_max, edge_max;
};
// The accumulators come in ACC_COPIES copies of npairs entries each, astride
// entries (a multiple of 256 bytes) apart; a block updates copy
// blockIdx % ACC_COPIES, and the kernel that reads a value folds the copies.
__device__ __forceinline__ PairAcc &acc_of(PairAcc *acc, int astride, int p) {
    return acc[(int64_t)acc_copy() * astride + p];
}

struct BuildState {
    int bad;
};

__global__ void k_init(PairAcc *acc, int npairs, int astride, BuildState *st) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        st->bad = 0;
    }
    if (i >= npairs * ACC_COPIES) return;
    PairAcc &a = acc[(int64_t)(i / npairs) * astride + i % npairs];
    for (int k = 0; k < 3; ++k) {
        a.bbox[k] = d2ord(__builtin_inf());
        a.bbox[3 + k] = d2ord(-__builtin_inf());
    }
    a.coord_max = d2ord(0.0);
    a.edge_max = d2ord(0.0);
}

// pair of a global face index (faces of pair p are [foff[p], foff[p+1]))
__device__ __forceinline__ int pair_of(const int64_t *__restrict__ foff, int npairs, int64_t f) {
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (foff[mid] <= f) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// one pair's device pointers
struct PairSrc {
    const double *V;
    const int32_t *F;
    int64_t m;
};

// validate faces and compute each pair's vertex box (through its faces).
// Every lane of a launched wave takes part (inactive lanes carry neutral
// values) so that the wave-wide reductions see 64 lanes. With several pairs
// the grid covers the faces (one each); with one pair it is capped
// (ONE_PAIR_GRID blocks) and every thread folds a grid-stride run of faces, so
// that fewer blocks end in the per-pair atomics.
constexpr unsigned ONE_PAIR_GRID = 1024;
inline unsigned face_grid(int64_t n, int npairs) {
    const unsigned g = grid_for(n, BLK);
    return npairs == 1 ? std::min(g, ONE_PAIR_GRID) : g;
}
__global__ void k_faces_check(const PairSrc *__restrict__ src, const int64_t *__restrict__ foff, int npairs,
                              int64_t n, PairAcc *acc, int astride, BuildState *st) {
    const int64_t f0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = f0 < n;
    const int p = pair_of(foff, npairs, valid ? f0 : n - 1); // every face of the thread's run (one pair)
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    for (int64_t f = f0; f < n; f += (int64_t)gridDim.x * blockDim.x) {
        PairSrc ps = src[p];
        int64_t lf = f - foff[p];
        for (int j = 0; j < 3; ++j) {
            int32_t v = ps.F[3 * lf + j];
            if (v < 0 || v >= ps.m) {
                st->bad = 1;
                continue;
            }
            for (int k = 0; k < 3; ++k) {
                double x = ps.V[3 * (int64_t)v + k];
                if (!__builtin_isfinite(x)) {
                    st->bad = 1;
                    continue;
                }
                lo[k] = fmin(lo[k], x);
                hi[k] = fmax(hi[k], x);
            }
        }
    }
    const double v[6] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
    block_pair_minmax<6, 0x38u, BLK>(p, valid, v, [&](int q, int k) { return &acc_of(acc, astride, q).bbox[k]; });
}

// value k of pair p's box (0..2 lower, 3..5 upper), folded over the copies
__device__ unsigned long long fold_box(const PairAcc *acc, int astride, int p, int k) {
    unsigned long long b = acc[p].bbox[k];
    for (int c = 1; c < ACC_COPIES; ++c) {
        const unsigned long long x = acc[(int64_t)c * astride + p].bbox[k];
        b = k < 3 ? (x < b ? x : b) : (x > b ? x : b);
    }
    return b;
}

__device__ __forceinline__ uint32_t spread10(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000FFu;
    x = (x | (x << 8)) & 0x0300F00Fu;
    x = (x | (x << 4)) & 0x030C30C3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Centroid of each face (centred on its pair) and its key: the pair id above
// a 30-bit Morton code of the centroid on a 1024^3 grid over the pair's vertex
// box (centroids lie inside it). Also the pair's largest centred coordinate,
// and its centre (the box midpoint, written by the thread of its first face).
// A block folds the box copies of its pairs in LDS (when it spans few pairs;
// else every thread folds its own pair's).
constexpr int CENTRE_PAIRS = 8;
__global__ __launch_bounds__(BLK) void k_centroids(const PairSrc *__restrict__ src,
                                                   const int64_t *__restrict__ foff, int npairs, int64_t n,
                                                   BvhPair *__restrict__ pairs, int32_t *__restrict__ fpair,
                                                   PairAcc *acc, int astride, const BuildState *st,
                                                   unsigned long long *__restrict__ keys,
                                                   int32_t *__restrict__ vals) {
    __shared__ double s_box[CENTRE_PAIRS][6];
    const int64_t fs = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool bad = st->bad != 0;
    const bool valid = fs < n && !bad;
    // the pair of every face of the thread's run (one face per thread with
    // several pairs; a grid-stride run with one)
    const int p = pair_of(foff, npairs, fs < n ? fs : n - 1);
    const int64_t f0 = (int64_t)blockIdx.x * blockDim.x, f1 = std::min<int64_t>(f0 + blockDim.x, n) - 1;
    const int pa = pair_of(foff, npairs, f0), pb = pair_of(foff, npairs, f1);
    const bool in_lds = pb - pa < CENTRE_PAIRS;
    if (in_lds && (int)threadIdx.x < (pb - pa + 1) * 6)
        s_box[threadIdx.x / 6][threadIdx.x % 6] = ord2d(fold_box(acc, astride, pa + threadIdx.x / 6, threadIdx.x % 6));
    __syncthreads();
    double box[6];
    for (int k = 0; k < 6; ++k) box[k] = in_lds ? s_box[p - pa][k] : ord2d(fold_box(acc, astride, p, k));
    const double ctr[3] = {0.5 * (box[0] + box[3]), 0.5 * (box[1] + box[4]), 0.5 * (box[2] + box[5])};
    double m = 0;
    for (int64_t f = fs; f < n; f += (int64_t)gridDim.x * blockDim.x) {
    if (f == foff[p])
        for (int k = 0; k < 3; ++k) pairs[p].ctr[k] = ctr[k];
    if (!bad) {
        PairSrc ps = src[p];
        int64_t lf = f - foff[p];
        double c[3] = {0, 0, 0};
        for (int j = 0; j < 3; ++j) {
            int32_t v = ps.F[3 * lf + j];
            for (int k = 0; k < 3; ++k) {
                double x = ps.V[3 * (int64_t)v + k] - ctr[k];
                c[k] += x;
                m = fmax(m, fabs(x));
            }
        }
        uint32_t q[3];
        for (int k = 0; k < 3; ++k) {
            const double lo = box[k] - ctr[k], hi = box[3 + k] - ctr[k];
            const double ext = hi - lo;
            double t = ext > 0 ? (c[k] / 3.0 - lo) / ext : 0.5;
            t = t == t ? t : 0.5;
            int v = (int)(t * 1023.0);
            q[k] = (uint32_t)(v < 0 ? 0 : (v > 1023 ? 1023 : v));
        }
        keys[f] = ((unsigned long long)p << 32) | ((spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]));
        vals[f] = (int32_t)f;
    } else {
        keys[f] = (unsigned long long)p << 32;
        vals[f] = (int32_t)f;
    }
    fpair[f] = p;
    }
    const double v[1] = {m};
    block_pair_minmax<1, 1u, BLK>(p, valid, v, [&](int q, int) { return &acc_of(acc, astride, q).coord_max; });
}

__device__ __forceinline__ int delta(const unsigned long long *__restrict__ keys, int64_t n, int64_t i, int64_t j) {
    if (j < 0 || j >= n) return -1;
    unsigned long long a = keys[i], b = keys[j];
    if (a == b) return 64 + __clz((uint32_t)(i ^ j));
    return __clzll(a ^ b);
}

// Karras 2012, internal node i in [0, n-2]; also the node's leaf range
__device__ void karras_node(const unsigned long long *__restrict__ keys, int64_t n, int32_t *__restrict__ childL,
                            int32_t *__restrict__ childR, int32_t *__restrict__ parentN,
                            int32_t *__restrict__ parentL, int2 *__restrict__ range, int64_t i) {
    if (i == 0) parentN[0] = -1; // the root (every other node is some node's child)
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
    range[i] = make_int2((int)lo, (int)hi);
}

// leaf data in sorted order: outward-rounded box, frame records, ids; the
// longest edge of each pair
__device__ double build_leaf(const PairSrc *__restrict__ src, const int64_t *__restrict__ foff, int p, int32_t f,
                             const BvhPair *__restrict__ pairs, float4 *__restrict__ lbox, float4 *__restrict__ fr32,
                             double2 *__restrict__ fr64, int4 *__restrict__ ids, int64_t i);

// After the sort, thread i: leaf i (frames, box, ids) and internal node i
// of the hierarchy (karras_node); both read only the sorted keys and order.
__global__ __launch_bounds__(BLK) void k_leaves(const PairSrc *__restrict__ src, const int64_t *__restrict__ foff,
                                                const int32_t *__restrict__ fpair, const int32_t *__restrict__ order,
                                                int64_t n, const BvhPair *__restrict__ pairs, float4 *__restrict__ lbox,
                                                float4 *__restrict__ fr32, double2 *__restrict__ fr64,
                                                int4 *__restrict__ ids, PairAcc *acc, int astride,
                                                const BuildState *st, const unsigned long long *__restrict__ keys,
                                                int32_t *__restrict__ childL, int32_t *__restrict__ childR,
                                                int32_t *__restrict__ parentN, int32_t *__restrict__ parentL,
                                                int2 *__restrict__ range) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) karras_node(keys, n, childL, childR, parentN, parentL, range, i);
    const bool valid = i < n && !st->bad;
    int p = 0;
    double Lb = 0;
    if (valid) {
        int32_t f = order[i];
        p = fpair[f];
        Lb = build_leaf(src, foff, p, f, pairs, lbox, fr32, fr64, ids, i);
    }
    const double v[1] = {Lb};
    block_pair_minmax<1, 1u, BLK>(p, valid, v, [&](int q, int) { return &acc_of(acc, astride, q).edge_max; });
}

__device__ double build_leaf(const PairSrc *__restrict__ src, const int64_t *__restrict__ foff, int p, int32_t f,
                             const BvhPair *__restrict__ pairs, float4 *__restrict__ lbox, float4 *__restrict__ fr32,
                             double2 *__restrict__ fr64, int4 *__restrict__ ids, int64_t i) {
    PairSrc ps = src[p];
    int64_t lf = f - foff[p];
    // (no runtime-indexed private arrays here: they would be promoted to LDS)
    const int32_t v0 = ps.F[3 * lf], v1 = ps.F[3 * lf + 1], v2 = ps.F[3 * lf + 2];
    const double *c = pairs[p].ctr;
    auto load = [&](int32_t v) {
        return mk(ps.V[3 * (int64_t)v] - c[0], ps.V[3 * (int64_t)v + 1] - c[1], ps.V[3 * (int64_t)v + 2] - c[2]);
    };
    const V3<double> P0 = load(v0), P1 = load(v1), P2 = load(v2);
    V3<double> lo = mk(fmin(P0.x, fmin(P1.x, P2.x)), fmin(P0.y, fmin(P1.y, P2.y)), fmin(P0.z, fmin(P1.z, P2.z)));
    V3<double> hi = mk(fmax(P0.x, fmax(P1.x, P2.x)), fmax(P0.y, fmax(P1.y, P2.y)), fmax(P0.z, fmax(P1.z, P2.z)));
    lbox[2 * i] = make_float4(round_down_f(lo.x), round_down_f(lo.y), round_down_f(lo.z), 0.f);
    lbox[2 * i + 1] = make_float4(round_up_f(hi.x), round_up_f(hi.y), round_up_f(hi.z), 0.f);

    // frame anchored on the longest edge (P_k, P_k+1)
    double l0 = norm2(P1 - P0), l1 = norm2(P2 - P1), l2 = norm2(P0 - P2);
    int k = 0;
    if (l1 > l0) k = 1;
    if (l2 > (k == 0 ? l0 : l1)) k = 2;
    V3<double> A = k == 0 ? P0 : (k == 1 ? P1 : P2);
    V3<double> B = k == 0 ? P1 : (k == 1 ? P2 : P0);
    V3<double> C = k == 0 ? P2 : (k == 1 ? P0 : P1);
    const int32_t iA = k == 0 ? v0 : (k == 1 ? v1 : v2);
    const int32_t iB = k == 0 ? v1 : (k == 1 ? v2 : v0);
    const int32_t iC = k == 0 ? v2 : (k == 1 ? v0 : v1);
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
    fr32[4 * i + 3] = make_float4((float)ibc, (float)ica, (float)Lb, __builtin_bit_cast(float, (int32_t)lf));
    double2 *q = fr64 + 8 * i;
    q[0] = make_double2(A.x, A.y);
    q[1] = make_double2(A.z, Lb);
    q[2] = make_double2(ex.x, ex.y);
    q[3] = make_double2(ex.z, cx);
    q[4] = make_double2(ey.x, ey.y);
    q[5] = make_double2(ey.z, cy);
    q[6] = make_double2(ibc, ica);
    q[7] = make_double2(Lb, (double)lf);
    ids[i] = make_int4(iA, iB, iC, (int32_t)lf);
    return Lb;
}

__device__ __forceinline__ void load_box(const float4 *nbox, const float4 *__restrict__ lbox, int32_t c, float4 &lo,
                                         float4 &hi) {
    if (c >= 0) {
        lo = nbox[2 * (int64_t)c];
        hi = nbox[2 * (int64_t)c + 1];
    } else {
        lo = lbox[2 * (int64_t)(~c)];
        hi = lbox[2 * (int64_t)(~c) + 1];
    }
}

// Float boxes as six values; union is exact (min / max), so any grouping of
// the same leaf boxes gives the same node box.
struct FBox {
    float lx, ly, lz, hx, hy, hz;
};
__device__ __forceinline__ FBox fbox_empty() {
    const float inf = __builtin_inff();
    return FBox{inf, inf, inf, -inf, -inf, -inf};
}
__device__ __forceinline__ FBox fbox_union(const FBox &a, const FBox &b) {
    return FBox{fminf(a.lx, b.lx), fminf(a.ly, b.ly), fminf(a.lz, b.lz),
                fmaxf(a.hx, b.hx), fmaxf(a.hy, b.hy), fmaxf(a.hz, b.hz)};
}
__device__ __forceinline__ FBox fbox_load(const float4 *__restrict__ b, int64_t k) {
    const float4 lo = b[2 * k], hi = b[2 * k + 1];
    return FBox{lo.x, lo.y, lo.z, hi.x, hi.y, hi.z};
}
__device__ __forceinline__ void fbox_store(float4 *b, int64_t k, const FBox &x) {
    b[2 * k] = make_float4(x.lx, x.ly, x.lz, 0.f);
    b[2 * k + 1] = make_float4(x.hx, x.hy, x.hz, 0.f);
}
// 256 boxes in LDS, structure of arrays
struct LdsBoxes {
    float v[6][TILE];
    __device__ FBox get(int k) const { return FBox{v[0][k], v[1][k], v[2][k], v[3][k], v[4][k], v[5][k]}; }
    __device__ void set(int k, const FBox &x) {
        v[0][k] = x.lx;
        v[1][k] = x.ly;
        v[2][k] = x.lz;
        v[3][k] = x.hx;
        v[4][k] = x.hy;
        v[5][k] = x.hz;
    }
};

// Prefix and suffix unions of the block's 256 boxes (thread t holds box t),
// doubling the aligned run length h from 1 to 256: with P_h[t] the union from
// the start of t's h-run to t and S_h[t] the union from t to the end of its
// run, P_2h[t] adds the whole lower run when t lies in the upper half, S_2h[t]
// the whole upper run when t lies in the lower half. visit(h, P_h[t], S_h[t])
// sees every level h < 256 before it is doubled (the levels of a disjoint
// sparse table); the return value is (P_256[t], S_256[t]). Every thread of
// the block must call it.
template <class Visit>
__device__ void run_unions(FBox box, LdsBoxes &P, LdsBoxes &S, FBox &pre, FBox &suf, Visit visit) {
    static_assert(TILE == 256, "one thread per box");
    const int t = threadIdx.x;
    pre = box;
    suf = box;
    for (int h = 1; h < TILE; h <<= 1) {
        visit(h, pre, suf);
        P.set(t, pre);
        S.set(t, suf);
        __syncthreads();
        const int base = t & ~(2 * h - 1);
        if (t & h) pre = fbox_union(P.get(base + h - 1), pre);
        else suf = fbox_union(suf, S.get(base + h));
        __syncthreads();
    }
}

// Refit, middle level: group g of TILE consecutive tiles, by one workgroup.
// tpre / tsuf: unions of the group's tiles up to / from tile a; gbox: the
// group's box; tdst[l][a] (l = 0..7, h = 2^l): the union from a to the end of
// its h-run when bit l of a is clear, from the start of its h-run to a when it
// is set (a disjoint sparse table: tiles a < b of one group with highest
// differing bit l have union tdst[l][a] U tdst[l][b]).
__device__ void group_tables(int64_t g, int64_t ntiles, const float4 *__restrict__ tbox, float4 *__restrict__ tpre,
                             float4 *__restrict__ tsuf, float4 *__restrict__ gbox, float4 *__restrict__ tdst,
                             LdsBoxes &P, LdsBoxes &S) {
    const int64_t a = g * TILE + threadIdx.x;
    const FBox b = a < ntiles ? fbox_load(tbox, a) : fbox_empty();
    FBox pre, suf;
    run_unions(b, P, S, pre, suf, [&](int h, const FBox &ph, const FBox &sh) {
        if (a < ntiles) fbox_store(tdst + 2 * (int64_t)(__builtin_ctz(h)) * ntiles, a, (a & h) ? ph : sh);
    });
    if (a < ntiles) {
        fbox_store(tpre, a, pre);
        fbox_store(tsuf, a, suf);
    }
    if (threadIdx.x == TILE - 1) fbox_store(gbox, g, pre);
}

// Refit, bottom level: one workgroup per tile of TILE consecutive leaves.
//  - Nodes whose leaf range lies inside the tile (their index then lies in
//    the tile too): bottom-up climb in LDS, the second thread to reach a node
//    builds it.
//  - For every leaf i: lpre[i] = union of the tile's leaves up to i, lsuf[i]
//    = union of leaves i to the tile's end; tbox = the tile's box. Nodes that
//    span tiles take their boxes from these (k_nodes).
__global__ __launch_bounds__(TILE) void k_refit_tiles(int64_t n, const int32_t *__restrict__ childL,
                                                      const int32_t *__restrict__ childR,
                                                      const int32_t *__restrict__ parentN,
                                                      const int32_t *__restrict__ parentL,
                                                      const int2 *__restrict__ range, const float4 *__restrict__ lbox,
                                                      float4 *__restrict__ nbox, float4 *__restrict__ lpre,
                                                      float4 *__restrict__ lsuf, float4 *__restrict__ tbox) {
    __shared__ LdsBoxes leaf, node;
    __shared__ int s_cl[TILE], s_cr[TILE], s_pn[TILE], s_cnt[TILE];
    __shared__ bool s_in[TILE];
    const int t = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * TILE, t1 = t0 + TILE - 1;
    const int64_t i = t0 + t;
    const FBox lb = i < n ? fbox_load(lbox, i) : fbox_empty();
    leaf.set(t, lb);
    // node slot t: node t0 + t, when its range lies inside the tile
    bool inside = false;
    if (i < n - 1) {
        const int2 r = range[i];
        inside = r.x >= t0 && r.y <= t1;
        s_cl[t] = childL[i];
        s_cr[t] = childR[i];
        s_pn[t] = parentN[i];
    }
    s_in[t] = inside;
    s_cnt[t] = 0;
    int32_t p = i < n ? parentL[i] : -1;
    __syncthreads();
    while (p >= t0 && p <= t1) {
        const int k = (int)(p - t0);
        if (!s_in[k]) break; // spans tiles: left to k_nodes
        const int old = __hip_atomic_fetch_add(&s_cnt[k], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == 0) break;
        const int32_t a = s_cl[k], b = s_cr[k];
        const FBox ba = a >= 0 ? node.get((int)(a - t0)) : leaf.get((int)(~a - t0));
        const FBox bb = b >= 0 ? node.get((int)(b - t0)) : leaf.get((int)(~b - t0));
        node.set(k, fbox_union(ba, bb));
        p = s_pn[k];
    }
    __syncthreads();
    if (inside) fbox_store(nbox, i, node.get(t));
    __syncthreads();
    FBox pre, suf;
    run_unions(lb, leaf, node, pre, suf, [](int, const FBox &, const FBox &) {});
    if (i < n) {
        fbox_store(lpre, i, pre);
        fbox_store(lsuf, i, suf);
    }
    if (t == TILE - 1) fbox_store(tbox, blockIdx.x, pre);
}

// one workgroup per group of tiles (group_tables); a separate launch: as the
// tail of the tile kernel (the last tile of a group to finish) it cost more,
// every tile block then fencing its writes device-wide
__global__ __launch_bounds__(TILE) void k_refit_groups(int64_t ntiles, const float4 *__restrict__ tbox,
                                                       float4 *__restrict__ tpre, float4 *__restrict__ tsuf,
                                                       float4 *__restrict__ gbox, float4 *__restrict__ tdst) {
    __shared__ LdsBoxes P, S;
    group_tables(blockIdx.x, ntiles, tbox, tpre, tsuf, gbox, tdst, P, S);
}

// One pass over the internal nodes, after the tiles and groups:
//  - refit, top level: every node whose leaf range [lo, hi] spans tiles, on
//    its own: the union of lsuf[lo], lpre[hi] and the whole tiles between
//    (one sparse-table pair within a group, else the two partial groups and
//    the whole groups between);
//  - each pair's root: the node whose leaf range is exactly the pair's leaves
//    (an endpoint of a node's range is its index, so it is node tri_begin or
//    node tri_end - 1);
//  - the four-wide collapse: a wide node stands for a binary node at even
//    depth below its pair's root, and its slots hold that node's
//    grandchildren (or a child itself when the child is a leaf); flag[i] = 1
//    for such a representative;
//  - threads below npairs: the pair's maxima, folded from the copies.
__global__ void k_nodes(int64_t ninternal, int64_t ntiles, const int2 *__restrict__ range,
                        const float4 *__restrict__ lpre, const float4 *__restrict__ lsuf,
                        const float4 *__restrict__ tbox, const float4 *__restrict__ tpre,
                        const float4 *__restrict__ tsuf, const float4 *__restrict__ gbox,
                        const float4 *__restrict__ tdst, float4 *__restrict__ nbox, const int32_t *__restrict__ parentN,
                        const unsigned long long *__restrict__ keys, BvhPair *pairs, int npairs,
                        int32_t *__restrict__ flag, const PairAcc *__restrict__ acc, int astride) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid < npairs) {
        unsigned long long cm = 0, em = 0;
        for (int c = 0; c < ACC_COPIES; ++c) {
            const PairAcc &a = acc[(int64_t)c * astride + gid];
            cm = a.coord_max > cm ? a.coord_max : cm;
            em = a.edge_max > em ? a.edge_max : em;
        }
        pairs[gid].coord_max = ord2d(cm);
        pairs[gid].edge_max = ord2d(em);
    }
    for (int64_t i = gid; i < ninternal; i += (int64_t)gridDim.x * blockDim.x) {
        const int2 r = range[i];
        const int64_t ta = r.x / TILE, tb = r.y / TILE;
        if (ta != tb) {
            FBox x = fbox_union(fbox_load(lsuf, r.x), fbox_load(lpre, r.y));
            const int64_t a = ta + 1, b = tb - 1;
            if (a == b) {
                x = fbox_union(x, fbox_load(tbox, a));
            } else if (a < b) {
                const int64_t ga = a / TILE, gb = b / TILE;
                if (ga == gb) {
                    const int l = 31 - __clz((int)(a ^ b));
                    const float4 *d = tdst + 2 * (int64_t)l * ntiles;
                    x = fbox_union(x, fbox_union(fbox_load(d, a), fbox_load(d, b)));
                } else {
                    x = fbox_union(x, fbox_union(fbox_load(tsuf, a), fbox_load(tpre, b)));
                    for (int64_t g = ga + 1; g < gb; ++g) x = fbox_union(x, fbox_load(gbox, g));
                }
            }
            fbox_store(nbox, i, x);
        }
        int f = 0;
        const int p = (int)(keys[r.x] >> 32);
        if (p >= 0 && p < npairs) {
            const int64_t b0 = pairs[p].tri_begin, b1 = pairs[p].tri_end; // leaves [b0, b1)
            if (r.x >= b0 && (int64_t)r.y < b1 && b1 - b0 > 1) {
                const bool root_lo = range[b0].x == b0 && (int64_t)range[b0].y == b1 - 1;
                const int64_t root = root_lo ? b0 : b1 - 1;
                if (i == root) pairs[p].root = (int32_t)i;
                int depth = 0;
                int32_t x = (int32_t)i;
                while (x != root && x >= 0) {
                    x = parentN[x];
                    ++depth;
                }
                f = (x == root && (depth & 1) == 0) ? 1 : 0;
            }
        }
        flag[i] = f;
    }
}

// A four-wide node per flagged binary node, stored at the binary node's own
// index (the array is sparse: no scan to number the flagged nodes, and slot
// references are binary node indices).
__device__ void wide_node(int64_t i, const int32_t *__restrict__ childL, const int32_t *__restrict__ childR,
                          const float4 *__restrict__ nbox, const float4 *__restrict__ lbox, WideNode *__restrict__ out) {
    float lo[3][4], hi[3][4];
    int ref[4];
    int k = 0;
    auto put = [&](int32_t c) {
        float4 l, h;
        load_box(nbox, lbox, c, l, h);
        // k is at most 3 here; the stores below use constant indices
        const float lv[3] = {l.x, l.y, l.z}, hv[3] = {h.x, h.y, h.z};
        const int32_t rf = c;
#pragma unroll
        for (int s = 0; s < 4; ++s)
            if (s == k) {
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    lo[d][s] = lv[d];
                    hi[d][s] = hv[d];
                }
                ref[s] = rf;
            }
        ++k;
    };
    const int32_t c2[2] = {childL[i], childR[i]};
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int32_t c = c2[j];
        if (c < 0) {
            put(c);
        } else {
            put(childL[c]);
            put(childR[c]);
        }
    }
    WideNode w;
#pragma unroll
    for (int s = 0; s < 4; ++s)
        if (s >= k) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                lo[d][s] = 0.f;
                hi[d][s] = 0.f;
            }
            ref[s] = WIDE_EMPTY;
        }
    w.lox = make_float4(lo[0][0], lo[0][1], lo[0][2], lo[0][3]);
    w.loy = make_float4(lo[1][0], lo[1][1], lo[1][2], lo[1][3]);
    w.loz = make_float4(lo[2][0], lo[2][1], lo[2][2], lo[2][3]);
    w.hix = make_float4(hi[0][0], hi[0][1], hi[0][2], hi[0][3]);
    w.hiy = make_float4(hi[1][0], hi[1][1], hi[1][2], hi[1][3]);
    w.hiz = make_float4(hi[2][0], hi[2][1], hi[2][2], hi[2][3]);
    w.child = make_int4(ref[0], ref[1], ref[2], ref[3]);
    w.meta = make_int4(k, 0, 0, 0);
    out[i] = w;
}

// Entry t of pair 0's top-level table (see TOP_NODES), by thread t: entry
// 0 the root, 1 + k the root's child k, 5 + 4k + m child m of that child
// (entries of slots that are empty or leaves stay unused); references from
// the root and its children to tabled nodes become TOP_REF + entry.
__device__ void top_entry(const WideNode *__restrict__ nodes, int32_t root, WideNode *top, int t) {
    if (t >= TOP_NODES) return;
    int32_t x = root;
    if (t >= 1) {
        const int k = t <= 4 ? t - 1 : (t - 5) >> 2;
        x = (&nodes[root].child.x)[k];
        if (t >= 5 && x >= 0) x = (&nodes[x].child.x)[(t - 5) & 3];
    }
    if (x < 0) return;
    WideNode w = nodes[x];
    if (t <= 4) {
        const int first = t == 0 ? 1 : 5 + 4 * (t - 1);
        int32_t *ch = &w.child.x;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if (ch[m] >= 0) ch[m] = TOP_REF + first + m;
    }
    top[t] = w;
}

// the four-wide nodes, one thread per binary node
__global__ __launch_bounds__(BLK) void k_wide_nodes(int64_t ninternal, const int32_t *__restrict__ flag,
                                                    const int32_t *__restrict__ childL,
                                                    const int32_t *__restrict__ childR,
                                                    const float4 *__restrict__ nbox, const float4 *__restrict__ lbox,
                                                    WideNode *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ninternal && flag[i]) wide_node(i, childL, childR, nbox, lbox, out);
}

// pair 0's top-level table (a single-pair BVH with an internal root)
__global__ void k_wide_top(const WideNode *__restrict__ nodes, const BvhPair *pairs, WideNode *top) {
    const int32_t root = pairs[0].root;
    if (root >= 0) top_entry(nodes, root, top, threadIdx.x);
}


// build scratch, reused between builds on the same device; kept until the
// process ends (never destroyed: the HIP runtime may be gone by static
// destruction). A build that finds it busy uses a private one.
//
// The build is a fixed sequence of copies and kernels whose arguments depend
// only on the soup sizes and on the buffers (not on the data, which the
// device reads through the staged source records). It is captured once into a
// HIP graph per (sizes, buffers) and replayed on later builds: one graph
// launch instead of ~30 kernel launches, so the GPU runs the short build
// kernels back to back instead of waiting on the host for each. A few graphs
// are kept per device (builds alternate between the pooled BVH handles).
constexpr int BUILD_GRAPHS = 4;
constexpr int BUILD_KEY = 13;
struct BuildGraph {
    uintptr_t key[BUILD_KEY];
    hipGraphExec_t exec = nullptr;
};
struct BuildScratch {
    std::mutex mu;
    DBuf mem, sort_tmp, src;
    PinnedBuf host; // [0, 4) export sequence word; staged uploads; exported results
    hipStream_t capture = nullptr;     // stream the build is captured on (never run)
    std::vector<BuildGraph> graphs;    // most recently used last
};
std::atomic<int> g_build_graphs{1};
std::mutex g_scratch_mu;
BuildScratch *g_scratch[64] = {};
BuildScratch *scratch_for(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    BuildScratch *&b = g_scratch[dev & 63];
    if (!b) b = new BuildScratch();
    return b;
}

// Released BVH handles keep their device buffers for the next build on the
// same device (a few per device), so that repeated build/free cycles do not
// pay for hipMalloc and hipFree each time.
constexpr int SPARE_BVHS = 2;
std::mutex g_spare_mu;
std::vector<Bvh *> g_spare[64];

Bvh *take_bvh(int dev) {
    std::lock_guard<std::mutex> lk(g_spare_mu);
    std::vector<Bvh *> &v = g_spare[dev & 63];
    if (v.empty()) return new Bvh();
    Bvh *b = v.back();
    v.pop_back();
    return b;
}

} // namespace

int set_build_graphs(int enable) { return g_build_graphs.exchange(enable ? 1 : 0); }

void recycle_bvh(Bvh *b) {
    if (!b) return;
    // work queued on any stream may still read the BVH: wait for it, as the
    // hipFree calls of a plain delete would
    if (hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        delete b;
        return;
    }
    std::lock_guard<std::mutex> lk(g_spare_mu);
    std::vector<Bvh *> &v = g_spare[b->device & 63];
    if ((int)v.size() < SPARE_BVHS) {
        b->npairs = 0;
        b->nB = 0;
        b->hpairs.clear();
        v.push_back(b);
    } else {
        delete b;
    }
}

Bvh *build_bvh(int npairs, const double *const *VB, const int64_t *mB, const int32_t *const *FB, const int64_t *nBp,
               hipStream_t s) {
    if (npairs <= 0) throw Error{HD_E_INVALID, "no soup"};
    std::vector<int64_t> foff(npairs + 1, 0);
    for (int p = 0; p < npairs; ++p) {
        if (nBp[p] <= 0 || mB[p] <= 0 || !VB[p] || !FB[p]) throw Error{HD_E_INVALID, "empty soup B"};
        foff[p + 1] = foff[p] + nBp[p];
    }
    const int64_t n = foff[npairs];
    if (n >= (int64_t(1) << 30)) throw Error{HD_E_INVALID, "soups B too large (>= 2^30 faces)"};
    int dev = 0;
    HD_HIP(hipGetDevice(&dev));
    Bvh *b = take_bvh(dev);
    try {
        b->device = dev;
        BuildScratch *shared = scratch_for(b->device);
        std::unique_lock<std::mutex> lk(shared->mu, std::try_to_lock);
        std::unique_ptr<BuildScratch> priv;
        if (!lk.owns_lock()) priv.reset(new BuildScratch());
        BuildScratch &sc = lk.owns_lock() ? *shared : *priv;
        b->npairs = npairs;
        b->nB = n;
        // pinned staging: sources and face offsets, pair records; results
        auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
        const size_t o_src = 256, o_foff = o_src + al(npairs * sizeof(PairSrc)),
                     o_pairs = o_foff + al((npairs + 1) * sizeof(int64_t)),
                     o_rst = o_pairs + al(npairs * sizeof(BvhPair)), o_rpairs = o_rst + al(sizeof(BuildState)),
                     host_bytes = o_rpairs + al(npairs * sizeof(BvhPair));
        sc.host.reserve(host_bytes);
        const int64_t ni = n > 1 ? n - 1 : 1;
        size_t off = 0;
        auto take = [&](size_t bytes) {
            size_t o = off;
            off += (bytes + 255) & ~size_t(255);
            return o;
        };
        size_t o_state = take(sizeof(BuildState));
        const int astride = (int)(((npairs * sizeof(PairAcc) + 255) & ~size_t(255)) / sizeof(PairAcc));
        size_t o_acc = take((size_t)ACC_COPIES * astride * sizeof(PairAcc));
        size_t o_fpair = take(n * sizeof(int32_t));
        size_t o_keys = take(n * sizeof(unsigned long long));
        size_t o_vals = take(n * sizeof(int32_t));
        size_t o_keys2 = take(n * sizeof(unsigned long long));
        size_t o_vals2 = take(n * sizeof(int32_t));
        size_t o_cl = take(ni * sizeof(int32_t));
        size_t o_cr = take(ni * sizeof(int32_t));
        size_t o_pn = take(ni * sizeof(int32_t));
        size_t o_pl = take(n * sizeof(int32_t));
        const int64_t ntiles = (n + TILE - 1) / TILE, ngroups = (ntiles + TILE - 1) / TILE;
        size_t o_range = take(ni * sizeof(int2));
        size_t o_lps = take(2 * n * 2 * sizeof(float4)); // lpre, lsuf
        size_t o_tps = take(3 * ntiles * 2 * sizeof(float4)); // tbox, tpre, tsuf
        size_t o_tdst = take(8 * ntiles * 2 * sizeof(float4));
        size_t o_gbox = take(ngroups * 2 * sizeof(float4));
        size_t o_flag = take(ni * sizeof(int32_t));
        size_t o_lbox = take(n * 2 * sizeof(float4));
        size_t o_nbox = take(ni * 2 * sizeof(float4));
        sc.mem.reserve(off);
        char *base = sc.mem.as<char>();
        BuildState *st = (BuildState *)(base + o_state);
        PairAcc *acc = (PairAcc *)(base + o_acc);
        int32_t *fpair = (int32_t *)(base + o_fpair);
        unsigned long long *keys = (unsigned long long *)(base + o_keys);
        int32_t *vals = (int32_t *)(base + o_vals);
        unsigned long long *keys2 = (unsigned long long *)(base + o_keys2);
        int32_t *vals2 = (int32_t *)(base + o_vals2);
        int32_t *cl = (int32_t *)(base + o_cl);
        int32_t *cr = (int32_t *)(base + o_cr);
        int32_t *pn = (int32_t *)(base + o_pn);
        int32_t *pl = (int32_t *)(base + o_pl);
        int2 *range = (int2 *)(base + o_range);
        float4 *lpre = (float4 *)(base + o_lps), *lsuf = lpre + 2 * n;
        float4 *tbox = (float4 *)(base + o_tps), *tpre = tbox + 2 * ntiles, *tsuf = tpre + 2 * ntiles;
        float4 *tdst = (float4 *)(base + o_tdst);
        float4 *gbox = (float4 *)(base + o_gbox);
        int32_t *flag = (int32_t *)(base + o_flag);
        float4 *lbox = (float4 *)(base + o_lbox);
        float4 *nbox = (float4 *)(base + o_nbox);

        // every buffer the build writes, reserved before any work is enqueued
        // (the enqueued sequence allocates nothing, so that it can be captured)
        sc.src.reserve(o_pairs - o_src);
        b->pairs.reserve(npairs * sizeof(BvhPair));
        b->nodes.reserve(ni * sizeof(WideNode));
        b->frames32.reserve(n * 4 * sizeof(float4));
        b->frames64.reserve(n * 8 * sizeof(double2));
        b->ids.reserve(n * sizeof(int4));
        const bool with_top = npairs == 1 && n > 1;
        if (with_top) b->top.reserve((size_t)TOP_NODES * sizeof(WideNode));
        sc.sort_tmp.reserve(radix_sort_tmp_bytes(n));
        int pair_bits = 0;
        while ((1 << pair_bits) < npairs) ++pair_bits;

        // per-pair sources and face offsets, pair records: staged in pinned memory
        PairSrc *hsrc = sc.host.as<PairSrc>(o_src);
        for (int p = 0; p < npairs; ++p) hsrc[p] = PairSrc{VB[p], FB[p], mB[p]};
        std::memcpy(sc.host.as<char>(o_foff), foff.data(), (npairs + 1) * sizeof(int64_t));
        BvhPair *hp = sc.host.as<BvhPair>(o_pairs);
        for (int p = 0; p < npairs; ++p) {
            hp[p] = BvhPair{};
            hp[p].tri_begin = foff[p];
            hp[p].tri_end = foff[p + 1];
            hp[p].nB = (int32_t)nBp[p];
            hp[p].root = nBp[p] == 1 ? ~(int32_t)foff[p] : -1;
        }
        // source records and offsets share one device block with the pinned layout
        PairSrc *dsrc = sc.src.as<PairSrc>();
        int64_t *dfoff = (int64_t *)(sc.src.as<char>() + (o_foff - o_src));
        BvhPair *dpairs = b->pairs.as<BvhPair>();

        // the build, then the export of its state and pair records with
        // sequence word 1 (the host clears the word before each build)
        auto enqueue = [&](hipStream_t q) {
            HD_HIP(hipMemcpyAsync(dsrc, sc.host.as<char>(o_src), o_pairs - o_src, hipMemcpyHostToDevice, q));
            HD_HIP(hipMemcpyAsync(dpairs, hp, npairs * sizeof(BvhPair), hipMemcpyHostToDevice, q));
            k_init<<<grid_for((int64_t)npairs * ACC_COPIES, 64), 64, 0, q>>>(acc, npairs, astride, st);
            k_faces_check<<<face_grid(n, npairs), BLK, 0, q>>>(dsrc, dfoff, npairs, n, acc, astride, st);
            k_centroids<<<face_grid(n, npairs), BLK, 0, q>>>(dsrc, dfoff, npairs, n, dpairs, fpair,
                                                                                 acc, astride, st, keys, vals);
            HD_LAUNCH_CHECK();
            radix_sort_u64(keys, vals, keys2, vals2, n, pair_bits ? 32 + pair_bits : 30, sc.sort_tmp, q);
            k_leaves<<<grid_for(n, BLK), BLK, 0, q>>>(dsrc, dfoff, fpair, vals, n, dpairs, lbox,
                                                      b->frames32.as<float4>(), b->frames64.as<double2>(),
                                                      b->ids.as<int4>(), acc, astride, st, keys, cl, cr, pn, pl,
                                                      range);
            HD_LAUNCH_CHECK();
            if (n > 1) {
                k_refit_tiles<<<(unsigned)ntiles, TILE, 0, q>>>(n, cl, cr, pn, pl, range, lbox, nbox, lpre, lsuf,
                                                                 tbox);
                if (ntiles > 1)
                    k_refit_groups<<<(unsigned)ngroups, TILE, 0, q>>>(ntiles, tbox, tpre, tsuf, gbox, tdst);
            }
            const int64_t nint = n - 1; // internal nodes (none for a single triangle)
            k_nodes<<<grid_for(std::min<int64_t>(std::max<int64_t>(nint, npairs), 512 * BLK), BLK), BLK, 0, q>>>(
                nint, ntiles, range, lpre, lsuf, tbox, tpre, tsuf, gbox, tdst, nbox, pn, keys, dpairs, npairs, flag,
                acc, astride);
            if (n > 1)
                k_wide_nodes<<<grid_for(ni, BLK), BLK, 0, q>>>(ni, flag, cl, cr, nbox, lbox, b->nodes.as<WideNode>());
            if (with_top) k_wide_top<<<1, 64, 0, q>>>(b->nodes.as<WideNode>(), dpairs, b->top.as<WideNode>());
            HD_LAUNCH_CHECK();
            Export ex{};
            ex.n = 2;
            ex.src[0] = st;
            ex.dst[0] = sc.host.dev_as<char>(o_rst);
            ex.bytes[0] = sizeof(BuildState);
            ex.src[1] = dpairs;
            ex.dst[1] = sc.host.dev_as<char>(o_rpairs);
            ex.bytes[1] = npairs * sizeof(BvhPair);
            export_to_host(ex, sc.host.dev_as<unsigned>(0), 1u, q);
        };
        unsigned *seq_word = sc.host.as<unsigned>(0);
        __atomic_store_n(seq_word, 0u, __ATOMIC_RELEASE);
        if (lk.owns_lock() && g_build_graphs.load()) {
            const uintptr_t key[BUILD_KEY] = {(uintptr_t)n,
                                              (uintptr_t)npairs,
                                              (uintptr_t)sc.mem.p,
                                              (uintptr_t)sc.src.p,
                                              (uintptr_t)sc.sort_tmp.p,
                                              (uintptr_t)sc.host.p,
                                              (uintptr_t)b->pairs.p,
                                              (uintptr_t)b->nodes.p,
                                              (uintptr_t)b->frames32.p,
                                              (uintptr_t)b->frames64.p,
                                              (uintptr_t)b->ids.p,
                                              (uintptr_t)(with_top ? b->top.p : nullptr),
                                              (uintptr_t)dev};
            hipGraphExec_t exec = nullptr;
            for (size_t g = 0; g < sc.graphs.size(); ++g)
                if (std::memcmp(sc.graphs[g].key, key, sizeof(key)) == 0) {
                    BuildGraph hit = sc.graphs[g];
                    sc.graphs.erase(sc.graphs.begin() + g);
                    sc.graphs.push_back(hit);
                    exec = hit.exec;
                    break;
                }
            if (!exec) {
                if (!sc.capture) HD_HIP(hipStreamCreateWithFlags(&sc.capture, hipStreamNonBlocking));
                HD_HIP(hipStreamBeginCapture(sc.capture, hipStreamCaptureModeRelaxed));
                hipGraph_t graph = nullptr;
                try {
                    enqueue(sc.capture);
                } catch (...) {
                    if (hipStreamEndCapture(sc.capture, &graph) == hipSuccess && graph) (void)hipGraphDestroy(graph);
                    (void)hipGetLastError();
                    throw;
                }
                HD_HIP(hipStreamEndCapture(sc.capture, &graph));
                const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ie != hipSuccess) throw Error{HD_E_DEVICE, hipGetErrorString(ie)};
                if ((int)sc.graphs.size() == BUILD_GRAPHS) {
                    (void)hipGraphExecDestroy(sc.graphs.front().exec);
                    sc.graphs.erase(sc.graphs.begin());
                }
                BuildGraph bg;
                std::memcpy(bg.key, key, sizeof(key));
                bg.exec = exec;
                sc.graphs.push_back(bg);
            }
            HD_HIP(hipGraphLaunch(exec, s));
        } else {
            enqueue(s);
        }
        wait_host_seq(seq_word, 1u, s);
        const BuildState hs = *sc.host.as<BuildState>(o_rst);
        b->hpairs.assign(sc.host.as<BvhPair>(o_rpairs), sc.host.as<BvhPair>(o_rpairs) + npairs);
        if (hs.bad) throw Error{HD_E_INVALID, "soup B has an out-of-range index or a non-finite coordinate"};
        for (int p = 0; p < npairs; ++p)
            if (b->hpairs[p].nB > 1 && b->hpairs[p].root < 0) throw Error{HD_E_INTERNAL, "pair subtree root not found"};
        return b;
    } catch (...) {
        recycle_bvh(b);
        throw;
    }
}

} // namespace hd
