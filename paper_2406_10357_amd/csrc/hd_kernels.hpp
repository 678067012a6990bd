// hd_kernels.hpp -- device pieces of the branch-and-bound rounds: the
// frontier record layout, BVH traversal for point queries, the cascade with
// its rounding margins, and the FP64 re-bound of a frontier triangle.
#pragma once
#include "hd_geom.hpp"
#include "hd_internal.hpp"

namespace hd {

// ---------------------------------------------------------------------------
// Margins. For a value computed in precision T with unit roundoff u:
//   point query:    |d_computed - d_exact| <= mu_d * d + mu_0
//   triangle bound: |ub_computed - ub_exact| <= mu_d * dmax + mu_e * emax + mu_0
// with mu_d = 16u, mu_e = 48u and mu_0 = u * (48 * D_B + 12 * S): D_B the
// longest edge of B, S the largest coordinate magnitude after centring
// (forward-error analysis of the frame evaluation and of the bound formulas,
// with a safety factor of about 2).
// ---------------------------------------------------------------------------
struct Margins {
    double mu_d, mu_e, mu_0;
};

// Per pair state of one call, in two device arrays: constants read by every
// thread (written once after ingest), and the fields that kernels update
// with atomics. Keeping them on separate cache lines matters: a device-scope
// atomic evicts its line from every XCD's L2, and the constants are read by
// every query.
struct PairConst {
    double ctr[3];  // centre subtracted from every coordinate of the pair
    int32_t root;   // BVH subtree root (>= 0 node, < 0 leaf ~root)
    int32_t link;   // the pair whose lower bound this pair shares (itself unless linked)
    double eps_abs, dA;
    Margins m32, m64;
};
struct alignas(128) PairVar {
    unsigned long long Lord;      // ordered double: certified lower bound
    unsigned long long round_key; // best (d_lo, tie tag) key of the current query round
    unsigned long long Uord;      // ordered double: final upper bound
    unsigned long long Urounds;   // ordered double: largest live bound of the rounds
    unsigned long long best_key;  // best key so far
    double argmax_pos[3];         // centred FP64 position of the best vertex
    int32_t argmax_dirty;
    int32_t argmax_tri;           // closest triangle (sorted index) found for it by the query
    double L64;
    unsigned long long Uround;    // ordered double: largest live bound after a round (round log)
};

// The lower bound pair p's decisions use: its own, or, for two linked pairs
// (the two directions of a two-sided distance), the larger of the two. A
// triangle bounded below it cannot raise the maximum of the two distances.
HD_D double pair_L(const PairConst *pc, const PairVar *pv, int p) {
    const unsigned long long a = pv[p].Lord, b = pv[pc[p].link].Lord;
    return ord2d(a > b ? a : b);
}

// ---------------------------------------------------------------------------
// Frontier records (structure of arrays; one slot per triangle).
// A frontier triangle is a piece of an original face `face` of A, obtained by
// `lvl` rounds of 1->4 midpoint subdivision. Its vertex i sits at the exact
// dyadic barycentric position V0 + (ba[i] * E1 + bb[i] * E2) / 2^lvl of that
// face (E1 = V1 - V0, E2 = V2 - V0), so positions never accumulate rounding.
// ---------------------------------------------------------------------------
// One allocation of `cap` records, field by field (structure of arrays): 21
// fields of T, then 14 fields of 4 bytes. A view is a base and a capacity, so
// choosing among several lists per lane costs a few registers, not a table of
// pointers.
template <class T> struct FrontierView {
    char *base;
    int64_t cap; // a multiple of 64, so every field starts 256-byte aligned
    HD_HD T *v(int k) const { return (T *)base + (int64_t)k * cap; }       // vertex i coordinate c at k = 3i+c
    HD_HD T *q(int k) const { return (T *)base + (int64_t)(9 + k) * cap; } // closest point on B of vertex i
    HD_HD T *d(int i) const { return (T *)base + (int64_t)(18 + i) * cap; } // computed distance of vertex i to B
    HD_HD int *i32(int m) const { return (int *)((T *)base + 21 * cap) + (int64_t)m * cap; }
    HD_HD int *I(int i) const { return i32(i); } // closest triangle of vertex i (sorted index into B)
    HD_HD float *ub() const { return (float *)i32(3); } // upper bound, margin included, rounded up
    HD_HD int *face() const { return i32(4); }
    HD_HD int *lvl() const { return i32(5); }
    HD_HD int *pair() const { return i32(6); }
    HD_HD int *ba(int i) const { return i32(7 + i); } // dyadic barycentric numerators of vertex i
    HD_HD int *bb(int i) const { return i32(10 + i); }
    HD_HD float *score() const { return (float *)i32(13); } // learned proposal: predicted max distance (NaN: none)
    static constexpr size_t bytes_per_record() { return 21 * sizeof(T) + 14 * 4; }
};

// A's vertices and faces (all pairs concatenated; face indices are global).
struct AView {
    const double *V;
    const int32_t *F;
    const PairConst *pc;
};

HD_D V3<double> a_vertex(const AView &a, int pair, int32_t v) {
    const double *c = a.pc[pair].ctr;
    return {a.V[3 * (int64_t)v] - c[0], a.V[3 * (int64_t)v + 1] - c[1], a.V[3 * (int64_t)v + 2] - c[2]};
}

// exact dyadic point of face f (centred coordinates of its pair)
HD_D V3<double> a_point(const AView &a, int pair, int32_t f, int lvl, int ba, int bb) {
    V3<double> V0 = a_vertex(a, pair, a.F[3 * (int64_t)f]);
    V3<double> V1 = a_vertex(a, pair, a.F[3 * (int64_t)f + 1]);
    V3<double> V2 = a_vertex(a, pair, a.F[3 * (int64_t)f + 2]);
    double s = __builtin_ldexp(1.0, -lvl);
    double wa = (double)ba * s, wb = (double)bb * s;
    return V0 + (wa * (V1 - V0) + wb * (V2 - V0));
}

// order-independent 32-bit tag of a dyadic point (reduced fraction), used to
// break ties between equal keys the same way on every run
HD_HD uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352du;
    x ^= x >> 15;
    x *= 0x846ca68bu;
    x ^= x >> 16;
    return x;
}
HD_HD uint32_t point_tag(int32_t face, int lvl, int ba, int bb) {
    while (lvl > 0 && ((ba | bb) & 1) == 0) {
        ba >>= 1;
        bb >>= 1;
        --lvl;
    }
    return mix32((uint32_t)face * 0x9E3779B1u ^ mix32((uint32_t)ba * 0x85ebca6bu + (uint32_t)bb) ^ (uint32_t)lvl * 0xc2b2ae35u);
}

// ---------------------------------------------------------------------------
// Traversal
// ---------------------------------------------------------------------------
template <class T> HD_D T box_d2(const float4 &lo, const float4 &hi, const V3<T> &p) {
    T dx = hmax(hmax(T(lo.x) - p.x, p.x - T(hi.x)), T(0));
    T dy = hmax(hmax(T(lo.y) - p.y, p.y - T(hi.y)), T(0));
    T dz = hmax(hmax(T(lo.z) - p.z, p.z - T(hi.z)), T(0));
    return dx * dx + dy * dy + dz * dz;
}

HD_D float to_float_down(float x) { return x; }
HD_D float to_float_down(double x) {
    float f = (float)x;
    if ((double)f > x) f = next_down(f);
    return f;
}

// Per-lane short stack in LDS, entries [slot][lane of block], kept as a ring:
// a push onto a full stack overwrites the oldest entry and reports the loss;
// the traversal then restarts from the root once the stack runs empty, with
// the best distance found so far (every subtree whose entry was lost is
// still reachable from the root and is pruned or visited again).
template <int SD, int BLOCK> struct LdsStack {
    int *node;
    float *dist;
    int top = 0, cnt = 0;
    HD_D bool push(int n, float d) {
        node[top * BLOCK + threadIdx.x] = n;
        dist[top * BLOCK + threadIdx.x] = d;
        top = top + 1 == SD ? 0 : top + 1;
        if (cnt == SD) return false;
        ++cnt;
        return true;
    }
    HD_D bool pop(int &n, float &d) {
        if (cnt == 0) return false;
        top = top == 0 ? SD - 1 : top - 1;
        --cnt;
        n = node[top * BLOCK + threadIdx.x];
        d = dist[top * BLOCK + threadIdx.x];
        return true;
    }
    HD_D void clear() { top = cnt = 0; }
};

// per-lane stack in global memory (deep fallback)
struct GlobalStack {
    int2 *base; // depth x stride
    int64_t stride;
    int depth;
    int sp = 0;
    HD_D bool push(int n, float d) {
        if (sp >= depth) return false;
        base[(int64_t)sp * stride] = make_int2(n, __builtin_bit_cast(int, d));
        ++sp;
        return true;
    }
    HD_D bool pop(int &n, float &d) {
        if (sp == 0) return false;
        --sp;
        int2 e = base[(int64_t)sp * stride];
        n = e.x;
        d = __builtin_bit_cast(float, e.y);
        return true;
    }
    HD_D void clear() { sp = 0; }
};

// traversal restarts allowed after stack losses before the query is handed
// to the deep-stack path
constexpr int MAX_RESTARTS = 3;

template <class T> struct QueryResult {
    T d2;
    int s;    // sorted index of the closest triangle
    int orig; // its original face index
    int nbox, nleaf;
    bool overflow;
};

template <class T> HD_D QueryResult<T> empty_result() {
    QueryResult<T> r;
    r.d2 = T(__builtin_inf());
    r.s = -1;
    r.orig = 0x7fffffff;
    r.nbox = 0;
    r.nleaf = 0;
    r.overflow = false;
    return r;
}

// fold leaf s (its frame f) into the running result (exact ties: smallest
// original index)
template <class T> HD_D void fold_leaf(QueryResult<T> &r, const Frame<T> &f, const V3<T> &p, int s) {
    T d2 = frame_dist2<T, false>(f, p, nullptr);
    ++r.nleaf;
    if (d2 < r.d2 || (d2 == r.d2 && f.orig < r.orig)) {
        r.d2 = d2;
        r.s = s;
        r.orig = f.orig;
    }
}

template <class T>
HD_D void visit_leaf(QueryResult<T> &r, const BView<T> &bv, const int4 *__restrict__ ids, const V3<T> &p, int s) {
    fold_leaf(r, load_frame(bv.frames, s), p, s);
}

// seed a result with up to two candidate triangles (s < 0: none), both frames
// loaded before either is evaluated
template <class T>
HD_D void seed_two(QueryResult<T> &r, const BView<T> &bv, const V3<T> &p, int s0, int s1) {
    if (s1 == s0) s1 = -1;
    Frame<T> F0, F1;
    if (s0 >= 0) F0 = load_frame(bv.frames, s0);
    if (s1 >= 0) F1 = load_frame(bv.frames, s1);
    if (s0 >= 0) fold_leaf(r, F0, p, s0);
    if (s1 >= 0) fold_leaf(r, F1, p, s1);
}

// Where a traversal reads wide nodes: references below TOP_REF from global
// memory, TOP_REF + j from entry j of the top-level table staged in LDS
// (typed as LDS, so that those reads are ds_read rather than flat loads).
// Without a table no such reference occurs.
typedef __attribute__((address_space(3))) const float LdsFloat;
typedef __attribute__((address_space(3))) const int LdsInt;
struct NodeSrc {
    const WideNode *__restrict__ g;
    LdsFloat *top; // the table as WIDE_WORDS words per node
};

// the four child boxes and references of wide node x
struct WideView {
    float4 lx, ly, lz, hx, hy, hz;
    int4 ch;
};
HD_D WideView load_wide(const NodeSrc &ns, int x) {
    WideView v;
    if (x >= TOP_REF) {
        LdsFloat *t = ns.top + WIDE_WORDS * (x - TOP_REF);
        auto f4 = [&](int o) { return make_float4(t[o], t[o + 1], t[o + 2], t[o + 3]); };
        v.lx = f4(0);
        v.ly = f4(4);
        v.lz = f4(8);
        v.hx = f4(12);
        v.hy = f4(16);
        v.hz = f4(20);
        LdsInt *c = (LdsInt *)t + 24;
        v.ch = make_int4(c[0], c[1], c[2], c[3]);
        return v;
    }
    const WideNode *w = ns.g + x;
    v.lx = w->lox;
    v.ly = w->loy;
    v.lz = w->loz;
    v.hx = w->hix;
    v.hy = w->hiy;
    v.hz = w->hiz;
    v.ch = w->child;
    return v;
}

// FP32 leaf frames in flight at once per lane in `traverse` (1, 2 or 4):
// more loads in flight per lane against more registers, so fewer waves
#ifndef HD_LEAF_BATCH
#define HD_LEAF_BATCH 4
#endif
constexpr int LEAF_BATCH = HD_LEAF_BATCH;
static_assert(LEAF_BATCH == 1 || LEAF_BATCH == 2 || LEAF_BATCH == 4, "leaf batch of 1, 2 or 4 frames");

// Closest-first traversal from `root`, starting from the result `r` (empty,
// or seeded with candidate triangles). A child box is entered only when its
// distance is within (1 + 16u) of the best squared distance so far, which
// keeps pruning conservative under the rounding of the box test. Per wide
// node: leaf children are evaluated at once; the internal children still in
// range are sorted by box distance, the nearest is entered and the others are
// pushed farthest first.
template <class T>
HD_D void cswap(T &ea, int &fa, T &eb, int &fb) {
    if (eb < ea) {
        T te = ea;
        ea = eb;
        eb = te;
        int tf = fa;
        fa = fb;
        fb = tf;
    }
}

// Descent without a bound: nearest box first, nothing pushed, down to one
// leaf, whose distance then bounds the real traversal (without it every
// child would be in range and every sibling pushed).
template <class T>
HD_D void greedy_probe(const NodeSrc &nodes, const BView<T> &bv, const int4 *__restrict__ ids, const V3<T> &p,
                       int root, QueryResult<T> &r) {
    int x = root;
    for (int guard = 0; guard < 64 && x >= 0; ++guard) {
        const WideView w = load_wide(nodes, x);
        const float4 lx = w.lx, ly = w.ly, lz = w.lz, hx = w.hx, hy = w.hy, hz = w.hz;
        const int4 ch = w.ch;
        T best = T(__builtin_inf());
        int pick = WIDE_EMPTY;
        auto consider = [&](float a, float b, float c, float d, float e, float f, int ref) {
            if (ref == WIDE_EMPTY) return;
            T dd = box_d2<T>(make_float4(a, b, c, 0.f), make_float4(d, e, f, 0.f), p);
            if (pick == WIDE_EMPTY || dd < best) {
                best = dd;
                pick = ref;
            }
        };
        consider(lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, ch.x);
        consider(lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, ch.y);
        consider(lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, ch.z);
        consider(lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, ch.w);
        r.nbox += 4;
        if (pick == WIDE_EMPTY) break;
        if (pick < 0) {
            visit_leaf(r, bv, ids, p, ~pick);
            break;
        }
        x = pick;
    }
}

template <class T, class Stack>
HD_D QueryResult<T> traverse(const NodeSrc &nodes, const BView<T> &bv, const int4 *__restrict__ ids, const V3<T> &p,
                             int root, Stack &st, QueryResult<T> r) {
    const T slack = T(1) + T(16 * Prec<T>::u);
    const T inf = T(__builtin_inf());
    if (root < 0) {
        visit_leaf(r, bv, ids, p, ~root);
        return r;
    }
    // Without a bound every child is in range and every sibling would be
    // pushed; descend greedily first (see greedy_probe).
    if (!(r.d2 < T(__builtin_inf()))) greedy_probe(nodes, bv, ids, p, root, r);
    int node = root;
    bool lost = false;
    int restarts = 0;
    while (true) {
        const WideView w = load_wide(nodes, node);
        const float4 lx = w.lx, ly = w.ly, lz = w.lz, hx = w.hx, hy = w.hy, hz = w.hz;
        const int4 ch = w.ch;
        T e0 = box_d2<T>(make_float4(lx.x, ly.x, lz.x, 0.f), make_float4(hx.x, hy.x, hz.x, 0.f), p);
        T e1 = box_d2<T>(make_float4(lx.y, ly.y, lz.y, 0.f), make_float4(hx.y, hy.y, hz.y, 0.f), p);
        T e2 = box_d2<T>(make_float4(lx.z, ly.z, lz.z, 0.f), make_float4(hx.z, hy.z, hz.z, 0.f), p);
        T e3 = box_d2<T>(make_float4(lx.w, ly.w, lz.w, 0.f), make_float4(hx.w, hy.w, hz.w, 0.f), p);
        int f0 = ch.x, f1 = ch.y, f2 = ch.z, f3 = ch.w;
        r.nbox += (f0 != WIDE_EMPTY) + (f1 != WIDE_EMPTY) + (f2 != WIDE_EMPTY) + (f3 != WIDE_EMPTY);
        // leaves in range: their frames are loaded together (independent
        // loads in flight at once), then folded in slot order
        {
            const T thr = r.d2 * slack;
            const bool l0 = f0 < 0 && f0 != WIDE_EMPTY && e0 <= thr, l1 = f1 < 0 && f1 != WIDE_EMPTY && e1 <= thr,
                       l2 = f2 < 0 && f2 != WIDE_EMPTY && e2 <= thr, l3 = f3 < 0 && f3 != WIDE_EMPTY && e3 <= thr;
            if constexpr (sizeof(T) == 8 || LEAF_BATCH == 1) {
                // (FP64 frames are twice the size: one at a time)
                if (l0) visit_leaf(r, bv, ids, p, ~f0);
                if (l1 && e1 <= r.d2 * slack) visit_leaf(r, bv, ids, p, ~f1);
                if (l2 && e2 <= r.d2 * slack) visit_leaf(r, bv, ids, p, ~f2);
                if (l3 && e3 <= r.d2 * slack) visit_leaf(r, bv, ids, p, ~f3);
            } else if constexpr (LEAF_BATCH == 2) {
                if (l0 || l1) {
                    Frame<T> F0, F1;
                    if (l0) F0 = load_frame(bv.frames, ~f0);
                    if (l1) F1 = load_frame(bv.frames, ~f1);
                    if (l0) fold_leaf(r, F0, p, ~f0);
                    if (l1 && e1 <= r.d2 * slack) fold_leaf(r, F1, p, ~f1);
                }
                const bool m2 = l2 && e2 <= r.d2 * slack, m3 = l3 && e3 <= r.d2 * slack;
                if (m2 || m3) {
                    Frame<T> F2, F3;
                    if (m2) F2 = load_frame(bv.frames, ~f2);
                    if (m3) F3 = load_frame(bv.frames, ~f3);
                    if (m2) fold_leaf(r, F2, p, ~f2);
                    if (m3 && e3 <= r.d2 * slack) fold_leaf(r, F3, p, ~f3);
                }
            } else if (l0 || l1 || l2 || l3) {
                Frame<T> F0, F1, F2, F3;
                if (l0) F0 = load_frame(bv.frames, ~f0);
                if (l1) F1 = load_frame(bv.frames, ~f1);
                if (l2) F2 = load_frame(bv.frames, ~f2);
                if (l3) F3 = load_frame(bv.frames, ~f3);
                if (l0) fold_leaf(r, F0, p, ~f0);
                if (l1 && e1 <= r.d2 * slack) fold_leaf(r, F1, p, ~f1);
                if (l2 && e2 <= r.d2 * slack) fold_leaf(r, F2, p, ~f2);
                if (l3 && e3 <= r.d2 * slack) fold_leaf(r, F3, p, ~f3);
            }
        }
        // internal children in range, nearest first
        const T thr = r.d2 * slack;
        auto keep = [&](T &e, int &f) {
            if (!(f >= 0 && e <= thr)) {
                e = inf;
                f = -1;
            }
        };
        keep(e0, f0);
        keep(e1, f1);
        keep(e2, f2);
        keep(e3, f3);
        cswap(e0, f0, e1, f1);
        cswap(e2, f2, e3, f3);
        cswap(e0, f0, e2, f2);
        cswap(e1, f1, e3, f3);
        cswap(e1, f1, e2, f2);
        if (f0 >= 0) {
            if (f3 >= 0 && !st.push(f3, to_float_down(e3))) lost = true;
            if (f2 >= 0 && !st.push(f2, to_float_down(e2))) lost = true;
            if (f1 >= 0 && !st.push(f1, to_float_down(e1))) lost = true;
            node = f0;
            continue;
        }
        bool found = false;
        int n;
        float dn;
        while (st.pop(n, dn)) {
            if (T(dn) <= r.d2 * slack) {
                node = n;
                found = true;
                break;
            }
        }
        if (!found) {
            if (!lost) break;
            // entries were dropped: visit the tree again with the bound found
            if (++restarts > MAX_RESTARTS) {
                r.overflow = true;
                break;
            }
            lost = false;
            st.clear();
            node = root;
        }
    }
    return r;
}

// ---------------------------------------------------------------------------
// Four lanes per query. A quad (four consecutive lanes of a wave) runs one
// traversal: lane k tests child slot k of each wide node and evaluates that
// child when it is a triangle in range; quad permutes (DPP, no LDS) then give
// every lane of the quad the same view of the four children, and the lanes
// take identical decisions (next node, stack entries), so the quad stays in
// step. Per node this spreads the box tests and the closest-point
// evaluations over four lanes, and a launch of the same queries holds four
// times as many waves to hide the latency of the dependent node loads.
// Every quad-level helper below must be called by all four lanes of a quad.
// ---------------------------------------------------------------------------
template <int CTRL> HD_D int dpp_i32(int x) { return __builtin_amdgcn_mov_dpp(x, CTRL, 0xf, 0xf, false); }
template <int CTRL, class X> HD_D X dpp(X x) {
    if constexpr (sizeof(X) == 4) {
        return __builtin_bit_cast(X, dpp_i32<CTRL>(__builtin_bit_cast(int, x)));
    } else {
        static_assert(sizeof(X) == 8, "4- or 8-byte values");
        const unsigned long long v = __builtin_bit_cast(unsigned long long, x);
        const int lo = dpp_i32<CTRL>((int)(unsigned)v), hi = dpp_i32<CTRL>((int)(unsigned)(v >> 32));
        return __builtin_bit_cast(X, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    }
}
// quad_perm controls: lane j of the quad to all four lanes; xor 1; xor 2
template <int J, class X> HD_D X quad_bcast(X x) { return dpp<J * 0x55>(x); }
template <class X> HD_D X quad_xor1(X x) { return dpp<0xB1>(x); }
template <class X> HD_D X quad_xor2(X x) { return dpp<0x4E>(x); }
HD_D bool quad_any(bool b) { return ((__ballot(b) >> (__lane_id() & ~3u)) & 0xfull) != 0; }

// every lane of the quad takes the quad's best (d2, triangle), exact ties to
// the smallest original index; the counters stay per lane
template <class T> HD_D void quad_min(QueryResult<T> &r) {
    {
        const T d2 = quad_xor1(r.d2);
        const int s = quad_xor1(r.s), o = quad_xor1(r.orig);
        if (d2 < r.d2 || (d2 == r.d2 && o < r.orig)) {
            r.d2 = d2;
            r.s = s;
            r.orig = o;
        }
    }
    {
        const T d2 = quad_xor2(r.d2);
        const int s = quad_xor2(r.s), o = quad_xor2(r.orig);
        if (d2 < r.d2 || (d2 == r.d2 && o < r.orig)) {
            r.d2 = d2;
            r.s = s;
            r.orig = o;
        }
    }
}

// the quad's short stack in LDS: entries [slot][quad of block]; all four
// lanes hold the same top / count and write the same values
template <int SD, int NQ> struct QuadStack {
    int *node;
    float *dist;
    int col;
    int top = 0, cnt = 0;
    HD_D bool push(int n, float d) {
        node[top * NQ + col] = n;
        dist[top * NQ + col] = d;
        top = top + 1 == SD ? 0 : top + 1;
        if (cnt == SD) return false;
        ++cnt;
        return true;
    }
    HD_D bool pop(int &n, float &d) {
        if (cnt == 0) return false;
        top = top == 0 ? SD - 1 : top - 1;
        --cnt;
        n = node[top * NQ + col];
        d = dist[top * NQ + col];
        return true;
    }
    HD_D void clear() { top = cnt = 0; }
};


// lane k's child of wide node x: box distance, reference
template <class T, class F, class I> HD_D T slot_box_d2(F *b, I *c, int k, const V3<T> &p, int &ref) {
    ref = c[24 + k];
    return box_d2<T>(make_float4(b[k], b[4 + k], b[8 + k], 0.f), make_float4(b[12 + k], b[16 + k], b[20 + k], 0.f), p);
}
template <class T> HD_D T slot_box_d2(const NodeSrc &ns, int x, int k, const V3<T> &p, int &ref) {
    if (x >= TOP_REF) {
        LdsFloat *b = ns.top + WIDE_WORDS * (x - TOP_REF);
        return slot_box_d2<T>(b, (LdsInt *)b, k, p, ref);
    }
    const float *b = reinterpret_cast<const float *>(ns.g + x);
    return slot_box_d2<T>(b, reinterpret_cast<const int *>(b), k, p, ref);
}

// The traversal of `traverse` (same pruning, same order of descent, same
// ring stack with restarts) run by a quad; k = lane within the quad. The
// result (d2, s, orig, overflow) is the same on all four lanes; nbox and
// nleaf count each lane's own tests.
template <class T, class Stack>
HD_D QueryResult<T> traverse4(const NodeSrc &nodes, const BView<T> &bv, const int4 *__restrict__ ids, const V3<T> &p,
                              int root, Stack &st, QueryResult<T> r, int k) {
    const T slack = T(1) + T(16 * Prec<T>::u);
    const T inf = T(__builtin_inf());
    if (root < 0) {
        if (k == 0) visit_leaf(r, bv, ids, p, ~root);
        quad_min(r);
        return r;
    }
    if (!(r.d2 < inf)) {
        // greedy probe: nearest box first down to one leaf, nothing pushed
        int x = root;
        for (int guard = 0; guard < 64 && x >= 0; ++guard) {
            int ref;
            const T dd = slot_box_d2<T>(nodes, x, k, p, ref);
            r.nbox += ref != WIDE_EMPTY;
            const T d0 = quad_bcast<0>(dd), d1 = quad_bcast<1>(dd), d2 = quad_bcast<2>(dd), d3 = quad_bcast<3>(dd);
            const int c0 = quad_bcast<0>(ref), c1 = quad_bcast<1>(ref), c2 = quad_bcast<2>(ref),
                      c3 = quad_bcast<3>(ref);
            T best = inf;
            int pick = WIDE_EMPTY, slot = -1;
            auto consider = [&](T d, int c, int j) {
                if (c == WIDE_EMPTY) return;
                if (pick == WIDE_EMPTY || d < best) {
                    best = d;
                    pick = c;
                    slot = j;
                }
            };
            consider(d0, c0, 0);
            consider(d1, c1, 1);
            consider(d2, c2, 2);
            consider(d3, c3, 3);
            if (pick == WIDE_EMPTY) break;
            if (pick < 0) {
                if (k == slot) visit_leaf(r, bv, ids, p, ~pick);
                quad_min(r);
                break;
            }
            x = pick;
        }
    }
    int node = root;
    bool lost = false;
    int restarts = 0;
    while (true) {
        int f;
        const T e = slot_box_d2<T>(nodes, node, k, p, f);
        r.nbox += f != WIDE_EMPTY;
        // triangles in range: each lane its own, then the quad's best
        const bool leaf = f < 0 && f != WIDE_EMPTY && e <= r.d2 * slack;
        if (quad_any(leaf)) {
            if (leaf) visit_leaf(r, bv, ids, p, ~f);
            quad_min(r);
        }
        // internal children in range, nearest first
        const T thr = r.d2 * slack;
        const bool in = f >= 0 && e <= thr;
        const T ei = in ? e : inf;
        const int fi = in ? f : -1;
        T e0 = quad_bcast<0>(ei), e1 = quad_bcast<1>(ei), e2 = quad_bcast<2>(ei), e3 = quad_bcast<3>(ei);
        int f0 = quad_bcast<0>(fi), f1 = quad_bcast<1>(fi), f2 = quad_bcast<2>(fi), f3 = quad_bcast<3>(fi);
        cswap(e0, f0, e1, f1);
        cswap(e2, f2, e3, f3);
        cswap(e0, f0, e2, f2);
        cswap(e1, f1, e3, f3);
        cswap(e1, f1, e2, f2);
        if (f0 >= 0) {
            if (f3 >= 0 && !st.push(f3, to_float_down(e3))) lost = true;
            if (f2 >= 0 && !st.push(f2, to_float_down(e2))) lost = true;
            if (f1 >= 0 && !st.push(f1, to_float_down(e1))) lost = true;
            node = f0;
            continue;
        }
        bool found = false;
        int n;
        float dn;
        while (st.pop(n, dn)) {
            if (T(dn) <= r.d2 * slack) {
                node = n;
                found = true;
                break;
            }
        }
        if (!found) {
            if (!lost) break;
            if (++restarts > MAX_RESTARTS) {
                r.overflow = true;
                break;
            }
            lost = false;
            st.clear();
            node = root;
        }
    }
    return r;
}

// ---------------------------------------------------------------------------
// The cascade ("Upper bounds" subsection and Implementation section): the
// exact bound when all three closest triangles coincide; otherwise the
// bounds in the requested order, stopping at the first that falls below the
// lower bound L (discard), else the minimum of all of them.
// ---------------------------------------------------------------------------
struct CascadeCtx {
    int order[5]; // bounds 1..4, and 5 (the bound of Zheng et al., which needs the barycenter's query)
    int norder;
};

template <class T> HD_D double tri_margin(const Tri<T> &t, const Margins &m) {
    double dmax = (double)hmax(t.d[0], hmax(t.d[1], t.d[2]));
    double e = (double)hmax(norm2(t.v[0] - t.v[1]), hmax(norm2(t.v[1] - t.v[2]), norm2(t.v[2] - t.v[0])));
    return m.mu_d * dmax + m.mu_e * sqrt(e) + m.mu_0;
}

// FP64 recomputation of a frontier triangle: exact vertex positions, FP64
// distances to the recorded closest triangles (any point of B gives a valid
// upper-bound distance), then the full minimum over the bounds in the order
// set. Returns the bound with the FP64 margin.
HD_D double rebound64(const AView &a, int pair, int32_t face, int lvl, const int ba[3], const int bb[3],
                      const int I[3], const BView<double> &bv64, const IdView &iv, const CascadeCtx &c,
                      const Margins &m64, int *evals) {
    Tri<double> t;
    for (int i = 0; i < 3; ++i) {
        t.v[i] = a_point(a, pair, face, lvl, ba[i], bb[i]);
        t.I[i] = I[i];
        Frame<double> f = load_frame(bv64.frames, I[i]);
        V3<double> q;
        t.d[i] = sqrt(frame_dist2<double, true>(f, t.v[i], &q));
        t.q[i] = q;
    }
    *evals += 3;
    double mu = tri_margin(t, m64);
    if (t.I[0] == t.I[1] && t.I[1] == t.I[2]) return hmax(t.d[0], hmax(t.d[1], t.d[2])) + mu;
    // the minimum over the bounds in the set does not depend on their order
    // (the fifth bound needs a point query of the barycenter, which this
    // re-bound does not make: the minimum of the others is still a bound, and
    // u2 stands in when the fifth is the only one)
    unsigned used = 0;
    for (int i = 0; i < c.norder; ++i) used |= 1u << c.order[i];
    used &= 0x1eu;
    if (!used) used = 4u;
    double best = __builtin_inf();
    if (used & 2u) best = hmin(best, bound_u1(t));
    if (used & 4u) best = hmin(best, bound_u2(t));
    if (used & 16u) best = hmin(best, bound_u4(t));
    if (used & 8u) best = hmin(best, bound_u3(t, bv64, iv, nullptr, evals));
    return best + mu;
}

} // namespace hd
