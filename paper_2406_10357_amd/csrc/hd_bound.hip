// hd_bound.hip -- the branch-and-bound rounds on the GPU and the C ABI.
//
// Round 0 queries every referenced vertex of A, raises the lower bound L
// (eq. hausdorff_distance: every vertex distance is a lower bound of h) and
// bounds every face of A. Each later round takes the active frontier (upper
// bound above L + eps), optionally the sub-batch with the largest upper
// bounds, splits every selected triangle 1->4 at its edge midpoints, queries
// the three midpoints, raises L, bounds the four children with the cascade
// and compacts them into active (to subdivide), parked (within eps of L: kept
// for U, never subdivided) or discarded (below L). The loop ends when no
// triangle is active; then U - L <= eps (Branch and bound subsection). The
// final step re-evaluates L at the best vertex and the parked triangles'
// bounds in FP64.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <functional>

#include "hd_kernels.hpp"

namespace hd {

namespace {

constexpr int QBLOCK = 128;   // query kernel block
constexpr int QSTACK = 24;    // LDS stack entries per lane
constexpr int DEEP_STACK = 256;
constexpr int BLK = 256;

struct DevState {
    unsigned long long queries, evals, boxes, bounded, subdivided;
    unsigned long long discards[5];
    unsigned long long rechecked, overflows, q_leaves, q_boxes;
    unsigned long long Lord;      // ordered double: certified lower bound
    unsigned long long Uord;      // ordered double: upper bound of the final step
    unsigned long long round_key; // (ordered float of d_lo) << 32 | ~query index
    unsigned long long best_key;
    unsigned long long bbox[6];   // ordered FP64 bbox of A's referenced vertices (centred)
    unsigned long long coord_max; // ordered FP64
    int bad;
    int n_overflow;
    int argmax_dirty;
    double argmax_pos[3];
    double L64;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ void wave_add(unsigned long long *ctr, unsigned long long v) {
    v = wave_sum_u64(v);
    if (__lane_id() == 0 && v) atomicAdd(ctr, v);
}

__global__ void k_state_init(DevState *st) {
    memset(st, 0, sizeof(DevState));
    st->Lord = d2ord(0.0);
    st->Uord = d2ord(0.0);
    for (int k = 0; k < 3; ++k) {
        st->bbox[k] = d2ord(__builtin_inf());
        st->bbox[3 + k] = d2ord(-__builtin_inf());
    }
    st->coord_max = d2ord(0.0);
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// validate A, mark referenced vertices, bbox and coordinate range
__global__ void k_ingest_A(const double *__restrict__ V, int64_t m, const int32_t *__restrict__ F, int64_t n,
                           double cx, double cy, double cz, int32_t *__restrict__ ref, DevState *st) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    const double c[3] = {cx, cy, cz};
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    double cm = 0;
    for (int j = 0; j < 3; ++j) {
        int32_t v = F[3 * f + j];
        if (v < 0 || v >= m) {
            st->bad = 1;
            return;
        }
        ref[v] = 1;
        for (int k = 0; k < 3; ++k) {
            double x = V[3 * (int64_t)v + k];
            if (!__builtin_isfinite(x)) {
                st->bad = 1;
                return;
            }
            lo[k] = fmin(lo[k], x);
            hi[k] = fmax(hi[k], x);
            cm = fmax(cm, fabs(x - c[k]));
        }
    }
    for (int k = 0; k < 3; ++k) {
        atomicMin(&st->bbox[k], d2ord(lo[k]));
        atomicMax(&st->bbox[3 + k], d2ord(hi[k]));
    }
    atomicMax(&st->coord_max, d2ord(cm));
}

// compact the referenced vertex ids (order preserving)
__global__ void k_ref_scatter(const int32_t *__restrict__ ref, const int32_t *__restrict__ pos, int64_t m,
                              int32_t *__restrict__ out) {
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < m && ref[v]) out[pos[v]] = (int32_t)v;
}

// ---------------------------------------------------------------------------
// point queries
// ---------------------------------------------------------------------------
enum QMode { Q_POINTS = 0, Q_VERTICES = 1, Q_MIDPOINTS = 2 };

template <class T> struct QueryOut {
    T *d;
    int *I;
    T *q[3];
    T *p[3]; // query position (precision T), reused by the children kernel
};

struct QueryIn {
    int mode;
    const double *P;      // Q_POINTS: n x 3, uncentred
    const int32_t *vids;  // Q_VERTICES: referenced vertex ids
    AView a;              // Q_VERTICES / Q_MIDPOINTS
    const int *face, *lvl, *ba[3], *bb[3]; // Q_MIDPOINTS: selected parents
    double cx, cy, cz;    // centre
};

HD_D V3<double> query_point64(const QueryIn &in, int64_t i) {
    if (in.mode == Q_POINTS)
        return {in.P[3 * i] - in.cx, in.P[3 * i + 1] - in.cy, in.P[3 * i + 2] - in.cz};
    if (in.mode == Q_VERTICES) return a_vertex(in.a, in.vids[i]);
    int64_t j = i / 3;
    int e = (int)(i - 3 * j);
    int k = (e + 1) % 3;
    return a_point(in.a, in.face[j], in.lvl[j] + 1, in.ba[e][j] + in.ba[k][j], in.bb[e][j] + in.bb[k][j]);
}

struct QueryCfg {
    const NodeRec *nodes;
    const int4 *ids;
    Margins m;
    int raise_L; // fold d - mu into the lower bound and the argmax key
};

template <class T>
HD_D void finish_query(const QueryCfg &cfg, const BView<T> &bv, const QueryResult<T> &r, const V3<T> &p,
                       int64_t i, const QueryOut<T> &out, DevState *st) {
    V3<T> q = p;
    T d = T(__builtin_inf());
    if (r.s >= 0) {
        Frame<T> f = load_frame(bv.frames, r.s);
        d = hsqrt(frame_dist2<T, true>(f, p, &q));
    }
    out.d[i] = d;
    out.I[i] = r.s;
    out.q[0][i] = q.x;
    out.q[1][i] = q.y;
    out.q[2][i] = q.z;
    if (out.p[0]) {
        out.p[0][i] = p.x;
        out.p[1][i] = p.y;
        out.p[2][i] = p.z;
    }
    if (cfg.raise_L && r.s >= 0) {
        double dlo = (double)d - (cfg.m.mu_d * (double)d + cfg.m.mu_0);
        if (dlo > 0) {
            atomicMax(&st->Lord, d2ord(dlo));
            unsigned long long key =
                ((unsigned long long)f2ord(to_float_down(dlo)) << 32) | (unsigned long long)(0xffffffffu - (uint32_t)i);
            atomicMax(&st->round_key, key);
        }
    }
}

template <class T>
__global__ __launch_bounds__(QBLOCK) void k_query(QueryIn in, int64_t n, QueryCfg cfg, BView<T> bv,
                                                  QueryOut<T> out, DevState *st, int32_t *ovf_list) {
    __shared__ int s_node[QSTACK * QBLOCK];
    __shared__ float s_dist[QSTACK * QBLOCK];
    int64_t i = (int64_t)blockIdx.x * QBLOCK + threadIdx.x;
    unsigned long long nb = 0, nl = 0, nq = 0;
    if (i < n) {
        V3<T> p = cvt<T>(query_point64(in, i));
        LdsStack<QSTACK, QBLOCK> stk{s_node, s_dist, 0};
        QueryResult<T> r = traverse<T>(cfg.nodes, bv, cfg.ids, p, stk);
        nb = r.nbox;
        nl = r.nleaf;
        nq = 1;
        if (r.overflow) {
            int k = atomicAdd(&st->n_overflow, 1);
            ovf_list[k] = (int32_t)i;
        } else {
            finish_query<T>(cfg, bv, r, p, i, out, st);
        }
    }
    wave_add(&st->boxes, nb);
    wave_add(&st->evals, nl);
    wave_add(&st->q_leaves, nl);
    wave_add(&st->q_boxes, nb);
    wave_add(&st->queries, nq);
}

// queries whose LDS stack overflowed, redone with a deep stack in global memory
template <class T>
__global__ void k_query_deep(QueryIn in, QueryCfg cfg, BView<T> bv, QueryOut<T> out, DevState *st,
                             const int32_t *ovf_list, int2 *stack_mem, int64_t nslots) {
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int novf = st->n_overflow;
    unsigned long long nb = 0, nl = 0;
    if (k < novf && k < nslots) {
        int64_t i = ovf_list[k];
        V3<T> p = cvt<T>(query_point64(in, i));
        GlobalStack stk{stack_mem + k, nslots, DEEP_STACK, 0};
        QueryResult<T> r = traverse<T>(cfg.nodes, bv, cfg.ids, p, stk);
        nb = r.nbox;
        nl = r.nleaf;
        // a traversal deeper than the fallback stack flags the run as failed;
        // its (possibly suboptimal) result is still written so that later
        // kernels read initialised indices
        if (r.overflow) st->bad = 2;
        finish_query<T>(cfg, bv, r, p, i, out, st);
    }
    wave_add(&st->boxes, nb);
    wave_add(&st->evals, nl);
}

// after a query kernel: keep the FP64 position of the best vertex so far
__global__ void k_argmax_update(QueryIn in, DevState *st) {
    unsigned long long key = st->round_key;
    if (key > st->best_key) {
        st->best_key = key;
        int64_t i = (int64_t)(0xffffffffu - (uint32_t)(key & 0xffffffffull));
        V3<double> p = query_point64(in, i);
        st->argmax_pos[0] = p.x;
        st->argmax_pos[1] = p.y;
        st->argmax_pos[2] = p.z;
        st->argmax_dirty = 1;
    }
    st->round_key = 0;
}

// ---------------------------------------------------------------------------
// bounding children (or round-0 faces) and classifying them
// ---------------------------------------------------------------------------
struct ClassifyCfg {
    CascadeCtx c;
    int recheck; // FP32 + FP64 recheck of the ambiguity band
    AView a;
    BView<double> bv64;
    Margins m64;
    IdView iv;
};

template <class T> struct Corner {
    V3<T> v, q;
    T d;
    int I, ba, bb;
};

// bound one triangle, write its record at slot `o`, return its class
// (0 discard, 1 park, 2 active) and the bound that decided it
template <class T>
HD_D int bound_and_write(const Corner<T> cn[3], int face, int lvl, const ClassifyCfg &cc, const BView<T> &bv,
                         FrontierView<T> fo, int64_t o, int *decider, int *evals, int *rechecked) {
    Tri<T> t;
    for (int i = 0; i < 3; ++i) {
        t.v[i] = cn[i].v;
        t.q[i] = cn[i].q;
        t.d[i] = cn[i].d;
        t.I[i] = cn[i].I;
    }
    double ub = cascade<T>(t, cc.c, bv, cc.iv, decider, evals);
    const double L = cc.c.L, eps = cc.c.eps;
    const double park_lim = eps * (1.0 - 1.0 / 1024.0 / 1024.0 / 1024.0);
    if (cc.recheck) {
        // the FP32 margin might hide a discard or a park: redo in FP64
        double mu = tri_margin(t, cc.c.m);
        bool maybe_discard = ub >= L && ub - 2 * mu < L;
        bool maybe_park = ub - L > park_lim && ub - 2 * mu - L <= park_lim;
        if (maybe_discard || maybe_park) {
            int ba[3] = {cn[0].ba, cn[1].ba, cn[2].ba}, bb[3] = {cn[0].bb, cn[1].bb, cn[2].bb};
            double u64 = rebound64(cc.a, face, lvl, ba, bb, t.I, cc.bv64, cc.iv, cc.c, cc.m64, evals);
            ub = hmin(ub, u64);
            *rechecked += 1;
        }
    }
    int cls = ub < L ? 0 : (ub - L <= park_lim ? 1 : 2);
    if (cls != 0) {
        for (int i = 0; i < 3; ++i) {
            fo.v[3 * i][o] = cn[i].v.x;
            fo.v[3 * i + 1][o] = cn[i].v.y;
            fo.v[3 * i + 2][o] = cn[i].v.z;
            fo.q[3 * i][o] = cn[i].q.x;
            fo.q[3 * i + 1][o] = cn[i].q.y;
            fo.q[3 * i + 2][o] = cn[i].q.z;
            fo.d[i][o] = cn[i].d;
            fo.I[i][o] = cn[i].I;
            fo.ba[i][o] = cn[i].ba;
            fo.bb[i][o] = cn[i].bb;
        }
        float ubf = (float)ub;
        if ((double)ubf < ub) ubf = next_up(ubf);
        fo.ub[o] = ubf;
        fo.face[o] = face;
        fo.lvl[o] = lvl;
    }
    return cls;
}

struct CountOut {
    int32_t *flag_act, *flag_park;
};

template <class T>
HD_D void tally(DevState *st, int cls, int decider, int evals, int rechecked, bool valid) {
    unsigned long long dis[5] = {0, 0, 0, 0, 0};
    if (valid && cls == 0) dis[decider] = 1;
    for (int k = 0; k < 5; ++k) wave_add(&st->discards[k], dis[k]);
    wave_add(&st->evals, valid ? (unsigned long long)evals : 0ull);
    wave_add(&st->rechecked, valid ? (unsigned long long)rechecked : 0ull);
    wave_add(&st->bounded, valid ? 1ull : 0ull);
}

// round 0: every face of A from the per-vertex query results
template <class T>
__global__ void k_faces_round0(int64_t nA, const int32_t *__restrict__ FA, QueryOut<T> vq, ClassifyCfg cc,
                               BView<T> bv, FrontierView<T> fo, CountOut co, const DevState *stc, DevState *st) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = f < nA;
    int cls = 0, decider = 0, evals = 0, rechecked = 0;
    if (valid) {
        ClassifyCfg c = cc;
        c.c.L = ord2d(stc->Lord);
        Corner<T> cn[3];
        for (int j = 0; j < 3; ++j) {
            int32_t v = FA[3 * f + j];
            cn[j].v = {vq.p[0][v], vq.p[1][v], vq.p[2][v]};
            cn[j].q = {vq.q[0][v], vq.q[1][v], vq.q[2][v]};
            cn[j].d = vq.d[v];
            cn[j].I = vq.I[v];
            cn[j].ba = (j == 1);
            cn[j].bb = (j == 2);
        }
        cls = bound_and_write<T>(cn, (int)f, 0, c, bv, fo, f, &decider, &evals, &rechecked);
        co.flag_act[f] = cls == 2;
        co.flag_park[f] = cls == 1;
    }
    tally<T>(st, cls, decider, evals, rechecked, valid);
}

// round k: child c of selected parent c/4, from the parent's record and the
// three midpoint query results (midpoint e joins parent vertices e and e+1)
template <class T>
__global__ void k_children(int64_t nsel, FrontierView<T> par, QueryOut<T> mq, ClassifyCfg cc, BView<T> bv,
                           FrontierView<T> fo, CountOut co, const DevState *stc, DevState *st) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = c < 4 * nsel;
    int cls = 0, decider = 0, evals = 0, rechecked = 0;
    if (valid) {
        ClassifyCfg cfg = cc;
        cfg.c.L = ord2d(stc->Lord);
        int64_t j = c >> 2;
        int kid = (int)(c & 3);
        // corners: 0..2 parent vertices, 3..5 midpoints m01, m12, m20
        const int kids[4][3] = {{0, 3, 5}, {3, 1, 4}, {5, 4, 2}, {3, 4, 5}};
        Corner<T> cn[3];
        for (int i = 0; i < 3; ++i) {
            int s = kids[kid][i];
            if (s < 3) {
                cn[i].v = {par.v[3 * s][j], par.v[3 * s + 1][j], par.v[3 * s + 2][j]};
                cn[i].q = {par.q[3 * s][j], par.q[3 * s + 1][j], par.q[3 * s + 2][j]};
                cn[i].d = par.d[s][j];
                cn[i].I = par.I[s][j];
                cn[i].ba = 2 * par.ba[s][j];
                cn[i].bb = 2 * par.bb[s][j];
            } else {
                int e = s - 3, e2 = (e + 1) % 3;
                int64_t mi = 3 * j + e;
                cn[i].v = {mq.p[0][mi], mq.p[1][mi], mq.p[2][mi]};
                cn[i].q = {mq.q[0][mi], mq.q[1][mi], mq.q[2][mi]};
                cn[i].d = mq.d[mi];
                cn[i].I = mq.I[mi];
                cn[i].ba = par.ba[e][j] + par.ba[e2][j];
                cn[i].bb = par.bb[e][j] + par.bb[e2][j];
            }
        }
        // dyadic coordinates are int32 numerators over 2^lvl: level 30 is the
        // deepest representable one
        if (par.lvl[j] >= 30) st->bad = 3;
        cls = bound_and_write<T>(cn, par.face[j], par.lvl[j] + 1, cfg, bv, fo, c, &decider, &evals, &rechecked);
        co.flag_act[c] = cls == 2;
        co.flag_park[c] = cls == 1;
    }
    tally<T>(st, cls, decider, evals, rechecked, valid);
}

// ---------------------------------------------------------------------------
// record movement
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_scatter_vq(QueryOut<T> src, QueryOut<T> dst, const int32_t *__restrict__ vids, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t v = vids[i];
    dst.d[v] = src.d[i];
    dst.I[v] = src.I[i];
    for (int k = 0; k < 3; ++k) {
        dst.q[k][v] = src.q[k][i];
        dst.p[k][v] = src.p[k][i];
    }
}

template <class T>
HD_D void copy_record(const FrontierView<T> &src, int64_t i, const FrontierView<T> &dst, int64_t o) {
    for (int k = 0; k < 9; ++k) {
        dst.v[k][o] = src.v[k][i];
        dst.q[k][o] = src.q[k][i];
    }
    for (int k = 0; k < 3; ++k) {
        dst.d[k][o] = src.d[k][i];
        dst.I[k][o] = src.I[k][i];
        dst.ba[k][o] = src.ba[k][i];
        dst.bb[k][o] = src.bb[k][i];
    }
    dst.ub[o] = src.ub[i];
    dst.face[o] = src.face[i];
    dst.lvl[o] = src.lvl[i];
}

// scatter flagged records of src to dst at base + exclusive-scan position
template <class T>
__global__ void k_scatter(FrontierView<T> src, int64_t n, const int32_t *__restrict__ flag,
                          const int32_t *__restrict__ pos, FrontierView<T> dst, int64_t base) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && flag[i]) copy_record(src, i, dst, base + pos[i]);
}

// dst[o] = src[perm[o] (or off + o)]
template <class T>
__global__ void k_gather(FrontierView<T> src, const int32_t *__restrict__ perm, int64_t off, int64_t n,
                         FrontierView<T> dst) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) copy_record(src, perm ? perm[o] : off + o, dst, o);
}

// sort keys: descending upper bound (stable), as unsigned ascending
__global__ void k_ub_keys(const float *__restrict__ ub, int64_t n, uint32_t *__restrict__ keys,
                          int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        keys[i] = ~f2ord(ub[i]);
        vals[i] = (int32_t)i;
    }
}

// parked records still at or above L
__global__ void k_flag_ge(const float *__restrict__ ub, int64_t n, const DevState *st, int32_t *__restrict__ flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = (double)ub[i] >= ord2d(st->Lord);
}

// ---------------------------------------------------------------------------
// final FP64 step
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_final_U(FrontierView<T> fr, int64_t n, AView a, BView<double> bv64, IdView iv, CascadeCtx c,
                          Margins m64, DevState *st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long ev = 0;
    if (i < n) {
        int ba[3] = {fr.ba[0][i], fr.ba[1][i], fr.ba[2][i]};
        int bb[3] = {fr.bb[0][i], fr.bb[1][i], fr.bb[2][i]};
        int I[3] = {fr.I[0][i], fr.I[1][i], fr.I[2][i]};
        int evals = 0;
        double u64 = rebound64(a, fr.face[i], fr.lvl[i], ba, bb, I, bv64, iv, c, m64, &evals);
        double u = hmin(u64, (double)fr.ub[i]);
        atomicMax(&st->Uord, d2ord(u));
        ev = evals;
    }
    wave_add(&st->evals, ev);
}

// FP64 distance of the best vertex found so far (when it changed): the lower
// bound then carries the FP64 margin instead of the FP32 one, which the
// recheck band needs to park triangles within eps of it
__global__ void k_L64(const NodeRec *nodes, BView<double> bv64, const int4 *ids, Margins m64, DevState *st) {
    __shared__ int s_node[DEEP_STACK];
    __shared__ float s_dist[DEEP_STACK];
    if (threadIdx.x != 0) return;
    if (st->best_key == 0 || !st->argmax_dirty) return;
    st->argmax_dirty = 0;
    V3<double> p = {st->argmax_pos[0], st->argmax_pos[1], st->argmax_pos[2]};
    LdsStack<DEEP_STACK, 1> stk{s_node, s_dist, 0};
    QueryResult<double> r = traverse<double>(nodes, bv64, ids, p, stk);
    if (r.overflow || r.s < 0) return;
    double d = sqrt(r.d2);
    double dlo = d - (m64.mu_d * d + m64.mu_0);
    st->L64 = dlo;
    if (dlo > 0) atomicMax(&st->Lord, d2ord(dlo));
}

// ---------------------------------------------------------------------------
// test entry: all five bounds of given triangles
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_eval_bounds(const double *v, const double *d, const int32_t *Iorig, const double *q, int64_t n,
                              const int32_t *inv_perm, int64_t nB, BView<T> bv, IdView iv, double cx, double cy,
                              double cz, double *out, int32_t *u3case) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) {
        int32_t f = Iorig[3 * i + k];
        if (f < 0 || f >= nB) { // caller's face index out of range
            for (int j = 0; j < 5; ++j) out[5 * i + j] = __builtin_nan("");
            u3case[i] = 0;
            return;
        }
    }
    Tri<T> t;
    const double c[3] = {cx, cy, cz};
    for (int k = 0; k < 3; ++k) {
        t.v[k] = {T(v[9 * i + 3 * k] - c[0]), T(v[9 * i + 3 * k + 1] - c[1]), T(v[9 * i + 3 * k + 2] - c[2])};
        t.q[k] = {T(q[9 * i + 3 * k] - c[0]), T(q[9 * i + 3 * k + 1] - c[1]), T(q[9 * i + 3 * k + 2] - c[2])};
        t.d[k] = T(d[3 * i + k]);
        t.I[k] = inv_perm[Iorig[3 * i + k]];
    }
    int ev = 0, cs = 0;
    out[5 * i] = (t.I[0] == t.I[1] && t.I[1] == t.I[2]) ? (double)hmax(t.d[0], hmax(t.d[1], t.d[2])) : __builtin_nan("");
    out[5 * i + 1] = bound_u1(t);
    out[5 * i + 2] = bound_u2(t);
    out[5 * i + 3] = bound_u3(t, bv, iv, &cs, &ev);
    out[5 * i + 4] = bound_u4(t);
    u3case[i] = cs;
}

__global__ void k_inv_perm(const int4 *ids, int64_t n, int32_t *inv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[ids[i].w] = (int32_t)i;
}

template <class T>
__global__ void k_export_points(const QueryOut<T> r, int64_t n, const int4 *ids, double cx, double cy, double cz,
                                double *d, int32_t *I, double *Q) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    d[i] = (double)r.d[i];
    I[i] = r.I[i] >= 0 ? ids[r.I[i]].w : -1;
    if (Q) {
        Q[3 * i] = (double)r.q[0][i] + cx;
        Q[3 * i + 1] = (double)r.q[1][i] + cy;
        Q[3 * i + 2] = (double)r.q[2][i] + cz;
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
template <class T> struct Frontier {
    DBuf mem;
    int64_t cap = 0;
    FrontierView<T> v;
    void alloc(int64_t c) {
        size_t per = 21 * sizeof(T) + 12 * sizeof(int32_t);
        mem.reserve((size_t)c * per + 64 * 256);
        cap = c;
        char *p = mem.as<char>();
        auto take = [&](size_t sz) {
            char *r = p;
            p += ((size_t)c * sz + 255) & ~size_t(255);
            return r;
        };
        for (int k = 0; k < 9; ++k) v.v[k] = (T *)take(sizeof(T));
        for (int k = 0; k < 9; ++k) v.q[k] = (T *)take(sizeof(T));
        for (int k = 0; k < 3; ++k) v.d[k] = (T *)take(sizeof(T));
        for (int k = 0; k < 3; ++k) v.I[k] = (int *)take(4);
        v.ub = (float *)take(4);
        v.face = (int *)take(4);
        v.lvl = (int *)take(4);
        for (int k = 0; k < 3; ++k) v.ba[k] = (int *)take(4);
        for (int k = 0; k < 3; ++k) v.bb[k] = (int *)take(4);
    }
};

template <class T> void swap_frontier(Frontier<T> &a, Frontier<T> &b) {
    std::swap(a.mem.p, b.mem.p);
    std::swap(a.mem.bytes, b.mem.bytes);
    std::swap(a.cap, b.cap);
    std::swap(a.v, b.v);
}

template <class T> struct QBuf {
    DBuf mem;
    QueryOut<T> o;
    void alloc(int64_t n, bool with_p) {
        mem.reserve((size_t)n * (sizeof(T) * 7 + 4) + 16 * 256);
        char *p = mem.as<char>();
        auto take = [&](size_t sz) {
            char *r = p;
            p += ((size_t)n * sz + 255) & ~size_t(255);
            return r;
        };
        o.d = (T *)take(sizeof(T));
        o.I = (int *)take(4);
        for (int k = 0; k < 3; ++k) o.q[k] = (T *)take(sizeof(T));
        for (int k = 0; k < 3; ++k) o.p[k] = with_p ? (T *)take(sizeof(T)) : nullptr;
    }
};

Margins make_margins(double u, const Bvh *b, double coord_max) {
    Margins m;
    m.mu_d = 16 * u;
    m.mu_e = 48 * u;
    m.mu_0 = u * (48 * b->edge_max + 12 * coord_max);
    return m;
}

int parse_order(int32_t order, int out[4]) {
    if (order <= 0) order = 1234;
    int digits[8], n = 0;
    while (order > 0 && n < 8) {
        digits[n++] = order % 10;
        order /= 10;
    }
    if (order > 0 || n > 4) return -1;
    int used = 0;
    for (int i = 0; i < n; ++i) {
        int k = digits[n - 1 - i];
        if (k < 1 || k > 4 || (used >> k) & 1) return -1;
        used |= 1 << k;
        out[i] = k;
    }
    return n;
}

struct Runner {
    hipStream_t s;
    const Bvh *b;
    DBuf st_mem;
    DevState *st;
    DBuf scan_tmp, sort_tmp, ovf_mem, deep_stack;
    BView<double> bv64{};
    Margins m64{};
    // optional kernel timing with events on the call's stream
    bool profile = false;
    std::vector<hipEvent_t> qev, cev; // begin/end pairs
    hipEvent_t mark(std::vector<hipEvent_t> &v) {
        hipEvent_t e = nullptr;
        if (!profile) return e;
        HD_HIP(hipEventCreate(&e));
        HD_HIP(hipEventRecord(e, s));
        v.push_back(e);
        return e;
    }
    static double sum_pairs(std::vector<hipEvent_t> &v) {
        double ms = 0;
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float t = 0;
            if (hipEventElapsedTime(&t, v[i], v[i + 1]) == hipSuccess) ms += t;
        }
        return ms;
    }
    ~Runner() {
        for (auto e : qev) (void)hipEventDestroy(e);
        for (auto e : cev) (void)hipEventDestroy(e);
    }

    template <class T>
    void queries(const QueryIn &in, int64_t n, const QueryCfg &cfg, const BView<T> &bv, const QueryOut<T> &out,
                 int64_t *overflows) {
        if (n <= 0) return;
        ovf_mem.reserve((size_t)n * sizeof(int32_t));
        k_fill_i32<<<1, 1, 0, s>>>((int32_t *)&st->n_overflow, 1, 0);
        mark(qev);
        k_query<T><<<grid_for(n, QBLOCK), QBLOCK, 0, s>>>(in, n, cfg, bv, out, st, ovf_mem.as<int32_t>());
        HD_LAUNCH_CHECK();
        mark(qev);
        int novf = 0;
        HD_HIP(hipMemcpyAsync(&novf, &st->n_overflow, sizeof(int), hipMemcpyDeviceToHost, s));
        HD_HIP(hipStreamSynchronize(s));
        if (novf > 0) {
            *overflows += novf;
            deep_stack.reserve((size_t)novf * DEEP_STACK * sizeof(int2));
            k_query_deep<T><<<grid_for(novf, 64), 64, 0, s>>>(in, cfg, bv, out, st, ovf_mem.as<int32_t>(),
                                                              deep_stack.as<int2>(), novf);
            HD_LAUNCH_CHECK();
        }
        if (cfg.raise_L) {
            k_argmax_update<<<1, 1, 0, s>>>(in, st);
            k_L64<<<1, 64, 0, s>>>(cfg.nodes, bv64, cfg.ids, m64, st);
        }
        HD_LAUNCH_CHECK();
    }
};

// compact flagged records of src (n of them) into dst starting at base;
// returns how many were written
template <class T>
int64_t compact(Runner &R, const FrontierView<T> &src, int64_t n, const int32_t *flag, int32_t *pos,
                int32_t *d_total, const FrontierView<T> &dst, int64_t base) {
    if (n <= 0) return 0;
    scan_exclusive_i32(flag, pos, n, d_total, R.scan_tmp, R.s);
    k_scatter<T><<<grid_for(n, BLK), BLK, 0, R.s>>>(src, n, flag, pos, dst, base);
    HD_LAUNCH_CHECK();
    int32_t tot = 0;
    HD_HIP(hipMemcpyAsync(&tot, d_total, sizeof(int32_t), hipMemcpyDeviceToHost, R.s));
    HD_HIP(hipStreamSynchronize(R.s));
    return tot;
}

template <class T>
hd_status bound_impl(const double *VA, int64_t mA, const int32_t *FA, int64_t nA, const Bvh *B, double eps,
                     const hd_options &opt, hipStream_t s, double LU[2], hd_stats *stats) {
    auto t0 = std::chrono::steady_clock::now();
    Runner R;
    R.s = s;
    R.b = B;
    R.profile = opt.profile != 0;
    R.st_mem.reserve(sizeof(DevState));
    R.st = R.st_mem.as<DevState>();
    DevState *st = R.st;
    hd_stats S;
    std::memset(&S, 0, sizeof(S));

    CascadeCtx cctx;
    cctx.norder = parse_order(opt.order, cctx.order);
    if (cctx.norder <= 0) throw Error{HD_E_INVALID, "bad cascade order"};

    // ---- ingest A ---------------------------------------------------------
    DBuf ref_mem;
    ref_mem.reserve((size_t)mA * 2 * sizeof(int32_t) + 512);
    int32_t *ref = ref_mem.as<int32_t>();
    int32_t *refpos = ref + ((mA + 63) / 64) * 64;
    DBuf small;
    small.reserve(4096);
    int32_t *d_total = small.as<int32_t>();
    k_state_init<<<1, 1, 0, s>>>(st);
    k_fill_i32<<<grid_for(mA, BLK), BLK, 0, s>>>(ref, mA, 0);
    k_ingest_A<<<grid_for(nA, BLK), BLK, 0, s>>>(VA, mA, FA, nA, B->center[0], B->center[1], B->center[2], ref, st);
    HD_LAUNCH_CHECK();
    DevState hs;
    HD_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HD_HIP(hipStreamSynchronize(s));
    if (hs.bad) throw Error{HD_E_INVALID, "soup A has an out-of-range index or a non-finite coordinate"};
    double diag2 = 0;
    for (int k = 0; k < 3; ++k) {
        double e = ord2d(hs.bbox[3 + k]) - ord2d(hs.bbox[k]);
        diag2 += e * e;
    }
    S.dA = sqrt(diag2);
    S.eps_abs = eps * S.dA;
    cctx.eps = S.eps_abs;
    double coord_max = std::max(ord2d(hs.coord_max), B->coord_max);
    Margins m = make_margins(Prec<T>::u, B, coord_max);
    Margins m64 = make_margins(Prec<double>::u, B, coord_max);
    cctx.m = m;
    cctx.mu64_0 = m64.mu_0;
    R.bv64 = BView<double>{B->frames64.as<double2>()};
    R.m64 = m64;
    S.mu_coef_d = m.mu_d;
    S.mu_coef_0 = m.mu_0;

    // referenced vertices, in order
    scan_exclusive_i32(ref, refpos, mA, d_total, R.scan_tmp, s);
    int32_t nref = 0;
    HD_HIP(hipMemcpyAsync(&nref, d_total, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HD_HIP(hipStreamSynchronize(s));
    DBuf vids_mem;
    vids_mem.reserve((size_t)nref * sizeof(int32_t));
    k_ref_scatter<<<grid_for(mA, BLK), BLK, 0, s>>>(ref, refpos, mA, vids_mem.as<int32_t>());

    const BView<T> bv = [&] {
        if constexpr (sizeof(T) == 4) return BView<float>{B->frames32.as<float4>()};
        else return BView<double>{B->frames64.as<double2>()};
    }();
    const BView<double> bv64{B->frames64.as<double2>()};
    IdView iv{B->ids.as<int4>()};
    AView av{VA, FA, B->center[0], B->center[1], B->center[2]};
    QueryCfg qcfg{B->nodes.as<NodeRec>(), B->ids.as<int4>(), m, 1};

    // per-vertex results, indexed by vertex id (only referenced ones are set)
    QBuf<T> vq;
    vq.alloc(mA, true);
    {
        // query the referenced vertices; results land at their vertex id
        QBuf<T> tmp;
        tmp.alloc(nref, true);
        QueryIn in{};
        in.mode = Q_VERTICES;
        in.vids = vids_mem.as<int32_t>();
        in.a = av;
        in.cx = B->center[0];
        in.cy = B->center[1];
        in.cz = B->center[2];
        R.queries<T>(in, nref, qcfg, bv, tmp.o, &S.stack_overflows);
        // scatter to vertex ids
        k_scatter_vq<T><<<grid_for(nref, BLK), BLK, 0, s>>>(tmp.o, vq.o, vids_mem.as<int32_t>(), (int64_t)nref);
        HD_LAUNCH_CHECK();
        HD_HIP(hipStreamSynchronize(s));
    }

    // ---- frontier buffers -------------------------------------------------
    int64_t cap = opt.capacity > 0 ? opt.capacity : std::max<int64_t>(int64_t(1) << 22, 8 * nA);
    cap = std::max<int64_t>(cap, nA);
    Frontier<T> ACT, ACT2, PARK, CH;
    ACT.alloc(cap);
    ACT2.alloc(cap);
    PARK.alloc(cap);
    CH.alloc(std::max<int64_t>(cap, nA));
    DBuf flags_mem;
    int64_t fcap = std::max<int64_t>(CH.cap, cap);
    flags_mem.reserve((size_t)fcap * 4 * sizeof(int32_t) + 1024);
    int32_t *flag_act = flags_mem.as<int32_t>();
    int32_t *flag_park = flag_act + fcap;
    int32_t *pos = flag_park + fcap;
    int32_t *perm = pos + fcap;
    DBuf keys_mem;
    keys_mem.reserve((size_t)cap * 4 * sizeof(int32_t) + 1024);

    ClassifyCfg cc;
    cc.c = cctx;
    cc.recheck = (opt.precision == HD_PREC_FP32_RECHECK) && sizeof(T) == 4;
    cc.a = av;
    cc.bv64 = bv64;
    cc.m64 = m64;
    cc.iv = iv;

    // ---- round 0: bound every face ------------------------------------------
    R.mark(R.cev);
    k_faces_round0<T><<<grid_for(nA, BLK), BLK, 0, s>>>(nA, FA, vq.o, cc, bv, CH.v, CountOut{flag_act, flag_park},
                                                         st, st);
    HD_LAUNCH_CHECK();
    R.mark(R.cev);
    int64_t nAct = compact<T>(R, CH.v, nA, flag_act, pos, d_total, ACT.v, 0);
    int64_t nPark = compact<T>(R, CH.v, nA, flag_park, pos, d_total, PARK.v, 0);
    vq.mem.release();

    const double budget = (opt.budget_m > 0 ? opt.budget_m : 1e7) * (double)nA;
    double processed = (double)nA;
    int64_t subdivided = 0;
    int rounds = 0;
    S.max_frontier = nAct + nPark;
    QBuf<T> mq;
    hd_status status = HD_OK;
    while (nAct > 0) {
        if (opt.max_rounds > 0 && rounds >= opt.max_rounds) break;
        // how many to subdivide this round
        int64_t K = nAct;
        if (opt.subbatch > 0) K = std::min<int64_t>(K, opt.subbatch);
        K = std::min<int64_t>(K, (cap - nAct) / 3);
        K = std::min<int64_t>(K, (cap - nPark) / 4);
        K = std::min<int64_t>(K, CH.cap / 4);
        if (K <= 0 && nPark > 0) {
            // drop parked triangles that L has overtaken, then retry
            k_flag_ge<<<grid_for(nPark, BLK), BLK, 0, s>>>(PARK.v.ub, nPark, st, flag_park);
            nPark = compact<T>(R, PARK.v, nPark, flag_park, pos, d_total, CH.v, 0);
            swap_frontier(PARK, CH);
            K = std::min<int64_t>({nAct, (cap - nAct) / 3, (cap - nPark) / 4, CH.cap / 4});
            if (opt.subbatch > 0) K = std::min<int64_t>(K, opt.subbatch);
        }
        if (K <= 0) {
            status = HD_E_CAPACITY;
            break;
        }
        if (processed + 4.0 * K > budget) {
            status = HD_E_CAPACITY;
            break;
        }
        if (K < nAct) {
            // largest upper bounds first (the paper's priority-queue order)
            uint32_t *keys = keys_mem.as<uint32_t>();
            int32_t *vals = (int32_t *)(keys + cap);
            uint32_t *keys2 = (uint32_t *)(vals + cap);
            int32_t *vals2 = (int32_t *)(keys2 + cap);
            k_ub_keys<<<grid_for(nAct, BLK), BLK, 0, s>>>(ACT.v.ub, nAct, keys, vals);
            radix_sort_u32(keys, vals, keys2, vals2, nAct, 32, R.sort_tmp, s);
            k_gather<T><<<grid_for(nAct, BLK), BLK, 0, s>>>(ACT.v, vals, 0, nAct, ACT2.v);
            HD_LAUNCH_CHECK();
            swap_frontier(ACT, ACT2);
        }
        // midpoints of the K selected parents
        mq.alloc(3 * K, true);
        QueryIn in{};
        in.mode = Q_MIDPOINTS;
        in.a = av;
        in.face = ACT.v.face;
        in.lvl = ACT.v.lvl;
        for (int k = 0; k < 3; ++k) {
            in.ba[k] = ACT.v.ba[k];
            in.bb[k] = ACT.v.bb[k];
        }
        in.cx = B->center[0];
        in.cy = B->center[1];
        in.cz = B->center[2];
        R.queries<T>(in, 3 * K, qcfg, bv, mq.o, &S.stack_overflows);
        // children
        R.mark(R.cev);
        k_children<T><<<grid_for(4 * K, BLK), BLK, 0, s>>>(K, ACT.v, mq.o, cc, bv, CH.v,
                                                            CountOut{flag_act, flag_park}, st, st);
        HD_LAUNCH_CHECK();
        R.mark(R.cev);
        // new active list: unselected remainder, then active children
        int64_t rest = nAct - K;
        if (rest > 0) {
            k_gather<T><<<grid_for(rest, BLK), BLK, 0, s>>>(ACT.v, nullptr, K, rest, ACT2.v);
            HD_LAUNCH_CHECK();
        }
        int64_t na = compact<T>(R, CH.v, 4 * K, flag_act, pos, d_total, ACT2.v, rest);
        int64_t np = compact<T>(R, CH.v, 4 * K, flag_park, pos, d_total, PARK.v, nPark);
        swap_frontier(ACT, ACT2);
        nAct = rest + na;
        nPark += np;
        subdivided += K;
        processed += 4.0 * K;
        ++rounds;
        S.max_frontier = std::max<int64_t>(S.max_frontier, nAct + nPark);
        if (nAct > cap || nPark > cap) {
            status = HD_E_INTERNAL;
            break;
        }
        int bad = 0;
        HD_HIP(hipMemcpyAsync(&bad, &st->bad, sizeof(int), hipMemcpyDeviceToHost, s));
        HD_HIP(hipStreamSynchronize(s));
        if (bad == 3) { // subdivision depth exhausted (tolerance below what the arithmetic resolves)
            status = HD_E_CAPACITY;
            break;
        }
        if (bad) {
            status = HD_E_INTERNAL;
            break;
        }
    }
    HD_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
    HD_HIP(hipStreamSynchronize(s));
    if (hs.bad == 2) status = HD_E_INTERNAL; // traversal deeper than the fallback stack
    S.L_rounds = ord2d(hs.Lord);
    S.U_rounds = S.L_rounds;
    {
        // U reached by the rounds: largest live upper bound
        std::vector<float> ub_host;
        auto live_max = [&](const Frontier<T> &F, int64_t n) {
            if (n <= 0) return 0.0;
            ub_host.resize(n);
            HD_HIP(hipMemcpy(ub_host.data(), F.v.ub, n * sizeof(float), hipMemcpyDeviceToHost));
            return (double)*std::max_element(ub_host.begin(), ub_host.end());
        };
        S.U_rounds = std::max({S.L_rounds, live_max(ACT, nAct), live_max(PARK, nPark)});
    }

    if (status == HD_OK) {
        // final FP64 step: L was re-evaluated in FP64 at the best vertex after
        // every query round; now U over every live triangle
        if (nPark > 0)
            k_final_U<T><<<grid_for(nPark, BLK), BLK, 0, s>>>(PARK.v, nPark, av, bv64, iv, cctx, m64, st);
        if (nAct > 0)
            k_final_U<T><<<grid_for(nAct, BLK), BLK, 0, s>>>(ACT.v, nAct, av, bv64, iv, cctx, m64, st);
        HD_LAUNCH_CHECK();
        HD_HIP(hipMemcpyAsync(&hs, st, sizeof(hs), hipMemcpyDeviceToHost, s));
        HD_HIP(hipStreamSynchronize(s));
        double L = ord2d(hs.Lord);
        double U = std::max(L, ord2d(hs.Uord));
        LU[0] = L;
        LU[1] = U;
        if (nAct == 0 && U - L > S.eps_abs) status = HD_E_INTERNAL;
        if (nAct > 0 && opt.max_rounds <= 0) status = HD_E_INTERNAL;
    }
    S.rounds = rounds;
    S.status = status;
    S.nodes_bounded = (int64_t)hs.bounded;
    S.subdivided = subdivided;
    S.queries = (int64_t)hs.queries;
    S.pt_tri_evals = (int64_t)hs.evals;
    S.box_tests = (int64_t)hs.boxes;
    for (int k = 0; k < 5; ++k) S.discards[k] = (int64_t)hs.discards[k];
    S.rechecked64 = (int64_t)hs.rechecked;
    S.parked_final = nPark;
    S.query_leaf_evals = (int64_t)hs.q_leaves;
    S.query_box_tests = (int64_t)hs.q_boxes;
    if (R.profile) {
        HD_HIP(hipStreamSynchronize(s));
        S.ms_query_kernels = Runner::sum_pairs(R.qev);
        S.ms_cascade_kernels = Runner::sum_pairs(R.cev);
        S.query_launches = (int64_t)R.qev.size() / 2;
        S.cascade_launches = (int64_t)R.cev.size() / 2;
    }
    S.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (stats) *stats = S;
    return status;
}

} // namespace

} // namespace hd

// ============================================================================
// C ABI
// ============================================================================
using namespace hd;

static hd_status guard(const char *where, const std::function<hd_status()> &fn) {
    (void)where;
    try {
        return fn();
    } catch (const Error &e) {
        return e.st;
    } catch (...) {
        return HD_E_INTERNAL;
    }
}

extern "C" {

const char *hd_status_str(hd_status s) {
    switch (s) {
    case HD_OK: return "ok";
    case HD_E_INVALID: return "invalid argument";
    case HD_E_CAPACITY: return "capacity or face budget exceeded";
    case HD_E_NOMEM: return "device allocation failed";
    case HD_E_DEVICE: return "HIP runtime error";
    case HD_E_INTERNAL: return "internal invariant failed";
    }
    return "unknown status";
}

void hd_default_options(hd_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = HD_PREC_FP32_RECHECK;
    o->order = 1234;
    o->budget_m = 1e7;
}

hd_status hd_build_bvh(const double *VB, int64_t mB, const int32_t *FB, int64_t nB, hd_stream_t stream,
                       hd_bvh *out) {
    if (!out) return HD_E_INVALID;
    *out = nullptr;
    return guard("hd_build_bvh", [&] {
        Bvh *b = build_bvh(VB, mB, FB, nB, (hipStream_t)stream);
        *out = reinterpret_cast<hd_bvh>(b);
        return HD_OK;
    });
}

void hd_free_bvh(hd_bvh b) { delete reinterpret_cast<Bvh *>(b); }

hd_status hd_bound(const double *VA, int64_t mA, const int32_t *FA, int64_t nA, hd_bvh Bh, double eps,
                   const hd_options *opt, hd_stream_t stream, double LU_out[2], hd_stats *stats) {
    if (LU_out) LU_out[0] = LU_out[1] = NAN;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->status = HD_E_INVALID;
    }
    if (!LU_out || !Bh || !VA || !FA || mA <= 0 || nA <= 0 || !(eps > 0) || !std::isfinite(eps))
        return HD_E_INVALID;
    if (nA >= (int64_t(1) << 30)) return HD_E_INVALID;
    hd_options o;
    hd_default_options(&o);
    if (opt) o = *opt;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hd_status st = guard("hd_bound", [&] {
        double LU[2] = {NAN, NAN};
        hd_status r;
        if (o.precision == HD_PREC_FP64)
            r = bound_impl<double>(VA, mA, FA, nA, B, eps, o, (hipStream_t)stream, LU, stats);
        else if (o.precision == HD_PREC_FP32 || o.precision == HD_PREC_FP32_RECHECK)
            r = bound_impl<float>(VA, mA, FA, nA, B, eps, o, (hipStream_t)stream, LU, stats);
        else
            return HD_E_INVALID;
        if (r == HD_OK) {
            LU_out[0] = LU[0];
            LU_out[1] = LU[1];
        }
        return r;
    });
    if (stats) stats->status = st;
    return st;
}

hd_status hd_point_distances(const double *P, int64_t nP, hd_bvh Bh, int32_t precision, double *d, int32_t *I,
                             double *Q, hd_stream_t stream) {
    if (!Bh || nP < 0 || (nP > 0 && (!P || !d || !I))) return HD_E_INVALID;
    if (nP == 0) return HD_OK;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard("hd_point_distances", [&] {
        Runner R;
        R.s = s;
        R.b = B;
        R.st_mem.reserve(sizeof(DevState));
        R.st = R.st_mem.as<DevState>();
        k_state_init<<<1, 1, 0, s>>>(R.st);
        QueryIn in{};
        in.mode = Q_POINTS;
        in.P = P;
        in.cx = B->center[0];
        in.cy = B->center[1];
        in.cz = B->center[2];
        int64_t ovf = 0;
        auto run = [&](auto tag) {
            using T = decltype(tag);
            Margins m = make_margins(Prec<T>::u, B, B->coord_max);
            QueryCfg cfg{B->nodes.as<NodeRec>(), B->ids.as<int4>(), m, 0};
            QBuf<T> qb;
            qb.alloc(nP, false);
            BView<T> bv;
            if constexpr (sizeof(T) == 4) bv = BView<float>{B->frames32.as<float4>()};
            else bv = BView<double>{B->frames64.as<double2>()};
            R.queries<T>(in, nP, cfg, bv, qb.o, &ovf);
            k_export_points<T><<<grid_for(nP, BLK), BLK, 0, s>>>(qb.o, nP, B->ids.as<int4>(), B->center[0],
                                                                 B->center[1], B->center[2], d, I, Q);
            HD_LAUNCH_CHECK();
            HD_HIP(hipStreamSynchronize(s));
        };
        if (precision == HD_PREC_FP64) run(double{});
        else run(float{});
        DevState hs;
        HD_HIP(hipMemcpy(&hs, R.st, sizeof(hs), hipMemcpyDeviceToHost));
        if (hs.bad == 2) return HD_E_INTERNAL;
        return HD_OK;
    });
}

hd_status hd_eval_bounds(const double *v, const double *dd, const int32_t *I, const double *q, int64_t n, hd_bvh Bh,
                         int32_t precision, double *out, int32_t *u3_case, hd_stream_t stream) {
    if (!Bh || n < 0 || (n > 0 && (!v || !dd || !I || !q || !out || !u3_case))) return HD_E_INVALID;
    if (n == 0) return HD_OK;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard("hd_eval_bounds", [&] {
        DBuf inv;
        inv.reserve((size_t)B->nB * sizeof(int32_t));
        k_inv_perm<<<grid_for(B->nB, BLK), BLK, 0, s>>>(B->ids.as<int4>(), B->nB, inv.as<int32_t>());
        IdView iv{B->ids.as<int4>()};
        if (precision == HD_PREC_FP64)
            k_eval_bounds<double><<<grid_for(n, BLK), BLK, 0, s>>>(v, dd, I, q, n, inv.as<int32_t>(), B->nB,
                                                                   BView<double>{B->frames64.as<double2>()}, iv,
                                                                   B->center[0], B->center[1], B->center[2], out,
                                                                   u3_case);
        else
            k_eval_bounds<float><<<grid_for(n, BLK), BLK, 0, s>>>(v, dd, I, q, n, inv.as<int32_t>(), B->nB,
                                                                  BView<float>{B->frames32.as<float4>()}, iv,
                                                                  B->center[0], B->center[1], B->center[2], out,
                                                                  u3_case);
        HD_LAUNCH_CHECK();
        HD_HIP(hipStreamSynchronize(s));
        return HD_OK;
    });
}

} // extern "C"
