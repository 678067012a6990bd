// hd_engine.hip -- the branch-and-bound rounds on the GPU, for one pair or
// many pairs at once, and the C ABI.
//
// Round 0 queries every referenced vertex of A, raises the lower bound L of
// its pair (a vertex distance is a lower bound of h: Branch and bound
// subsection) and bounds every face of A with the cascade. Each later round
// takes the active frontier (upper bound above L + eps), optionally the
// sub-batch with the largest upper bounds (the paper's priority order),
// splits every selected triangle 1->4 at its edge midpoints, queries the three
// midpoints (seeded with the closest faces of the edge's endpoints), raises
// L, bounds the four children and appends them to the active list (to split
// again), the parked list (within eps of L: kept for U, never split) or drops
// them (below L). The loop ends when no triangle is active; then every pair
// has U - L <= eps (the paper's stopping rule). The final step re-evaluates
// the parked triangles' bounds in FP64.
//
// All pairs of a batched call share the kernels: records carry their pair id
// and every per-pair quantity (centre, BVH root, L, U, eps, margins) is read
// from the pair table. Without sub-batches the device plans each round
// (k_report_plan) and the host enqueues one round ahead of the small report
// it polls; with sub-batches (or the frontier log) the host selects each
// round's sub-batch from the report of the previous one.
#include <math.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <unistd.h>
#include <utility>
#include <vector>

#include "hd_kernels.hpp"
#include "hd_learned.hpp"
#include "hd_mlp.hpp"
#include "hd_reduce.hpp"

namespace hd {

namespace {

constexpr int QSTACK = 16;    // LDS ring-stack entries per lane (16 KB per block)
constexpr int SMALL_STACK = 1; // test hook: a one-entry LDS stack, forces the deep path
constexpr int DEEP_STACK = 256;
constexpr int DEEP_SLOTS = 256;  // deep traversals at once: one per thread of the query kernel's last block
constexpr int BLK = 256;
constexpr int NW = BLK / 64;
constexpr unsigned GRID_MAX = 2048;  // persistent cap of grid-stride launches (8 blocks per CU)
constexpr unsigned XCDS = 8;         // accelerator complex dies, each with its own L2
constexpr unsigned QGRID_MAX = 4096; // the same for the query kernel's smaller blocks
constexpr unsigned C_GRID_MAX = 256;  // stage C (FP64 re-bounds of the few records in the recheck band)

// Device control block. Atomics on one line serialise at the memory side
// (about 9 ns each), and lines closer than 256 bytes still share that queue:
// each append counter (every active block of a cascade kernel takes a
// returning atomic on each list it appends to) sits on a 256-byte line of its
// own, and the statistics are spread over ACC_COPIES copies (block b adds to
// copy b % ACC_COPIES; readers sum the copies).
enum {
    ST_EVALS,
    ST_BOUNDED,
    ST_RECHECKED,
    ST_DISCARDS, // six entries, one per deciding bound (uexact, u1..u5)
    ST_QUERIES = ST_DISCARDS + 6,
    ST_BOXES,
    ST_QLEAVES,
    ST_SKIPS, // records whose u3 / u4 the learned policy skipped
    ST_STALE, // active records dropped by the sub-batch selection (bound below L)
    ST_OVERFLOWS, // queries redone with the deep stack (their LDS stack overflowed)
    ST_N
};
constexpr int ST_STRIDE = 32; // 256 bytes per copy
static_assert(ST_N <= ST_STRIDE, "statistics copy overflows its line");

// Counts of the blocks of a launch that have finished, to find the last
// one (last_block). Atomics on one address serialise at the memory side (tens
// of nanoseconds each when thousands of blocks end together), so blocks count
// on LB_WAYS separate lines, and the block that completes a line counts on
// the top line: the block that completes the top line is the last.
constexpr int LB_WAYS = 16;
// launches of at most this many blocks count on one line (the second level
// would only lengthen the last block's path)
constexpr unsigned LB_SPLIT_MIN = 256;
struct BlockCounter {
    struct alignas(256) Line {
        unsigned n;
    };
    Line way[LB_WAYS];
    Line top;
};
// way w's share of nactive blocks dealt to the ways in turn
HD_D unsigned way_share(unsigned nactive, unsigned w) {
    return nactive / LB_WAYS + (w < nactive % LB_WAYS ? 1u : 0u);
}

struct Ctl {
    alignas(256) unsigned long long act_next; // append counters of the current round
    alignas(256) unsigned long long park_next;
    alignas(256) unsigned long long b_next; // records waiting for cascade stage B
    alignas(256) unsigned long long c_next; // records waiting for cascade stage C
    // 2 traversal deeper than the fallback stack, 3 depth exhausted, 4 an upper
    // bound below a vertex distance of its triangle (unsound), 5 plain FP32
    // with a tolerance below its margin at the lower bound
    alignas(256) int bad;
    int bad_input;        // 1: soup A has an out-of-range index or a non-finite coordinate
    int n_overflow;       // queries whose LDS stack overflowed this round
    int log_rounds;       // 1: reports carry the lower bound, upper bound and statistics
    alignas(256) unsigned long long stat[ACC_COPIES][ST_STRIDE];
    // after a query launch that raises L: some pair has a round key above its
    // best key (the argmax step then has a new point to take to FP64)
    alignas(256) int argmax_new;
    // device-planned rounds (written by plan_round, read by the round's kernels)
    alignas(256) unsigned long long plan_K, plan_rest; // parents split this round, records carried over
    unsigned long long plan_Q;                         // the round's point queries (3 or 12 per parent)
    int plan_two;                                      // levels each parent is split this round, less
                                                       // one: 0 (1 -> 4), 2 (1 -> 16) or 4 (1 -> 256)
    int lvl_bound;                                     // no record is deeper than this subdivision level
    unsigned long long nref;                           // referenced vertices of A (round 0's queries)
    unsigned long long subdivided, rounds;             // totals over the planned rounds
    double processed;                                  // faces processed (the paper's budget count)
    int stall;                                         // 1: capacity left no room to split
    int over_budget;                                   // 1: the next split would exceed the budget
    int c_decision;                                    // stage C this round: 0 undecided, 1 run, 2 deferred
    // device sub-batch selection (sel_round): plan_round leaves the list as it
    // is and sets the target; the selection passes pick the records and
    // finish the plan
    unsigned long long plan_kcap;  // most parents the lists have room for this round
    unsigned long long sel_n;      // active records when the selection started
    unsigned long long sel_live;   // of those, neither below L nor within eps of it
    unsigned long long sel_above1; // live records in first-level bins above sel_b1
    unsigned sel_b1, sel_thr;      // boundary bin of the first pass; the ordered-key threshold
    int sel_mode;                  // SEL_NONE, SEL_ALL or SEL_THRESHOLD
    int learn_off;                 // learned order: a round found no record predicted to raise L, so
                                   // every later round splits all live records (no more scoring)
    alignas(256) unsigned long long sel_prom;  // learned order: live records predicted above L + eps
    alignas(256) unsigned long long sel_next;  // selected parents appended (their record indices)
    alignas(256) unsigned long long rest_next; // unselected live records appended
    // blocks of the current query / argmax / stage C / selection launch that
    // have finished (the last one does the launch's tail work; every count
    // is back at zero after it). Last in the block: the host never reads them.
    BlockCounter q_done, f_done, c_done, h1_done, h2_done;
};
// the part of the control block the host reads
constexpr size_t CTL_HOST_BYTES = offsetof(Ctl, q_done);
static_assert(CTL_HOST_BYTES % 8 == 0, "exported control block size");

// Item count of a launch: a host value, or (device-planned rounds) a count
// the device wrote, times a multiplicity. Kernels that take one loop over it
// with a grid stride, so their grid need not match it.
struct DevCount {
    const unsigned long long *p;
    int64_t mult;
    int64_t host_n;
    HD_D int64_t get() const { return p ? (int64_t)(*p) * mult : host_n; }
};
inline DevCount host_count(int64_t n) { return DevCount{nullptr, 1, n}; }

struct PairSrcA {
    const double *V;
    const int32_t *F;
    int64_t m;
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

// True in every thread of the one of `nactive` blocks that finishes last,
// which then sees every write the other blocks made before finishing with
// release set (a device-scope fence, which writes the XCD's L2 back: a block
// whose plain stores the last block does not read passes false; its returning
// atomics were performed before its ticket anyway). *counter (zero at launch)
// is reset for the next launch. Every thread of each of those blocks must call
// it, once, at the end of its work, with the same release; blocks that had no
// work (a grid sized for a larger count) must not: every call is an atomic on
// one address, and these serialise.
__device__ bool last_block(BlockCounter *c, unsigned way, unsigned way_blocks, unsigned ways, bool release = true) {
    __shared__ int last;
    __syncthreads();
    if (threadIdx.x == 0) {
        if (release) __threadfence();
        int l = 0;
        if (atomicAdd(&c->way[way].n, 1u) == way_blocks - 1) {
            atomicExch(&c->way[way].n, 0u);
            if (ways == 1) {
                l = 1;
            } else {
                __threadfence(); // the way's blocks, ahead of the top count
                if (atomicAdd(&c->top.n, 1u) == ways - 1) {
                    atomicExch(&c->top.n, 0u);
                    l = 1;
                }
            }
        }
        last = l;
    }
    __syncthreads();
    if (last) __threadfence();
    return last;
}

// the same when the blocks with work are blocks 0 .. nactive - 1 (way: the
// block index modulo LB_WAYS; one way for small grids)
__device__ bool last_block(BlockCounter *c, unsigned nactive, bool release = true) {
    if (nactive <= LB_SPLIT_MIN) return last_block(c, 0, nactive, 1, release);
    const unsigned w = blockIdx.x % LB_WAYS;
    return last_block(c, w, way_share(nactive, w), LB_WAYS, release);
}

__device__ __forceinline__ int pair_of(const int64_t *__restrict__ off, int npairs, int64_t x) {
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class T> HD_HD const Margins &margins_of(const PairConst &p);
template <> HD_HD const Margins &margins_of<float>(const PairConst &p) { return p.m32; }
template <> HD_HD const Margins &margins_of<double>(const PairConst &p) { return p.m64; }

// atomicMax of (a, b) into pair `pair`'s L and round key: one atomic per wave
// when every contributing lane has the same pair, else one per lane. All
// lanes of the wave must call it; lanes with nothing to add pass zeros.
// Both values only grow while a launch runs, so an atomic that cannot raise
// the value is skipped: a plain read of it (possibly an older copy in this
// XCD's L2, which is never above the current value) decides. Without that
// test every wave of a query launch queues one atomic on the same line,
// and those serialise at the memory side.
HD_D bool may_raise(const unsigned long long *x, unsigned long long v) {
    return v && v > __hip_atomic_load(x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ void pair_max2(PairVar *pv, int pair, unsigned long long a, unsigned long long b) {
    unsigned long long has = __ballot(a != 0 || b != 0);
    if (!has) return;
    int first = __ffsll(has) - 1;
    int p0 = __shfl(pair, first, 64);
    bool uni = __ballot((a != 0 || b != 0) && pair != p0) == 0;
    if (uni) {
        for (int o = 32; o >= 1; o >>= 1) {
            unsigned long long ta = __shfl_xor(a, o, 64), tb = __shfl_xor(b, o, 64);
            a = ta > a ? ta : a;
            b = tb > b ? tb : b;
        }
        if (__lane_id() == 0) {
            if (may_raise(&pv[p0].Lord, a)) atomicMax(&pv[p0].Lord, a);
            if (may_raise(&pv[p0].round_key, b)) atomicMax(&pv[p0].round_key, b);
        }
    } else {
        if (may_raise(&pv[pair].Lord, a)) atomicMax(&pv[pair].Lord, a);
        if (may_raise(&pv[pair].round_key, b)) atomicMax(&pv[pair].round_key, b);
    }
}


// zero the control block (by the threads of block 0)
__device__ void ctl_zero(Ctl *c) {
    static_assert(sizeof(Ctl) % 8 == 0, "control block size");
    if (blockIdx.x != 0) return;
    unsigned long long *w = reinterpret_cast<unsigned long long *>(c);
    for (int k = threadIdx.x; k < (int)(sizeof(Ctl) / 8); k += blockDim.x) w[k] = 0;
}

__global__ void k_ctl_init(Ctl *c) { ctl_zero(c); }

// What the host needs between rounds, written by the device into pinned host
// memory; `seq` last, after a system-scope fence, so that a host that sees
// the new seq sees the fields too.
// Reports go to a ring of MB_SLOTS slots (slot seq % MB_SLOTS), so that a
// report may be in flight while the host reads the previous one.
constexpr int MB_SLOTS = 4;
struct alignas(128) Mailbox {
    int64_t act, park, rounds, subdivided;
    int32_t bad_input, pad;
    int64_t pend_c; // records waiting for stage C (deferred)
    int bad, stall, over_budget;
    unsigned seq;
    // with Ctl::log_rounds: pair 0's bounds and the statistics so far
    double L0, U0;
    int64_t bounded, discards[5];
};
// the pinned host block: the report ring, then the export's sequence word
constexpr size_t HOST_RING = 0, HOST_EXPORT_SEQ = MB_SLOTS * sizeof(Mailbox), HOST_UPLOAD = HOST_EXPORT_SEQ + 256;

__device__ void report_to(const Ctl *ctl, const PairVar *pv, Mailbox *ring, unsigned seq) {
    Mailbox *mb = ring + seq % MB_SLOTS;
    if (ctl->log_rounds) {
        const double L = ord2d(pv[0].Lord);
        mb->L0 = L;
        mb->U0 = fmax(L, ord2d(pv[0].Uround));
        unsigned long long b = 0, dc[5] = {0, 0, 0, 0, 0};
        for (int c = 0; c < ACC_COPIES; ++c) {
            b += ctl->stat[c][ST_BOUNDED];
            for (int k = 0; k < 5; ++k) dc[k] += ctl->stat[c][ST_DISCARDS + k];
        }
        mb->bounded = (int64_t)b;
        for (int k = 0; k < 5; ++k) mb->discards[k] = (int64_t)dc[k];
    }
    mb->act = (long long)ctl->act_next;
    mb->park = (long long)ctl->park_next;
    mb->bad_input = ctl->bad_input;
    mb->rounds = (long long)ctl->rounds;
    mb->subdivided = (long long)ctl->subdivided;
    // records still waiting for stage C: none once stage C ran this round
    // (its count is cleared only by the next plan)
    mb->pend_c = ctl->c_decision == 1 ? 0 : (long long)ctl->c_next;
    mb->bad = ctl->bad;
    mb->stall = ctl->stall;
    mb->over_budget = ctl->over_budget;
    __threadfence_system();
    __hip_atomic_store(&mb->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ void k_report(const Ctl *ctl, const PairVar *pv, Mailbox *ring, unsigned seq) {
    if (threadIdx.x == 0) report_to(ctl, pv, ring, seq);
}

// Device-planned round: how many active records to split (all of them,
// capped by the list capacities and the face budget) and the per-round
// counters. A round planned with nothing to do leaves everything in place.
// the points of a resolution-16 barycentric lattice (corners included), the
// query set of a four-level round; such rounds take at most this many parents
constexpr int LAT16_N = 16;
constexpr int LAT16_PTS = (LAT16_N + 1) * (LAT16_N + 2) / 2;
constexpr int64_t FOUR_LEVEL_MAX = 64;
struct PlanCaps {
    int64_t act, park, pend, pend_c, mq; // capacities (records / queries)
    double budget;               // the paper's m * nA
    int grow_act, grow_park;     // 1: the host can still grow the active / parked lists
    int64_t subbatch;            // > 0: the round splits the sub-batch the device selects
    int learned;                 // sub-batches in learned order (the selection may take all)
    int64_t two_max;             // breadth-first rounds of at most this many parents split two
                                 // levels deep (0: never)
    int64_t four_max;            // and of at most this many, four (0: never)
};
__device__ void plan_round(Ctl *c, const PlanCaps &caps) {
    const int64_t nAct = (int64_t)c->act_next, nPark = (int64_t)c->park_next;
    // with sub-batches the round splits at most this many (the selection
    // may also drop or park up to all of the others)
    // (the learned order splits every live record once none is predicted to
    // raise L, so its rounds are planned for all of them)
    const int64_t want =
        caps.subbatch > 0 && !caps.learned ? (nAct < caps.subbatch ? nAct : caps.subbatch) : nAct;
    const int64_t reserve_park = caps.subbatch > 0 ? nAct : 0;
    // records waiting for stage C may each still join either list
    const int64_t nc = c->c_decision == 1 ? 0 : (int64_t)c->c_next;
    int64_t K = 0, kcap = 0;
    if (!c->bad && !c->stall && !c->over_budget && nAct > 0) {
        // room in the active-side lists (the pending and midpoint lists are
        // sized with the active ones) and in the parked list
        int64_t ka = (caps.act - nAct - nc) / 3;
        ka = ka < caps.pend / 4 ? ka : caps.pend / 4;
        ka = ka < (caps.pend_c - nc) / 4 ? ka : (caps.pend_c - nc) / 4;
        ka = ka < caps.mq / 3 ? ka : caps.mq / 3;
        const int64_t kp = (caps.park - nPark - nc - reserve_park) / 4;
        kcap = ka < kp ? ka : kp;
        K = want < kcap ? want : kcap;
        // split all or, while the list that lacks room can grow, none (a
        // stall: the host grows it), so that the rounds do not depend on the
        // capacities that earlier calls left behind
        if ((ka < want && caps.grow_act) || (kp < want && caps.grow_park)) K = 0;
        if (K <= 0) {
            K = 0;
            c->stall = 1;
        } else if (caps.subbatch <= 0 && c->processed + 4.0 * (double)K > caps.budget) {
            K = 0;
            c->over_budget = 1;
        }
    }
    if (caps.subbatch > 0) {
        // the selection passes pick about K records and finish the plan
        // (split count, carried count, budget, totals)
        c->plan_two = 0;
        c->plan_Q = 0;
        c->plan_K = (unsigned long long)K;
        c->plan_kcap = (unsigned long long)(kcap > 0 ? kcap : 0);
        c->sel_prom = 0;
        c->b_next = 0;
        if (c->c_decision != 2) c->c_next = 0;
        c->c_decision = 0;
        c->n_overflow = 0;
        return;
    }
    // A round with few parents is bound by the latency of its kernels, not
    // by their work: splitting each parent two levels deep at once (its 16
    // grandchildren, from the 12 non-corner points of its resolution-4
    // lattice) does the next round's splits of its children in the same
    // launches. Every grandchild is bounded as usual; a child that a
    // one-level round would have discarded just has its four children
    // bounded (and discarded) instead. Only while every record is at least
    // two levels above the depth limit, and when the lists and the budget
    // have room for 16 children per parent.
    // A round of at most FOUR_LEVEL_MAX parents (the very last ones) goes
    // four levels deep: the 153 points of each parent's resolution-16
    // lattice and its 256 descendants at that level.
    auto room = [&](int64_t kids, int64_t queries) {
        int64_t kd = (caps.act - nAct - nc) / (kids - 1);
        kd = kd < caps.pend / kids ? kd : caps.pend / kids;
        kd = kd < (caps.pend_c - nc) / kids ? kd : (caps.pend_c - nc) / kids;
        kd = kd < caps.mq / queries ? kd : caps.mq / queries;
        const int64_t kpd = (caps.park - nPark - nc) / kids;
        return K <= kd && K <= kpd && c->processed + (double)kids * (double)K <= caps.budget;
    };
    int dep = 0; // extra levels
    if (K > 0 && K <= caps.two_max) {
        if (K <= caps.four_max && c->lvl_bound + 4 <= 30 && room(256, LAT16_PTS)) dep = 4;
        else if (c->lvl_bound + 2 <= 30 && room(16, 12)) dep = 2;
    }
    const int kids = dep == 4 ? 256 : (dep == 2 ? 16 : 4);
    c->plan_K = (unsigned long long)K;
    c->plan_Q = (unsigned long long)K * (dep == 4 ? (unsigned)LAT16_PTS : (dep == 2 ? 12u : 3u));
    c->plan_two = dep;
    c->plan_rest = (unsigned long long)(nAct - K);
    c->processed += (double)kids * (double)K;
    c->subdivided += (unsigned long long)K;
    if (K > 0) {
        c->rounds += 1;
        c->lvl_bound += dep ? dep : 1;
    }
    c->act_next = (unsigned long long)(nAct - K);
    c->park_next = (unsigned long long)nPark;
    c->b_next = 0;
    // stage C's list is emptied when stage C ran; deferred records stay
    if (c->c_decision != 2) c->c_next = 0;
    c->c_decision = 0;
    c->n_overflow = 0;
}

// the end of a device-planned round: report its state, then plan the next
// round (a planned round that is never enqueued changes nothing the host
// reads afterwards)
__global__ void k_report_plan(Ctl *ctl, const PairVar *pv, Mailbox *ring, unsigned seq, PlanCaps caps) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    report_to(ctl, pv, ring, seq);
    plan_round(ctl, caps);
}


// the list counts as the host last saw them (records waiting for stage C
// stay), before stage C runs outside a round
__global__ void k_set_counts(Ctl *c, unsigned long long act, unsigned long long park) {
    if (threadIdx.x != 0) return;
    c->act_next = act;
    c->park_next = park;
    c->c_decision = 0;
}

__global__ void k_zero_u32(unsigned *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ void k_clear_stall(Ctl *c) {
    if (threadIdx.x == 0) c->stall = 0;
}

__global__ void k_round_setup(Ctl *c, unsigned long long act_base, unsigned long long park_base) {
    c->n_overflow = 0;
    c->act_next = act_base;
    c->park_next = park_base;
    c->b_next = 0;
    c->c_next = 0;
}

// linked: pairs 2k and 2k + 1 share their lower bound (two-sided distance)
__device__ void pair_init(PairConst *pc, PairVar *pv, const BvhPair *__restrict__ bp, int p, int linked = 0) {
    PairConst c;
    memset(&c, 0, sizeof(c));
    PairVar d;
    memset(&d, 0, sizeof(d));
    for (int k = 0; k < 3; ++k) c.ctr[k] = bp[p].ctr[k];
    c.root = bp[p].root;
    c.link = linked ? (p ^ 1) : p;
    d.Lord = d2ord(0.0);
    d.Uord = d2ord(0.0);
    d.Urounds = d2ord(0.0);
    d.Uround = d2ord(0.0);
    pc[p] = c;
    pv[p] = d;
}

// Accumulators of the ingest (ordered FP64 bits): the box of A's referenced
// vertices and the largest centred coordinate. ACC_COPIES copies of npairs
// entries, astride entries (a multiple of 256 bytes) apart.
struct PairBox {
    unsigned long long bbox[6];
    unsigned long long coord_max;
    unsigned long long pad;
};
inline int pbox_stride(int npairs) { return (int)(((npairs * sizeof(PairBox) + 255) & ~size_t(255)) / sizeof(PairBox)); }

__device__ void pbox_init(PairBox *pb, int npairs, int astride, int64_t i) {
    if (i >= (int64_t)npairs * ACC_COPIES) return;
    PairBox &b = pb[(i / npairs) * astride + i % npairs];
    for (int k = 0; k < 3; ++k) {
        b.bbox[k] = d2ord(__builtin_inf());
        b.bbox[3 + k] = d2ord(-__builtin_inf());
    }
    b.coord_max = d2ord(0.0);
}

__global__ void k_pairs_init(PairConst *pc, PairVar *pv, const BvhPair *__restrict__ bp, int npairs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) pair_init(pc, pv, bp, p);
}

// the start of a call: control block, pair tables, referenced-vertex marks
__global__ void k_bound_init(Ctl *ctl, PairConst *pc, PairVar *pv, PairBox *pb, int astride,
                             const BvhPair *__restrict__ bp, int npairs, int32_t *__restrict__ ref, int64_t m,
                             int log_rounds, int linked) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    ctl_zero(ctl);
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) ctl->log_rounds = log_rounds;
    if (i < npairs) pair_init(pc, pv, bp, (int)i, linked);
    pbox_init(pb, npairs, astride, i);
    if (i < m) ref[i] = 0;
}

// Validate A's faces, gather every pair's faces into one array with global
// vertex ids (and the referenced vertices into one vertex array), mark the
// referenced vertices, and accumulate each pair's bbox and coordinate range.
__global__ void k_ingest(const PairSrcA *__restrict__ src, const int64_t *__restrict__ foff,
                         const int64_t *__restrict__ voff, int npairs, int64_t n, int32_t *__restrict__ Fout,
                         double *__restrict__ Vout, int32_t *__restrict__ fpair, int32_t *__restrict__ ref,
                         const PairConst *__restrict__ pc, PairBox *pb, int astride, Ctl *ctl) {
    // one face per thread with several pairs; with one, a grid-stride run of
    // faces per thread (a capped grid: fewer blocks end in the atomics)
    const int64_t f0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = f0 < n;
    const int p = pair_of(foff, npairs, valid ? f0 : n - 1);
    double lo[3] = {__builtin_inf(), __builtin_inf(), __builtin_inf()};
    double hi[3] = {-__builtin_inf(), -__builtin_inf(), -__builtin_inf()};
    double cm = 0;
    for (int64_t f = f0; f < n; f += (int64_t)gridDim.x * blockDim.x) {
        PairSrcA s = src[p];
        int64_t lf = f - foff[p];
        fpair[f] = p;
        for (int j = 0; j < 3; ++j) {
            int32_t v = s.F[3 * lf + j];
            if (v < 0 || v >= s.m) {
                ctl->bad_input = 1;
                Fout[3 * f + j] = (int32_t)voff[p];
                continue;
            }
            int64_t vg = voff[p] + v;
            Fout[3 * f + j] = (int32_t)vg;
            ref[vg] = 1;
            for (int k = 0; k < 3; ++k) {
                double x = s.V[3 * (int64_t)v + k];
                if (!__builtin_isfinite(x)) {
                    ctl->bad_input = 1;
                    x = 0;
                }
                Vout[3 * vg + k] = x;
                lo[k] = fmin(lo[k], x);
                hi[k] = fmax(hi[k], x);
                cm = fmax(cm, fabs(x - pc[p].ctr[k]));
            }
        }
    }
    const double v[7] = {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], cm};
    block_pair_minmax<7, 0x78u, BLK>(p, valid, v, [&](int q, int k) {
        PairBox &b = pb[(int64_t)acc_copy() * astride + q];
        return k < 6 ? &b.bbox[k] : &b.coord_max;
    });
}

constexpr unsigned INGEST_ONE_PAIR_GRID = 1024;

__device__ Margins make_margins(double u, double edge_max, double coord_max) {
    Margins m;
    m.mu_d = 16 * u;
    m.mu_e = 48 * u;
    m.mu_0 = u * (48 * edge_max + 12 * coord_max);
    return m;
}

// diagonal of the box of pair p's referenced A vertices (folding the copies)
__device__ double pair_diag(const PairBox *pb, int astride, int p) {
    unsigned long long b[6];
    for (int k = 0; k < 6; ++k) b[k] = pb[p].bbox[k];
    for (int c = 1; c < ACC_COPIES; ++c) {
        const PairBox &x = pb[(int64_t)c * astride + p];
        for (int k = 0; k < 3; ++k) {
            b[k] = x.bbox[k] < b[k] ? x.bbox[k] : b[k];
            b[3 + k] = x.bbox[3 + k] > b[3 + k] ? x.bbox[3 + k] : b[3 + k];
        }
    }
    double d2 = 0;
    for (int k = 0; k < 3; ++k) {
        const double e = ord2d(b[3 + k]) - ord2d(b[k]);
        d2 += e * e;
    }
    return sqrt(d2);
}

// pair p's dA, eps * dA and margins, once the ingest has its bbox and
// coordinate range
__device__ void pair_post(PairConst *pc, const PairBox *pb, int astride, const BvhPair *__restrict__ bp, int p,
                          const double *__restrict__ eps, int eps_per_pair, int eps_rel) {
    // fold the copies of the coordinate range
    unsigned long long cmo = 0;
    for (int c = 0; c < ACC_COPIES; ++c) {
        const unsigned long long x = pb[(int64_t)c * astride + p].coord_max;
        cmo = x > cmo ? x : cmo;
    }
    const double dA = pair_diag(pb, astride, p);
    pc[p].dA = dA;
    // the tolerance: absolute, or the paper's relative form (times dA; two
    // linked pairs take the larger diagonal, so that both use one tolerance)
    const int q = pc[p].link;
    const double scale = q == p ? dA : fmax(dA, pair_diag(pb, astride, q));
    pc[p].eps_abs = eps[eps_per_pair ? p : 0] * (eps_rel ? scale : 1.0);
    double cm = fmax(ord2d(cmo), bp[p].coord_max);
    pc[p].m32 = make_margins(Prec<float>::u, bp[p].edge_max, cm);
    pc[p].m64 = make_margins(Prec<double>::u, bp[p].edge_max, cm);
}

// after the ingest: compact the referenced vertex ids (order preserving),
// finish the pair tables, and set up round 0's counters
__global__ void k_ingest_post(const int32_t *__restrict__ ref, const int32_t *__restrict__ pos, int64_t m,
                              const int32_t *__restrict__ nref, int32_t *__restrict__ out, PairConst *pc,
                              const PairBox *pb, int astride, const BvhPair *__restrict__ bp, int npairs,
                              const double *__restrict__ eps, int eps_per_pair, int eps_rel, Ctl *ctl) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v < m && ref[v]) out[pos[v]] = (int32_t)v;
    if (v < npairs) pair_post(pc, pb, astride, bp, (int)v, eps, eps_per_pair, eps_rel);
    if (v == 0) {
        ctl->nref = (unsigned long long)*nref;
        ctl->n_overflow = 0;
        ctl->act_next = 0;
        ctl->park_next = 0;
        ctl->b_next = 0;
        ctl->c_next = 0;
    }
}

// ---------------------------------------------------------------------------
// point queries
// ---------------------------------------------------------------------------
enum QMode { Q_POINTS = 0, Q_VERTICES = 1, Q_MIDPOINTS = 2, Q_LATTICE = 3, Q_BARYCENTERS = 4 };

// The twelve non-corner points of the resolution-4 barycentric lattice of a
// triangle (weights (4 - a1 - a2, a1, a2) / 4), two bits per weight.
constexpr int LATTICE_PTS = 12;
constexpr uint32_t LATTICE_A1 = (1u << 0) | (0u << 2) | (2u << 4) | (1u << 6) | (0u << 8) | (3u << 10) | (2u << 12) |
                                (1u << 14) | (0u << 16) | (3u << 18) | (2u << 20) | (1u << 22);
constexpr uint32_t LATTICE_A2 = (0u << 0) | (1u << 2) | (0u << 4) | (1u << 6) | (2u << 8) | (0u << 10) | (1u << 12) |
                                (2u << 14) | (3u << 16) | (1u << 18) | (2u << 20) | (3u << 22);

template <class T> struct QueryOut {
    T *d;
    int *I;
    T *q[3];
    T *p[3];                 // query position (precision T), reused by the bound kernels
    unsigned long long *key; // (d_lo, tag) key for the argmax (raise_L only)
};

template <class T> struct QueryIn {
    int mode;
    int npairs;
    const double *P;         // Q_POINTS: n x 3, uncentred, pair 0
    const int32_t *vids;     // Q_VERTICES: referenced vertex ids (global)
    const int64_t *voff;     // Q_VERTICES: vertex offsets of the pairs
    AView a;                 // Q_VERTICES / Q_MIDPOINTS
    FrontierView<T> par;     // Q_MIDPOINTS / Q_LATTICE: selected parents
    const PairConst *pc;
    const int32_t *sel;      // Q_MIDPOINTS: record index of each parent (null: the first parents)
    const int *two;          // Q_MIDPOINTS: the round's extra levels (Ctl::plan_two; null: none).
                             // 2: each parent's 12 non-corner resolution-4 lattice points instead
                             // of its 3 midpoints; 4: all 153 points of its resolution-16 lattice
};

// the extra subdivision levels of a Q_MIDPOINTS round (0, 2 or 4)
HD_D int two_level(const int *two) { return two ? *two : 0; }

// point t of the resolution-N lattice, rows of constant a2 in order (row r
// holds a1 = 0 .. N - r): its weights a1, a2 of parent corners 1 and 2 (over N)
HD_D void lattice_point(int N, int t, int &a1, int &a2) {
    int r = 0;
    while (t > N - r) {
        t -= N - r + 1;
        ++r;
    }
    a1 = t;
    a2 = r;
}
HD_D int lattice_index(int N, int a1, int a2) { return a2 * (N + 1) - (a2 * (a2 - 1)) / 2 + a1; }

struct QPoint {
    V3<double> p;
    int pair;
    int64_t out;  // output slot
    uint32_t tag; // argmax tie-break tag
    int seed[2];  // candidate triangles (or -1)
};

template <class T> HD_D QPoint query_point(const QueryIn<T> &in, int64_t i) {
    QPoint q;
    q.seed[0] = q.seed[1] = -1;
    if (in.mode == Q_POINTS) {
        q.pair = 0;
        const double *c = in.pc[0].ctr;
        q.p = {in.P[3 * i] - c[0], in.P[3 * i + 1] - c[1], in.P[3 * i + 2] - c[2]};
        q.out = i;
        q.tag = 0;
        return q;
    }
    if (in.mode == Q_VERTICES) {
        int32_t v = in.vids[i];
        q.pair = pair_of(in.voff, in.npairs, v);
        q.p = a_vertex(in.a, q.pair, v);
        q.out = v;
        q.tag = mix32((uint32_t)v ^ 0x5bd1e995u);
        return q;
    }
    if (in.mode == Q_BARYCENTERS) {
        // the barycenter of record i of the list (the fifth bound's S_b):
        // the mean of its exact corners; seeded with two corners' closest
        // triangles (records waiting for stage B keep a decider in the
        // level field's upper bits)
        const int face = in.par.face()[i], lvl = in.par.lvl()[i] & 0xff;
        q.pair = in.par.pair()[i];
        const V3<double> c0 = a_point(in.a, q.pair, face, lvl, in.par.ba(0)[i], in.par.bb(0)[i]);
        const V3<double> c1 = a_point(in.a, q.pair, face, lvl, in.par.ba(1)[i], in.par.bb(1)[i]);
        const V3<double> c2 = a_point(in.a, q.pair, face, lvl, in.par.ba(2)[i], in.par.bb(2)[i]);
        q.p = (1.0 / 3.0) * (c0 + c1 + c2);
        q.out = i;
        q.tag = 0;
        q.seed[0] = in.par.I(0)[i];
        q.seed[1] = in.par.I(1)[i];
        return q;
    }
    if (in.mode == Q_LATTICE) {
        const int64_t j = i / LATTICE_PTS;
        const int k = (int)(i - LATTICE_PTS * j);
        const int a1 = (LATTICE_A1 >> (2 * k)) & 3, a2 = (LATTICE_A2 >> (2 * k)) & 3, a0 = 4 - a1 - a2;
        const int face = in.par.face()[j], lvl = in.par.lvl()[j];
        q.pair = in.par.pair()[j];
        if (lvl + 2 <= 30) {
            const int ba = a0 * in.par.ba(0)[j] + a1 * in.par.ba(1)[j] + a2 * in.par.ba(2)[j];
            const int bb = a0 * in.par.bb(0)[j] + a1 * in.par.bb(1)[j] + a2 * in.par.bb(2)[j];
            q.p = a_point(in.a, q.pair, face, lvl + 2, ba, bb);
        } else { // not representable: the first corner (such parents are not logged)
            q.p = a_point(in.a, q.pair, face, lvl, in.par.ba(0)[j], in.par.bb(0)[j]);
        }
        q.out = i;
        q.tag = 0;
        const int heavy = a0 >= a1 && a0 >= a2 ? 0 : (a1 >= a2 ? 1 : 2);
        q.seed[0] = in.par.I(heavy)[j];
        q.seed[1] = in.par.I(heavy == 2 ? 0 : heavy + 1)[j];
        return q;
    }
    if (two_level(in.two) == 4) {
        // four-level round: every point of the parent's resolution-16 lattice
        // (corners included), at the parent's level + 4
        const int64_t js = i / LAT16_PTS;
        int a1, a2;
        lattice_point(LAT16_N, (int)(i - LAT16_PTS * js), a1, a2);
        const int a0 = LAT16_N - a1 - a2;
        const int64_t j = in.sel ? (int64_t)in.sel[js] : js;
        const int face = in.par.face()[j], lvl = in.par.lvl()[j] + 4;
        const int ba = a0 * in.par.ba(0)[j] + a1 * in.par.ba(1)[j] + a2 * in.par.ba(2)[j];
        const int bb = a0 * in.par.bb(0)[j] + a1 * in.par.bb(1)[j] + a2 * in.par.bb(2)[j];
        q.pair = in.par.pair()[j];
        q.p = a_point(in.a, q.pair, face, lvl, ba, bb);
        q.out = i;
        q.tag = point_tag(face, lvl, ba, bb);
        const int heavy = a0 >= a1 && a0 >= a2 ? 0 : (a1 >= a2 ? 1 : 2);
        q.seed[0] = in.par.I(heavy)[j];
        q.seed[1] = in.par.I(heavy == 2 ? 0 : heavy + 1)[j];
        return q;
    }
    if (two_level(in.two)) {
        const int64_t js = i / LATTICE_PTS;
        const int k = (int)(i - LATTICE_PTS * js);
        const int a1 = (LATTICE_A1 >> (2 * k)) & 3, a2 = (LATTICE_A2 >> (2 * k)) & 3, a0 = 4 - a1 - a2;
        const int64_t j = in.sel ? (int64_t)in.sel[js] : js;
        // (the plan keeps every parent at least two levels above the limit)
        const int face = in.par.face()[j], lvl = in.par.lvl()[j] + 2;
        const int ba = a0 * in.par.ba(0)[j] + a1 * in.par.ba(1)[j] + a2 * in.par.ba(2)[j];
        const int bb = a0 * in.par.bb(0)[j] + a1 * in.par.bb(1)[j] + a2 * in.par.bb(2)[j];
        q.pair = in.par.pair()[j];
        q.p = a_point(in.a, q.pair, face, lvl, ba, bb);
        q.out = i;
        q.tag = point_tag(face, lvl, ba, bb);
        const int heavy = a0 >= a1 && a0 >= a2 ? 0 : (a1 >= a2 ? 1 : 2);
        q.seed[0] = in.par.I(heavy)[j];
        q.seed[1] = in.par.I(heavy == 2 ? 0 : heavy + 1)[j];
        return q;
    }
    const int64_t js = i / 3;
    const int e = (int)(i - 3 * js);
    const int k = (e + 1) % 3;
    const int64_t j = in.sel ? (int64_t)in.sel[js] : js;
    int face = in.par.face()[j], lvl = in.par.lvl()[j] + 1;
    int ba = in.par.ba(e)[j] + in.par.ba(k)[j], bb = in.par.bb(e)[j] + in.par.bb(k)[j];
    q.pair = in.par.pair()[j];
    q.p = a_point(in.a, q.pair, face, lvl, ba, bb);
    q.out = i;
    q.tag = point_tag(face, lvl, ba, bb);
    q.seed[0] = in.par.I(e)[j];
    q.seed[1] = in.par.I(k)[j];
    return q;
}

// the pair of query i (what query_point gives, without the point)
template <class T> HD_D int query_pair(const QueryIn<T> &in, int64_t i) {
    if (in.npairs == 1 || in.mode == Q_POINTS) return 0;
    if (in.mode == Q_VERTICES) return pair_of(in.voff, in.npairs, in.vids[i]);
    if (in.mode == Q_BARYCENTERS) return in.par.pair()[i];
    if (in.mode == Q_LATTICE) return in.par.pair()[i / LATTICE_PTS];
    const int dep = two_level(in.two);
    const int64_t js = i / (dep == 4 ? LAT16_PTS : (dep ? LATTICE_PTS : 3));
    return in.par.pair()[in.sel ? (int64_t)in.sel[js] : js];
}

struct QueryCfg {
    const WideNode *nodes;
    const int4 *ids;
    int raise_L;         // fold d - mu into the lower bound and the argmax key
    const WideNode *top; // single-pair BVH: its top-level table (staged in LDS), else null
};

// writes the result; returns in *lord, *key what the pair's L and round key
// must be raised to (0: nothing)
template <class T>
HD_D void finish_query(const QueryCfg &cfg, const BView<T> &bv, const QueryResult<T> &r, const QPoint &qp,
                       const V3<T> &p, const QueryOut<T> &out, const PairConst *pc, unsigned long long *lord,
                       unsigned long long *keyout) {
    V3<T> q = p;
    T d = T(__builtin_inf());
    if (r.s >= 0) {
        Frame<T> f = load_frame(bv.frames, r.s);
        d = hsqrt(frame_dist2<T, true>(f, p, &q));
    }
    const int64_t o = qp.out;
    out.d[o] = d;
    out.I[o] = r.s < 0 ? 0 : r.s;
    out.q[0][o] = q.x;
    out.q[1][o] = q.y;
    out.q[2][o] = q.z;
    if (out.p[0]) {
        out.p[0][o] = p.x;
        out.p[1][o] = p.y;
        out.p[2][o] = p.z;
    }
    *lord = 0;
    *keyout = 0;
    if (cfg.raise_L) {
        unsigned long long key = 0;
        if (r.s >= 0) {
            const Margins &m = margins_of<T>(pc[qp.pair]);
            double dlo = (double)d - (m.mu_d * (double)d + m.mu_0);
            if (dlo > 0) {
                *lord = d2ord(dlo);
                key = ((unsigned long long)f2ord(to_float_down(dlo)) << 32) | qp.tag;
            }
        }
        *keyout = key;
        out.key[o] = key;
    }
}

// The query kernel. A launch with many queries runs one lane per query: the
// machine is full and each lane's traversal overlaps with the others. A
// launch with few queries (at most quad_max) is bound by the latency of each
// traversal's chain of dependent node loads; it runs a quad of lanes per
// query instead (see traverse4), which shortens every step of the chain.
// Both paths give each block a run of consecutive queries in the same
// XCD-aware tile order and write the same results (the quad's lane 0 writes).
struct QueryTally {
    unsigned long long nb = 0, nl = 0, nq = 0;
    int ovf = 0; // this thread listed an overflowed query
};

// XCD-aware order: the hardware deals consecutive blocks to the eight XCDs in
// turn; number the tiles so that each XCD takes a contiguous run of them
// (nearby points, shared BVH paths, hits in that XCD's L2). A grid that is
// not a multiple of XCDS takes them in plain order.
struct TileOrder {
    int64_t ntiles, per;
    unsigned xs, x, gx, first;
    HD_D TileOrder(int64_t n, int tile) {
        ntiles = (n + tile - 1) / tile;
        xs = gridDim.x % XCDS == 0 ? XCDS : 1;
        per = (ntiles + xs - 1) / xs;
        x = blockIdx.x % xs;
        gx = gridDim.x / xs;
        first = blockIdx.x / xs;
    }
    HD_D bool valid(int64_t tt) const { return tt < per && x * per + tt < ntiles; }
    HD_D int64_t tile(int64_t tt) const { return x * per + tt; }
    // whether this block has a tile
    HD_D bool active() const { return valid(first); }
    // the blocks of XCD slot y with a tile: first = 0 .. lim(y) - 1
    HD_D int64_t lim(unsigned y) const {
        int64_t k = ntiles - (int64_t)y * per;
        k = k < per ? k : per;
        k = k < (int64_t)gx ? k : (int64_t)gx;
        return k > 0 ? k : 0;
    }
    // last_block over the blocks with a tile: way first % LB_WAYS, its share
    // summed over the XCD slots, and the ways that have blocks (slot 0 has
    // the most); one way for small grids
    HD_D bool last(BlockCounter *c, bool release) const {
        unsigned total = 0;
        for (unsigned y = 0; y < xs; ++y) total += (unsigned)lim(y);
        if (total <= LB_SPLIT_MIN) return last_block(c, 0, total, 1, release);
        const unsigned w = first % LB_WAYS;
        unsigned share = 0;
        for (unsigned y = 0; y < xs; ++y) share += way_share((unsigned)lim(y), w);
        const int64_t l0 = lim(0);
        return last_block(c, w, share, (unsigned)(l0 < LB_WAYS ? l0 : LB_WAYS), release);
    }
};

template <class T, int SD, int QB>
__device__ void query_lanes1(const QueryIn<T> &in, int64_t n, const TileOrder &to, const QueryCfg &cfg,
                             const NodeSrc &ns, const BView<T> &bv, const QueryOut<T> &out,
                             const PairConst *__restrict__ pc, PairVar *pv, Ctl *ctl, int32_t *ovf_list, int *s_node,
                             float *s_dist, QueryTally &t) {
    for (int64_t tt = to.first; to.valid(tt); tt += to.gx) {
        const int64_t i = to.tile(tt) * QB + threadIdx.x;
        unsigned long long lord = 0, key = 0;
        int pair = 0;
        if (i < n) {
            QPoint qp = query_point(in, i);
            pair = qp.pair;
            V3<T> p = cvt<T>(qp.p);
            QueryResult<T> r = empty_result<T>();
            seed_two(r, bv, p, qp.seed[0], qp.seed[1]);
            LdsStack<SD, QB> stk{s_node, s_dist, 0};
            r = traverse<T>(ns, bv, cfg.ids, p, cfg.top ? TOP_REF : pc[qp.pair].root, stk, r);
            t.nb += r.nbox;
            t.nl += r.nleaf;
            t.nq += 1;
            if (r.overflow) {
                int k = atomicAdd(&ctl->n_overflow, 1);
                ovf_list[k] = (int32_t)i;
                t.ovf = 1;
            } else {
                finish_query<T>(cfg, bv, r, qp, p, out, pc, &lord, &key);
            }
        }
        pair_max2(pv, pair, lord, key);
    }
}

template <class T, int SD, int QB>
__device__ void query_lanes4(const QueryIn<T> &in, int64_t n, const TileOrder &to, const QueryCfg &cfg,
                             const NodeSrc &ns, const BView<T> &bv, const QueryOut<T> &out,
                             const PairConst *__restrict__ pc, PairVar *pv, Ctl *ctl, int32_t *ovf_list, int *s_node,
                             float *s_dist, QueryTally &t) {
    constexpr int NQ = QB / 4; // queries per tile
    const int g = threadIdx.x >> 2, k = threadIdx.x & 3;
    for (int64_t tt = to.first; to.valid(tt); tt += to.gx) {
        const int64_t i = to.tile(tt) * NQ + g;
        unsigned long long lord = 0, key = 0;
        int pair = 0;
        if (i < n) { // the same for the four lanes of a quad
            QPoint qp = query_point(in, i);
            pair = qp.pair;
            V3<T> p = cvt<T>(qp.p);
            QueryResult<T> r = empty_result<T>();
            // the two candidate triangles: one lane each
            const int seed = k == 0 ? qp.seed[0] : (k == 1 && qp.seed[1] != qp.seed[0] ? qp.seed[1] : -1);
            if (seed >= 0) visit_leaf(r, bv, cfg.ids, p, seed);
            quad_min(r);
            QuadStack<SD, NQ> stk{s_node, s_dist, g};
            r = traverse4<T>(ns, bv, cfg.ids, p, cfg.top ? TOP_REF : pc[qp.pair].root, stk, r, k);
            t.nb += r.nbox;
            t.nl += r.nleaf;
            if (k == 0) {
                t.nq += 1;
                if (r.overflow) {
                    int slot = atomicAdd(&ctl->n_overflow, 1);
                    ovf_list[slot] = (int32_t)i;
                    t.ovf = 1;
                } else {
                    finish_query<T>(cfg, bv, r, qp, p, out, pc, &lord, &key);
                }
            }
        }
        pair_max2(pv, pair, lord, key);
    }
}

template <class T>
__device__ void deep_queries(const QueryIn<T> &in, const QueryCfg &cfg, const BView<T> &bv, const QueryOut<T> &out,
                             const PairConst *__restrict__ pc, PairVar *pv, Ctl *ctl, const int32_t *ovf_list,
                             int2 *stack_mem);

// ... and the block that finishes last redoes the queries whose LDS stack
// overflowed (deep_queries).
template <class T, int SD, int QB>
__global__ __launch_bounds__(QB) void k_query(QueryIn<T> in, DevCount cnt, QueryCfg cfg, BView<T> bv,
                                              QueryOut<T> out, const PairConst *__restrict__ pc, PairVar *pv,
                                              Ctl *ctl, int32_t *ovf_list, int2 *deep_stack, int64_t quad_max) {
    static_assert(QB <= DEEP_SLOTS, "every thread of the last block has a deep-stack slot");
    __shared__ int s_node[SD * QB];
    __shared__ float s_dist[SD * QB];
    constexpr int TOP_F4 = WIDE_WORDS / 4; // float4 per table entry
    __shared__ float4 s_top[TOP_NODES * TOP_F4];
    const int64_t n = cnt.get();
    const bool quad = n <= quad_max;
    const TileOrder to(n, quad ? QB / 4 : QB);
    if (!to.active()) return; // the grid is sized for a larger count
    QueryTally t;
    // stage the top levels of the tree, where every traversal starts (and
    // every greedy descent passes), in LDS: the words a traversal reads of
    // each entry (without a table no reference reaches the copy)
    if (cfg.top) {
        const float4 *src = reinterpret_cast<const float4 *>(cfg.top);
        constexpr int NODE_F4 = (int)(sizeof(WideNode) / 16);
        for (int i = threadIdx.x; i < TOP_NODES * TOP_F4; i += QB) s_top[i] = src[(i / TOP_F4) * NODE_F4 + i % TOP_F4];
        __syncthreads();
    }
    const NodeSrc ns{cfg.nodes, (LdsFloat *)s_top};
    if (quad)
        query_lanes4<T, SD, QB>(in, n, to, cfg, ns, bv, out, pc, pv, ctl, ovf_list, s_node, s_dist, t);
    else
        query_lanes1<T, SD, QB>(in, n, to, cfg, ns, bv, out, pc, pv, ctl, ovf_list, s_node, s_dist, t);
    unsigned long long *st = ctl->stat[acc_copy()];
    block_add<3, QB>({t.nb, t.nl, t.nq}, {st + ST_BOXES, st + ST_QLEAVES, st + ST_QUERIES});
    // the last block reads only the overflow list (and its atomic count);
    // then, the round keys being final, whether the argmax step has work:
    // some pair's best point of the round beats its best so far and, taken
    // to FP64, could raise L. (The computed distance is within the margin of
    // the exact one, so the FP64 lower bound of that point is at most its
    // key's lower bound plus twice the margin.)
    if (to.last(&ctl->q_done, __syncthreads_or(t.ovf) != 0)) {
        deep_queries<T>(in, cfg, bv, out, pc, pv, ctl, ovf_list, deep_stack);
        if (cfg.raise_L) {
            __syncthreads();
            int fresh = 0;
            for (int p = threadIdx.x; p < in.npairs; p += QB) {
                const unsigned long long rk =
                    __hip_atomic_load(&pv[p].round_key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if (rk <= pv[p].best_key) continue;
                const Margins &m = margins_of<T>(pc[p]);
                const double lo = (double)next_up(ord2f((uint32_t)(rk >> 32))); // above the key's d - mu
                const double d = (lo + m.mu_0) / (1.0 - m.mu_d);                 // above the computed d
                const double reach = (lo + 2.0 * (m.mu_d * d + m.mu_0)) * (1.0 + 1e-9);
                const unsigned long long a =
                    __hip_atomic_load(&pv[p].Lord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                const unsigned long long b =
                    __hip_atomic_load(&pv[pc[p].link].Lord, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                fresh |= reach > ord2d(a > b ? a : b);
            }
            fresh = __syncthreads_or(fresh);
            if (threadIdx.x == 0) ctl->argmax_new = fresh;
        }
    }
}

// queries whose LDS stack overflowed, redone with a deep stack in global
// memory by the threads of one block (thread t uses stack slot t of
// DEEP_SLOTS); the list is empty but for unusual trees
template <class T>
__device__ void deep_queries(const QueryIn<T> &in, const QueryCfg &cfg, const BView<T> &bv, const QueryOut<T> &out,
                             const PairConst *__restrict__ pc, PairVar *pv, Ctl *ctl, const int32_t *ovf_list,
                             int2 *stack_mem) {
    const int novf = ctl->n_overflow;
    unsigned long long nb = 0, nl = 0;
    for (int k = threadIdx.x; k < novf; k += blockDim.x) {
        int64_t i = ovf_list[k];
        QPoint qp = query_point(in, i);
        V3<T> p = cvt<T>(qp.p);
        QueryResult<T> r = empty_result<T>();
        seed_two(r, bv, p, qp.seed[0], qp.seed[1]);
        GlobalStack stk{stack_mem + threadIdx.x, DEEP_SLOTS, DEEP_STACK, 0};
        r = traverse<T>(NodeSrc{cfg.nodes, nullptr}, bv, cfg.ids, p, pc[qp.pair].root, stk, r);
        nb += r.nbox;
        nl += r.nleaf;
        // a traversal deeper than the fallback stack fails the call; its
        // (possibly suboptimal) result is still written so that later
        // kernels read initialised indices
        if (r.overflow) ctl->bad = 2;
        unsigned long long lord, key;
        finish_query<T>(cfg, bv, r, qp, p, out, pc, &lord, &key);
        if (lord) atomicMax(&pv[qp.pair].Lord, lord);
        if (key) atomicMax(&pv[qp.pair].round_key, key);
    }
    wave_add(&ctl->stat[acc_copy()][ST_BOXES], nb);
    wave_add(&ctl->stat[acc_copy()][ST_QLEAVES], nl);
    // the list is done: a later query launch of the same round starts empty
    __syncthreads();
    if (threadIdx.x == 0) {
        if (novf) atomicAdd(&ctl->stat[acc_copy()][ST_OVERFLOWS], (unsigned long long)novf);
        ctl->n_overflow = 0;
    }
}

// Launch shapes of the query kernel (LDS stack entries per query, block
// size) that the autotuner chooses from; entry 0 is the default.
struct QVariant {
    int sd, qb;
};
constexpr QVariant QVARIANTS[] = {{16, 128}, {8, 64}, {16, 64}, {32, 128}, {8, 256},
                                   {16, 256}, {12, 128}, {12, 256}, {24, 128}};
constexpr int NQVAR = sizeof(QVARIANTS) / sizeof(QVARIANTS[0]);
static_assert(NQVAR == HD_QUERY_SHAPES, "the header counts the launch shapes");

// Launches of at most this many queries run a quad of lanes per query. Below
// it the one-lane kernel holds too few waves to hide its latency: measured
// on MI355X, a quad per query is about 30% faster for launches of a few
// thousand queries or fewer, even around 25k, and up to 2.5x slower for
// launches of 10^5 queries and more (there every lane's redundant share of
// the sort and stack work costs issue slots).
constexpr int64_t QUAD_MAX_DEFAULT = 32768;

// grid of a query launch of block size qb for up to n queries: a multiple of
// XCDS, capped at a persistent size; launches that may take the quad path
// get four lanes per query
inline unsigned qgrid_b(int64_t n, int qb, int64_t quad_max) {
    const int64_t lanes = n <= quad_max ? 4 : 1;
    const unsigned g = (unsigned)std::min<int64_t>((lanes * n + qb - 1) / qb, (int64_t)QGRID_MAX * 128 / qb);
    return std::max<unsigned>((g + XCDS - 1) / XCDS * XCDS, XCDS);
}

// variant v (-1: the tiny-stack test hook) for up to n_max queries; launches
// of at most quad_max queries (by the count the kernel reads) take the quad
// path; deep: DEEP_SLOTS x DEEP_STACK entries for the overflowed queries
template <class T>
void launch_query(int v, int64_t n_max, int64_t quad_max, const QueryIn<T> &qi, DevCount cnt, const QueryCfg &cfg,
                  const BView<T> &bv, const QueryOut<T> &out, const PairConst *pc, PairVar *pv, Ctl *ctl,
                  int32_t *ovf, int2 *deep, hipStream_t s) {
#define HD_QLAUNCH(SD, QB)                                                                                             \
    k_query<T, SD, QB><<<qgrid_b(n_max, QB, quad_max), QB, 0, s>>>(qi, cnt, cfg, bv, out, pc, pv, ctl, ovf, deep,    \
                                                                    quad_max)
    switch (v) {
    case -1: HD_QLAUNCH(SMALL_STACK, 128); break;
    case 1: HD_QLAUNCH(8, 64); break;
    case 2: HD_QLAUNCH(16, 64); break;
    case 3: HD_QLAUNCH(32, 128); break;
    case 4: HD_QLAUNCH(8, 256); break;
    case 5: HD_QLAUNCH(16, 256); break;
    case 6: HD_QLAUNCH(12, 128); break;
    case 7: HD_QLAUNCH(12, 256); break;
    case 8: HD_QLAUNCH(24, 128); break;
    default: HD_QLAUNCH(16, 128); break;
    }
#undef HD_QLAUNCH
    HD_LAUNCH_CHECK();
}

__global__ void k_zero_query_stats(Ctl *c) {
    const int k = threadIdx.x;
    if (k < ACC_COPIES)
        c->stat[k][ST_QUERIES] = c->stat[k][ST_BOXES] = c->stat[k][ST_QLEAVES] = c->stat[k][ST_OVERFLOWS] = 0;
    if (k == 0) c->n_overflow = 0;
}

// FP64 distance of pair p's best vertex when it changed: the lower bound
// then carries the FP64 margin instead of the FP32 one, which the recheck
// band needs to park triangles within eps of it
HD_D void l64_pair(const NodeSrc &ns, const BView<double> &bv64, const int4 *ids, const PairConst *pc,
                         PairVar *pv, int p, int npairs, int2 *stack_mem, int k) {
    // run by the four lanes of a quad (k = lane in the quad): all read, lane 0 writes
    PairVar &P = pv[p];
    const PairConst &C = pc[p];
    const unsigned long long rk = P.round_key, bk = P.best_key;
    const int dirty = P.argmax_dirty;
    const V3<double> x = {P.argmax_pos[0], P.argmax_pos[1], P.argmax_pos[2]};
    const int tri = P.argmax_tri;
    if (k == 0) {
        if (rk > bk) P.best_key = rk;
        P.round_key = 0;
        P.argmax_dirty = 0;
    }
    if (!dirty) return;
    // every lane of the quad sees the same stack state and writes the same entries
    GlobalStack stk{stack_mem + p, npairs, DEEP_STACK, 0};
    // the FP32 query's closest triangle bounds the FP64 distance from above,
    // so the traversal starts with a tight pruning radius
    QueryResult<double> r = empty_result<double>();
    if (k == 0) visit_leaf(r, bv64, ids, x, tri);
    quad_min(r);
    r = traverse4<double>(ns, bv64, ids, x, C.root, stk, r, k);
    if (k != 0 || r.overflow || r.s < 0) return;
    double d = sqrt(r.d2);
    double dlo = d - (C.m64.mu_d * d + C.m64.mu_0);
    P.L64 = dlo;
    if (dlo > 0 && d2ord(dlo) > P.Lord) P.Lord = d2ord(dlo);
}

struct L64Cfg {
    const WideNode *nodes;
    BView<double> bv64;
    const int4 *ids;
    const PairConst *pc;
    int npairs;
    int2 *stack_mem; // npairs x DEEP_STACK entries
    int check_fp32;  // plain FP32 rounds: the tolerance must exceed the margin at L
};

// pair p's FP64 argmax step (l64_pair) by the four lanes of a quad, then
// the plain-FP32 tolerance check. Plain FP32 parks a triangle only when its
// bound plus the FP32 margin lies within the tolerance of L; near the
// maximum that margin tends to mu_d * h + mu_0 as the triangles shrink, so a
// tolerance below it cannot be reached (the rounds would split to the depth
// limit).
constexpr int ARGMAX_LAST_BLOCK_PAIRS = BLK / 4;
__device__ void argmax_step(const L64Cfg &lc, PairVar *pv, int p, Ctl *ctl) {
    __shared__ float4 s_none[1]; // no top-level table here (no reference reaches it)
    const NodeSrc ns{lc.nodes, (LdsFloat *)s_none};
    l64_pair(ns, lc.bv64, lc.ids, lc.pc, pv, p, lc.npairs, lc.stack_mem, threadIdx.x & 3);
    if (lc.check_fp32 && (threadIdx.x & 3) == 0) {
        const PairConst &C = lc.pc[p];
        if (C.eps_abs <= C.m32.mu_d * pair_L(lc.pc, pv, p) + C.m32.mu_0) ctl->bad = 5;
    }
}

// after a query round: the query holding its pair's best key records its
// exact position (keys are unique up to a tag collision of one point); the
// block that finishes last then takes each pair's new best point to FP64
// (a quad of lanes per pair: the traversal is one latency-bound chain)
template <class T>
__global__ __launch_bounds__(BLK) void k_argmax_finalize(QueryIn<T> in, DevCount cnt,
                                                         const unsigned long long *__restrict__ keys,
                                                         const int *__restrict__ tri, PairVar *pv, L64Cfg lc, Ctl *ctl) {
    const int64_t n = cnt.get();
    if ((int64_t)blockIdx.x * BLK >= n) return; // the grid is sized for a larger count
    if (!ctl->argmax_new) {
        // no key above its pair's best: no new point, L stands; only the
        // plain-FP32 tolerance check (L may still have risen within the
        // rounding of a key)
        if (blockIdx.x == 0 && lc.check_fp32)
            for (int p = threadIdx.x; p < lc.npairs; p += blockDim.x) {
                const PairConst &C = lc.pc[p];
                if (C.eps_abs <= C.m32.mu_d * pair_L(lc.pc, pv, p) + C.m32.mu_0) ctl->bad = 5;
            }
        return;
    }
    int wrote = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int64_t o = in.mode == Q_VERTICES ? in.vids[i] : i;
        unsigned long long key = keys[o];
        if (key == 0) continue;
        const PairVar &Pq = pv[query_pair(in, i)];
        if (key != Pq.round_key || key <= Pq.best_key) continue;
        QPoint qp = query_point(in, i);
        PairVar &P = pv[qp.pair];
        if (key == P.round_key && key > P.best_key) {
            P.argmax_pos[0] = qp.p.x;
            P.argmax_pos[1] = qp.p.y;
            P.argmax_pos[2] = qp.p.z;
            P.argmax_tri = tri[o];
            P.argmax_dirty = 1;
            wrote = 1;
        }
    }
    // many pairs: their FP64 steps run in k_argmax_pairs, a quad per pair
    // over as many blocks as needed, instead of in turns in one block
    if (lc.npairs > ARGMAX_LAST_BLOCK_PAIRS) return;
    const int64_t need = (n + BLK - 1) / BLK;
    // the last block reads only the argmax records (written by one block)
    if (last_block(&ctl->f_done, (unsigned)(need < (int64_t)gridDim.x ? need : (int64_t)gridDim.x),
                   __syncthreads_or(wrote) != 0)) {
        for (int p = threadIdx.x >> 2; p < lc.npairs; p += blockDim.x >> 2) argmax_step(lc, pv, p, ctl);
    }
}

// the FP64 argmax steps of more than ARGMAX_LAST_BLOCK_PAIRS pairs, after
// k_argmax_finalize (which wrote the argmax records): a quad per pair
__global__ __launch_bounds__(BLK) void k_argmax_pairs(PairVar *pv, L64Cfg lc, Ctl *ctl) {
    if (!ctl->argmax_new) return; // (k_argmax_finalize made the plain-FP32 check)
    const int p = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 2);
    if (p < lc.npairs) argmax_step(lc, pv, p, ctl);
}

// ---------------------------------------------------------------------------
// bounding children (or round-0 faces), classifying them and appending the
// survivors to the active or parked list
// ---------------------------------------------------------------------------
struct ClassifyCfg {
    CascadeCtx c;
    int recheck; // FP32 + FP64 recheck of the ambiguity band
    double shift; // test hook: subtracted from every bound of stages A and B
    AView a;
    BView<double> bv64;
    IdView iv;
    const PairConst *pc;
    const PairVar *pv;
};

template <class T> struct Corner {
    V3<T> v, q;
    T d;
    int I, ba, bb;
};

// The cascade runs in three stages, each its own kernel, so that the
// frequent cheap cases do not carry the registers of the expensive ones:
//   A: the exact bound, then the bounds listed before u3 in the order;
//   B: u3 and every bound after it (triangles A could not decide);
//   C: the FP64 re-bound of triangles whose decision lies within the FP32
//      margin (the recheck band).
// The decision is the same as the one-pass cascade in the same order.
enum { TO_DISCARD = -1, TO_ACT = 0, TO_PARK = 1, TO_B = 2, TO_C = 3 };

template <class T> HD_D Tri<T> make_tri(const Corner<T> cn[3]) {
    Tri<T> t;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        t.v[i] = cn[i].v;
        t.q[i] = cn[i].q;
        t.d[i] = cn[i].d;
        t.I[i] = cn[i].I;
    }
    return t;
}

HD_D double park_limit(double eps) { return eps * (1.0 - 1.0 / 1024.0 / 1024.0 / 1024.0); }

HD_D float round_up_to_float(double x) {
    float f = (float)x;
    if ((double)f < x) f = next_up(f);
    return f;
}

// list for a final bound ub (margin mu included). Records keep their bound
// rounded up to FP32, and the final U is taken over those stored values (or
// the FP64 re-bound when smaller): a triangle is parked only when its stored
// bound lies within eps of L.
HD_D int decide(double ub, double L, double eps, double mu, bool recheck) {
    const double lim = park_limit(eps);
    const double stored = (double)round_up_to_float(ub);
    if (recheck) {
        bool maybe_discard = ub >= L && ub - 2 * mu < L;
        bool maybe_park = stored - L > lim && ub - 2 * mu - L <= lim;
        if (maybe_discard || maybe_park) return TO_C;
    }
    return ub < L ? TO_DISCARD : (stored - L <= lim ? TO_PARK : TO_ACT);
}

template <class T> HD_D T bound_cheap(int k, const Tri<T> &t) {
    return k == 1 ? bound_u1(t) : (k == 2 ? bound_u2(t) : bound_u4(t));
}

// A valid upper bound over T is at least the distance at each vertex of T,
// and a computed one plus its margin at least the computed vertex distance
// minus that margin: a bound below is unsound (flagged in *unsound).
template <class T> HD_D void check_sound(double u, const Tri<T> &t, double mu, int *unsound) {
    if (u < (double)hmax(t.d[0], hmax(t.d[1], t.d[2])) - mu) *unsound = 1;
}

// stage A; *carry receives the running minimum for stage B
template <class T>
HD_D int stage_a(const Corner<T> cn[3], int pair, const ClassifyCfg &cc, double *carry, int *decider,
                 int *unsound) {
    const Tri<T> t = make_tri(cn);
    const PairConst &P = cc.pc[pair];
    const double L = pair_L(cc.pc, cc.pv, pair);
    const double mu = tri_margin(t, margins_of<T>(P));
    if (t.I[0] == t.I[1] && t.I[1] == t.I[2]) {
        *decider = 0;
        double ub = (double)hmax(t.d[0], hmax(t.d[1], t.d[2])) - cc.shift + mu;
        check_sound(ub, t, mu, unsound);
        *carry = ub;
        return decide(ub, L, P.eps_abs, mu, cc.recheck);
    }
    double best = __builtin_inf();
    *decider = cc.c.order[cc.c.norder - 1];
    for (int i = 0; i < cc.c.norder; ++i) {
        int k = cc.c.order[i];
        if (k == 3 || k == 5) { // the bounds that evaluate at fixed B triangles: stage B
            *carry = best;
            return TO_B;
        }
        double u = (double)bound_cheap<T>(k, t) - cc.shift + mu;
        check_sound(u, t, mu, unsound);
        if (u < L) {
            *decider = k;
            *carry = u;
            return TO_DISCARD;
        }
        if (u < best) {
            best = u;
            *decider = k;
        }
    }
    *carry = best;
    return decide(best, L, P.eps_abs, mu, cc.recheck);
}

// stage B: u3 and the bounds after it, from the running minimum `best`
template <class T>
HD_D int stage_b(const Corner<T> cn[3], int pair, const ClassifyCfg &cc, const BView<T> &bv, double best,
                 int best_k, double *carry, int *decider, int *evals, int *unsound, int Sb) {
    const Tri<T> t = make_tri(cn);
    const PairConst &P = cc.pc[pair];
    const double L = pair_L(cc.pc, cc.pv, pair);
    const double mu = tri_margin(t, margins_of<T>(P));
    int i3 = 0;
    while (cc.c.order[i3] != 3 && cc.c.order[i3] != 5) ++i3;
    *decider = best_k;
    for (int i = i3; i < cc.c.norder; ++i) {
        int k = cc.c.order[i];
        const T b = k == 3 ? bound_u3(t, bv, cc.iv, nullptr, evals)
                           : (k == 5 ? bound_u5(t, bv, Sb, evals) : bound_cheap<T>(k, t));
        double u = (double)b - cc.shift + mu;
        check_sound(u, t, mu, unsound);
        if (u < L) {
            *decider = k;
            *carry = u;
            return TO_DISCARD;
        }
        if (u < best) {
            best = u;
            *decider = k;
        }
    }
    *carry = best;
    return decide(best, L, P.eps_abs, mu, cc.recheck);
}

template <class T>
HD_D void write_record(const FrontierView<T> &fo, int64_t o, const Corner<T> cn[3], float ub, int face, int lvl,
                       int pair) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        fo.v(3 * i)[o] = cn[i].v.x;
        fo.v(3 * i + 1)[o] = cn[i].v.y;
        fo.v(3 * i + 2)[o] = cn[i].v.z;
        fo.q(3 * i)[o] = cn[i].q.x;
        fo.q(3 * i + 1)[o] = cn[i].q.y;
        fo.q(3 * i + 2)[o] = cn[i].q.z;
        fo.d(i)[o] = cn[i].d;
        fo.I(i)[o] = cn[i].I;
        fo.ba(i)[o] = cn[i].ba;
        fo.bb(i)[o] = cn[i].bb;
    }
    fo.ub()[o] = ub;
    fo.face()[o] = face;
    fo.lvl()[o] = lvl;
    fo.pair()[o] = pair;
    fo.score()[o] = __builtin_nanf("");
}

// Records waiting for stage B or C carry the index of the bound that gave
// their running minimum in bits 8.. of the level field.
HD_D int lvl_field(int list, int lvl, int decider) { return list >= TO_B ? lvl | (decider << 8) : lvl; }

// Block-aggregated append to one of four lists (TO_ACT, TO_PARK, TO_B, TO_C;
// anything else appends nothing): one atomic per block and list; records of
// one block stay in thread order. Every thread of the block must call it.
__device__ int64_t append_slot(int list, Ctl *ctl) {
    __shared__ int wc[4][NW];
    __shared__ unsigned long long base[4];
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    unsigned long long m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        m[k] = __ballot(list == k);
        if (lane == 0) wc[k][w] = __popcll(m[k]);
    }
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        int tot = 0;
        for (int j = 0; j < NW; ++j) {
            int c = wc[k][j];
            wc[k][j] = tot;
            tot += c;
        }
        unsigned long long *ctr = k == 0 ? &ctl->act_next : (k == 1 ? &ctl->park_next : (k == 2 ? &ctl->b_next : &ctl->c_next));
        base[k] = tot ? atomicAdd(ctr, (unsigned long long)tot) : 0;
    }
    __syncthreads();
    int64_t slot = -1;
#pragma unroll
    for (int k = 0; k < 4; ++k)
        if (list == k) slot = (int64_t)(base[k] + wc[k][w] + __popcll(m[k] & lt));
    __syncthreads();
    return slot;
}

// block-aggregated statistics of a cascade kernel (every thread must call it)
__device__ void tally(Ctl *ctl, int list, int decider, int evals, int rechecked, bool valid, bool bounded) {
    const bool dis = valid && list == TO_DISCARD;
    unsigned long long *st = ctl->stat[acc_copy()];
    block_add<9, BLK>({dis && decider == 0 ? 1ull : 0ull, dis && decider == 1 ? 1ull : 0ull,
                       dis && decider == 2 ? 1ull : 0ull, dis && decider == 3 ? 1ull : 0ull,
                       dis && decider == 4 ? 1ull : 0ull, dis && decider == 5 ? 1ull : 0ull,
                       valid ? (unsigned long long)evals : 0ull, valid ? (unsigned long long)rechecked : 0ull,
                       valid && bounded ? 1ull : 0ull},
                      {st + ST_DISCARDS, st + ST_DISCARDS + 1, st + ST_DISCARDS + 2, st + ST_DISCARDS + 3,
                       st + ST_DISCARDS + 4, st + ST_DISCARDS + 5, st + ST_EVALS, st + ST_RECHECKED,
                       st + ST_BOUNDED});
}

template <class T> struct Dest {
    FrontierView<T> act, park, b, c;
};

// A wave-uniform 64-bit value passed through readfirstlane: the compiler can
// no longer trace it to the kernel argument it was loaded from, so a per-lane
// choice between such values stays a register select (choosing between the
// argument fields themselves makes it copy the argument struct to scratch
// memory and index that).
HD_D uint64_t uniform_value(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// append a record to list `list` of d (nothing for TO_DISCARD)
template <class T>
HD_D void write_to(const Dest<T> &d, int list, int64_t o, const Corner<T> cn[3], float ub, int face, int lvl,
                   int pair) {
    if (list < 0) return;
    const uint64_t b0 = uniform_value((uint64_t)d.act.base), b1 = uniform_value((uint64_t)d.park.base),
                   b2 = uniform_value((uint64_t)d.b.base), b3 = uniform_value((uint64_t)d.c.base);
    const uint64_t c0 = uniform_value((uint64_t)d.act.cap), c1 = uniform_value((uint64_t)d.park.cap),
                   c2 = uniform_value((uint64_t)d.b.cap), c3 = uniform_value((uint64_t)d.c.cap);
    const uint64_t b = list == TO_ACT ? b0 : (list == TO_PARK ? b1 : (list == TO_B ? b2 : b3));
    const uint64_t c = list == TO_ACT ? c0 : (list == TO_PARK ? c1 : (list == TO_B ? c2 : c3));
    write_record(FrontierView<T>{(char *)b, (int64_t)c}, o, cn, ub, face, lvl, pair);
}

// load a record's corners
template <class T> HD_D void load_corners(const FrontierView<T> &f, int64_t j, Corner<T> cn[3]) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        cn[i].v = {f.v(3 * i)[j], f.v(3 * i + 1)[j], f.v(3 * i + 2)[j]};
        cn[i].q = {f.q(3 * i)[j], f.q(3 * i + 1)[j], f.q(3 * i + 2)[j]};
        cn[i].d = f.d(i)[j];
        cn[i].I = f.I(i)[j];
        cn[i].ba = f.ba(i)[j];
        cn[i].bb = f.bb(i)[j];
    }
}

// round 0: every face of A from the per-vertex query results (stage A)
// (FUSE: as in k_children, stage B for an undecided triangle at once)
template <class T, int FUSE = 0>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(FUSE ? 3 : 1))) void k_round0(
    int64_t nA, const int32_t *__restrict__ F, const int32_t *__restrict__ fpair, QueryOut<T> vq, ClassifyCfg cc,
    Dest<T> dst, Ctl *ctl, BView<T> bv) {
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool valid = f < nA;
    int list = TO_DISCARD, decider = 0, pair = 0, evals = 0;
    double carry = 0;
    Corner<T> cn[3];
    if (valid) {
        pair = fpair[f];
        for (int j = 0; j < 3; ++j) {
            int32_t v = F[3 * f + j];
            cn[j].v = {vq.p[0][v], vq.p[1][v], vq.p[2][v]};
            cn[j].q = {vq.q[0][v], vq.q[1][v], vq.q[2][v]};
            cn[j].d = vq.d[v];
            cn[j].I = vq.I[v];
            cn[j].ba = (j == 1);
            cn[j].bb = (j == 2);
        }
        int unsound = 0;
        list = stage_a<T>(cn, pair, cc, &carry, &decider, &unsound);
        if (FUSE && list == TO_B)
            list = stage_b<T>(cn, pair, cc, bv, (double)round_up_to_float(carry), decider, &carry, &decider, &evals,
                              &unsound, -1);
        if (unsound) ctl->bad = 4;
    }
    int64_t slot = append_slot(valid ? list : TO_DISCARD, ctl);
    if (valid)
        write_to(dst, list, slot, cn, round_up_to_float(carry), (int)f, lvl_field(list, 0, decider), pair);
    tally(ctl, list, decider, evals, 0, valid, true);
}

template <class T> HD_D void copy_record(const FrontierView<T> &src, int64_t i, const FrontierView<T> &dst, int64_t o);

// round k: child c of selected parent c/4, from the parent's record and the
// three midpoint query results (midpoint e joins parent vertices e and e+1).
// carry (device-planned rounds): the records the round does not split,
// par[nsel .. nsel + plan_rest), move to the head of the active output,
// ahead of the appended children (plan_round starts the append count there).
// With sel and rest (device sub-batch selection) the parents and the carried
// records are the ones those index lists name.
//
// A two-level round (ctl->plan_two == 2, planned rounds only) gives every
// parent its 16 grandchildren instead (a four-level round, below, its 256
// descendants): the unit triangles of its resolution-4 lattice, (i,j) (i+1,j) (i,j+1) for i + j <= 3 and (i+1,j) (i+1,j+1)
// (i,j+1) for i + j <= 2, with (i,j) the weights of parent corners 1 and 2
// over 4 (so each keeps the parent's orientation). TWO_CORNER[c] holds, four
// bits per grandchild, where its corner c comes from: 0..11 the parent's
// lattice query of that index, 12..14 the parent's corner 0..2.
// (The two forms are separate instantiations, both enqueued in planned
// breadth-first rounds, the one that does not match the plan returning at
// once: in one kernel the two-level form's registers would cost the large
// one-level rounds occupancy.)
//
// FUSE (FP32, orders without the fifth bound, no learned bound policy): a
// child that stage A leaves undecided goes through stage B at once, in
// registers, instead of being written to stage B's list and read back by
// k_stage_b (which then finds that list empty); the one-level form is
// compiled, as k_stage_b is, for three waves per SIMD.
constexpr uint64_t TWO_CORNER[3] = {0x567230567823401cull, 0x9ab673d9ab567230ull, 0x6783419abe678341ull};
template <class T, int TWO, int FUSE = 0>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(FUSE && !TWO ? 3 : 1))) void k_children(
    DevCount nselc, FrontierView<T> par, QueryOut<T> mq, ClassifyCfg cc, Dest<T> dst, Ctl *ctl, int carry,
    const int32_t *__restrict__ sel, const int32_t *__restrict__ rest, BView<T> bv) {
    if (carry && (ctl->plan_two != 0) != (TWO != 0)) return;
    const int64_t nsel = nselc.get();
    if (carry) {
        const int64_t nrest = (int64_t)ctl->plan_rest;
        for (int64_t o = (int64_t)blockIdx.x * BLK + threadIdx.x; o < nrest; o += (int64_t)gridDim.x * BLK)
            copy_record(par, rest ? (int64_t)rest[o] : nsel + o, dst.act, o);
    }
    constexpr bool two = TWO != 0;
    const int dep = two ? ctl->plan_two : 0; // 2: 16 grandchildren; 4: 256 descendants
    const int64_t nkids = (dep == 4 ? 256 : (two ? 16 : 4)) * nsel;
    for (int64_t cbase = (int64_t)blockIdx.x * BLK; cbase < nkids; cbase += (int64_t)gridDim.x * BLK) {
    const int64_t c = cbase + threadIdx.x;
    bool valid = c < nkids;
    int list = TO_DISCARD, decider = 0, pair = 0, face = 0, lvl = 0;
    double carry = 0;
    Corner<T> cn[3];
    if (valid && two && dep == 4) {
        // four-level round: unit triangle g of the parent's resolution-16
        // lattice; its strip r (between rows a2 = r and r + 1) holds 2(N - r) - 1
        // triangles, up (i,r) (i+1,r) (i,r+1) and down (i+1,r) (i+1,r+1) (i,r+1)
        // alternating; every lattice point, corners included, was queried
        constexpr int N = LAT16_N;
        const int64_t js = c >> 8;
        const int64_t j = sel ? (int64_t)sel[js] : js;
        int g = (int)(c & 255), r = 0;
        while (g >= 2 * (N - r) - 1) {
            g -= 2 * (N - r) - 1;
            ++r;
        }
        const int i0 = g >> 1;
        const bool up = (g & 1) == 0;
        const int ca1[3] = {up ? i0 : i0 + 1, i0 + 1, i0};
        const int ca2[3] = {r, up ? r : r + 1, r + 1};
        const int pba[3] = {par.ba(0)[j], par.ba(1)[j], par.ba(2)[j]};
        const int pbb[3] = {par.bb(0)[j], par.bb(1)[j], par.bb(2)[j]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Corner<T> &o = cn[k];
            const int64_t mi = LAT16_PTS * js + lattice_index(N, ca1[k], ca2[k]);
            o.v = {mq.p[0][mi], mq.p[1][mi], mq.p[2][mi]};
            o.q = {mq.q[0][mi], mq.q[1][mi], mq.q[2][mi]};
            o.d = mq.d[mi];
            o.I = mq.I[mi];
            const int a0 = N - ca1[k] - ca2[k];
            o.ba = a0 * pba[0] + ca1[k] * pba[1] + ca2[k] * pba[2];
            o.bb = a0 * pbb[0] + ca1[k] * pbb[1] + ca2[k] * pbb[2];
        }
        pair = par.pair()[j];
        face = par.face()[j];
        lvl = par.lvl()[j] + 4;
    } else if (valid && two) {
        const int64_t js = c >> 4;
        const int64_t j = sel ? (int64_t)sel[js] : js;
        const int g = (int)(c & 15);
        const int pba[3] = {par.ba(0)[j], par.ba(1)[j], par.ba(2)[j]};
        const int pbb[3] = {par.bb(0)[j], par.bb(1)[j], par.bb(2)[j]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Corner<T> &o = cn[k];
            const int src = (int)((TWO_CORNER[k] >> (4 * g)) & 15u);
            int a1, a2;
            if (src >= LATTICE_PTS) {
                const int pk = src - LATTICE_PTS; // a parent corner
                o.v = {par.v(3 * pk)[j], par.v(3 * pk + 1)[j], par.v(3 * pk + 2)[j]};
                o.q = {par.q(3 * pk)[j], par.q(3 * pk + 1)[j], par.q(3 * pk + 2)[j]};
                o.d = par.d(pk)[j];
                o.I = par.I(pk)[j];
                a1 = pk == 1 ? 4 : 0;
                a2 = pk == 2 ? 4 : 0;
            } else {
                const int64_t mi = LATTICE_PTS * js + src;
                o.v = {mq.p[0][mi], mq.p[1][mi], mq.p[2][mi]};
                o.q = {mq.q[0][mi], mq.q[1][mi], mq.q[2][mi]};
                o.d = mq.d[mi];
                o.I = mq.I[mi];
                a1 = (LATTICE_A1 >> (2 * src)) & 3;
                a2 = (LATTICE_A2 >> (2 * src)) & 3;
            }
            // the point's dyadic numerators at the parent's level + 2 (the
            // lattice query used the same ones)
            const int a0 = 4 - a1 - a2;
            o.ba = a0 * pba[0] + a1 * pba[1] + a2 * pba[2];
            o.bb = a0 * pbb[0] + a1 * pbb[1] + a2 * pbb[2];
        }
        pair = par.pair()[j];
        face = par.face()[j];
        lvl = par.lvl()[j] + 2;
    } else if (valid) {
        const int64_t js = c >> 2;                       // the parent's position in the round
        const int64_t j = sel ? (int64_t)sel[js] : js;   // its record
        const int kid = (int)(c & 3);
        // The four children, counter-clockwise like the parent:
        // (v0, m01, m20), (m01, v1, m12), (m20, m12, v2), (m01, m12, m20).
        // Corner k of child kid is the parent's corner k when kid == k, else
        // the midpoint of parent edge (e, e+1) with e = MID(kid, k). Each
        // corner is assembled the same way for every child (no branch per
        // child), and the parent fields are read at compile-time corner
        // indices, so the view's pointers stay in scalar registers.
        constexpr unsigned MID = (0u << 0) | (0u << 2) | (2u << 4) |  // child 0
                                 (0u << 6) | (0u << 8) | (1u << 10) | // child 1
                                 (2u << 12) | (1u << 14) | (0u << 16) | // child 2
                                 (0u << 18) | (1u << 20) | (2u << 22);  // child 3
        const int pba[3] = {par.ba(0)[j], par.ba(1)[j], par.ba(2)[j]};
        const int pbb[3] = {par.bb(0)[j], par.bb(1)[j], par.bb(2)[j]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            Corner<T> &o = cn[k];
            if (kid == k) {
                o.v = {par.v(3 * k)[j], par.v(3 * k + 1)[j], par.v(3 * k + 2)[j]};
                o.q = {par.q(3 * k)[j], par.q(3 * k + 1)[j], par.q(3 * k + 2)[j]};
                o.d = par.d(k)[j];
                o.I = par.I(k)[j];
                o.ba = 2 * pba[k];
                o.bb = 2 * pbb[k];
            } else {
                const int e = (int)((MID >> (2 * (3 * kid + k))) & 3u);
                const int64_t mi = 3 * js + e;
                o.v = {mq.p[0][mi], mq.p[1][mi], mq.p[2][mi]};
                o.q = {mq.q[0][mi], mq.q[1][mi], mq.q[2][mi]};
                o.d = mq.d[mi];
                o.I = mq.I[mi];
                // parent corners e and e + 1, selected per lane
                o.ba = (e == 0 ? pba[0] + pba[1] : (e == 1 ? pba[1] + pba[2] : pba[2] + pba[0]));
                o.bb = (e == 0 ? pbb[0] + pbb[1] : (e == 1 ? pbb[1] + pbb[2] : pbb[2] + pbb[0]));
            }
        }
        pair = par.pair()[j];
        face = par.face()[j];
        lvl = par.lvl()[j] + 1;
    }
    int evals = 0;
    if (valid) {
        // dyadic coordinates are int32 numerators over 2^lvl: level 30 is the
        // deepest representable one
        if (lvl > 30) ctl->bad = 3;
        int unsound = 0;
        list = stage_a<T>(cn, pair, cc, &carry, &decider, &unsound);
        if (FUSE && list == TO_B)
            // stage B on the stored (rounded up) stage-A bound, as k_stage_b would
            list = stage_b<T>(cn, pair, cc, bv, (double)round_up_to_float(carry), decider, &carry, &decider, &evals,
                              &unsound, -1);
        if (unsound) ctl->bad = 4;
    }
    int64_t slot = append_slot(valid ? list : TO_DISCARD, ctl);
    if (valid)
        write_to(dst, list, slot, cn, round_up_to_float(carry), face, lvl_field(list, lvl, decider), pair);
    tally(ctl, list, decider, evals, 0, valid, true);
    }
}

// stage B over the records stage A left undecided (count in ctl->b_next;
// grid-stride); Sb (when the order has the fifth bound): the closest B
// triangle (sorted index) of each record's barycenter
// (FP32: registers capped for three waves per SIMD, a small spill; it hides
// more of the latency of the B frames the bounds read, measured 6-7% faster
// than two waves. FP64 would spill far more: uncapped.)
template <class T>
__global__ __launch_bounds__(BLK) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 3 : 1))) void k_stage_b(
    FrontierView<T> in, ClassifyCfg cc, BView<T> bv, Dest<T> dst, Ctl *ctl, const int *__restrict__ Sb) {
    const int64_t n = (int64_t)ctl->b_next;
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK) {
        const int64_t j = base + threadIdx.x;
        const bool valid = j < n;
        int list = TO_DISCARD, decider = 0, evals = 0, pair = 0, face = 0, lvl = 0;
        double carry = 0;
        Corner<T> cn[3];
        if (valid) {
            load_corners(in, j, cn);
            pair = in.pair()[j];
            face = in.face()[j];
            lvl = in.lvl()[j] & 0xff;
            int unsound = 0;
            list = stage_b<T>(cn, pair, cc, bv, (double)in.ub()[j], in.lvl()[j] >> 8, &carry, &decider, &evals,
                              &unsound, Sb ? Sb[j] : -1);
            if (unsound) ctl->bad = 4;
        }
        int64_t slot = append_slot(valid ? list : TO_DISCARD, ctl);
        if (valid)
            write_to(dst, list, slot, cn, round_up_to_float(carry), face, lvl_field(list, lvl, decider), pair);
        tally(ctl, list, decider, evals, 0, valid, false);
    }
}

// stage C: FP64 re-bound of the recheck band (count in ctl->c_next).
// A few records take one wave the latency of a long FP64 chain, the same
// as a few thousand: in device-planned rounds (defer = 1) the band is left
// to accumulate and runs only once C_FLUSH_MIN records wait or no active
// record is left (the rounds would end). The first block to arrive decides
// for all (before any block appends); the plan keeps deferred records.
constexpr int64_t C_FLUSH_MIN = 4096;

// device-planned rounds: a pending round that splits at most this many
// triangles is not followed by one enqueued ahead of its report
constexpr int64_t LOOKAHEAD_MIN = 64;

// device-planned breadth-first rounds of at most this many parents split each
// of them two levels deep (hd_options.split_levels)
constexpr int64_t TWO_LEVEL_MAX = 8192;

// FP32 runs take stage B inside the kernel that bounds the new triangles
// (k_round0 and the one-level k_children, FUSE)
constexpr bool FUSE_STAGE_B = true;

// stage C's records [0, n) in a grid-stride loop (every thread of the block)
template <class T>
__device__ void stage_c_records(const FrontierView<T> &in, const ClassifyCfg &cc, const Dest<T> &dst, Ctl *ctl,
                                int64_t n) {
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK) {
        const int64_t j = base + threadIdx.x;
        const bool valid = j < n;
        int list = TO_DISCARD, decider = 0, evals = 0, pair = 0, face = 0, lvl = 0;
        double ub = 0;
        Corner<T> cn[3];
        if (valid) {
            load_corners(in, j, cn);
            pair = in.pair()[j];
            face = in.face()[j];
            lvl = in.lvl()[j] & 0xff;
            decider = in.lvl()[j] >> 8;
            const PairConst &P = cc.pc[pair];
            int ba[3] = {cn[0].ba, cn[1].ba, cn[2].ba}, bb[3] = {cn[0].bb, cn[1].bb, cn[2].bb};
            int I[3] = {cn[0].I, cn[1].I, cn[2].I};
            double u64 = rebound64(cc.a, pair, face, lvl, ba, bb, I, cc.bv64, cc.iv, cc.c, P.m64, &evals);
            ub = hmin((double)in.ub()[j], u64);
            list = decide(ub, pair_L(cc.pc, cc.pv, pair), P.eps_abs, 0.0, false);
        }
        int64_t slot = append_slot(valid ? list : TO_DISCARD, ctl);
        if (valid) write_to(dst, list, slot, cn, round_up_to_float(ub), face, lvl, pair);
        tally(ctl, list, decider, evals, 1, valid, false);
    }
}

// With seq != 0 the kernel also ends a device-planned round: once every
// block with records has decided (and run), the last of them reports the
// round (report_to) and plans the next (plan_round), the work of
// k_report_plan without a launch of its own; with no record at all, block 0
// does it at once.
template <class T>
__global__ __launch_bounds__(BLK) void k_stage_c(FrontierView<T> in, ClassifyCfg cc, Dest<T> dst, Ctl *ctl,
                                                 int defer, Mailbox *ring, unsigned seq, PlanCaps caps) {
    const int64_t n = (int64_t)ctl->c_next;
    const int64_t need = (n + BLK - 1) / BLK;
    const unsigned nact = (unsigned)(need < (int64_t)gridDim.x ? need : (int64_t)gridDim.x);
    // blocks without records leave at once (the grid is sized for a larger
    // count; a decision per block is an atomic on one address)
    if (blockIdx.x >= nact) {
        if (seq && nact == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
            report_to(ctl, cc.pv, ring, seq);
            plan_round(ctl, caps);
        }
        return;
    }
    bool run = true;
    if (defer) {
        __shared__ int s_run;
        if (threadIdx.x == 0) {
            const int mine = n >= C_FLUSH_MIN || ctl->act_next == 0 ? 1 : 2;
            const int first = atomicCAS(&ctl->c_decision, 0, mine);
            s_run = (first == 0 ? mine : first) == 1;
        }
        __syncthreads();
        run = s_run;
    }
    if (run) stage_c_records(in, cc, dst, ctl, n);
    // (the plan resets the decision and the counters for the next round: it
    // waits until every block with records has read them)
    if (seq && last_block(&ctl->c_done, nact) && threadIdx.x == 0) {
        report_to(ctl, cc.pv, ring, seq);
        plan_round(ctl, caps);
    }
}

// ---------------------------------------------------------------------------
// learned proposal: features, predictions, logging, bound policy
// ---------------------------------------------------------------------------
struct LearnCfg {
    const PairConst *pc;
    const PairVar *pv;
    IdView iv;
};

template <class T> HD_D Tri<T> record_tri(const FrontierView<T> &f, int64_t j) {
    Corner<T> cn[3];
    load_corners(f, j, cn);
    return make_tri(cn);
}

// predicted maximum distance of a record: largest vertex distance plus the
// network's output times the longest edge
template <class T> HD_D float predicted_max(const Tri<T> &t, float y) {
    const T ell = hmax(hsqrt(norm2(t.v[1] - t.v[0])), hmax(hsqrt(norm2(t.v[2] - t.v[1])), hsqrt(norm2(t.v[0] - t.v[2]))));
    const T dmax = hmax(t.d[0], hmax(t.d[1], t.d[2]));
    return (float)dmax + (float)ell * y;
}

// Network scores of a block of records: each thread's 16 features go to an
// LDS tile, each wave runs the network on its 64 rows (four 16-row tiles on
// the matrix cores), and the thread reads back its prediction. Every thread
// of the block must call this.
struct ScoreLds {
    mlp::Weights W;
    alignas(16) float X[BLK * 16];
    alignas(16) unsigned short stage[NW][16 * 64];
    float y[BLK];
};
template <class T>
__device__ float score_block(ScoreLds &S, bool valid, const Tri<T> &t, double L, double dA, const BView<T> &bv,
                             const IdView &iv) {
    float f[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) f[k] = 0.f;
    if (valid) tri_features(t, L, dA, bv, iv, f);
#pragma unroll
    for (int k = 0; k < 16; ++k) S.X[threadIdx.x * 16 + k] = f[k];
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = __lane_id(), g = l >> 4, c = l & 15;
    for (int q = 0; q < 4; ++q) {
        mlp::Tile tl;
        mlp::tile_forward(S.X + wave * 64 * 16, nullptr, 16 * q, 64, S.W, S.stage[wave], tl);
        if (c == 0)
            for (int j = 0; j < 4; ++j) S.y[wave * 64 + 16 * q + 4 * g + j] = tl.y[j];
    }
    __syncthreads();
    return S.y[threadIdx.x];
}

// score records from..from+n-1 of a list (those the round appended)
template <class T>
__global__ __launch_bounds__(BLK) void k_score(FrontierView<T> fr, int64_t from, int64_t n, LearnCfg lc, BView<T> bv,
                                               const float *__restrict__ params) {
    __shared__ ScoreLds S;
    for (int i = threadIdx.x; i < mlp::NPARAM; i += BLK) mlp::set_param(S.W, i, params[i]);
    const int64_t j = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = j < from + n;
    Tri<T> t{};
    double L = 0, dA = 1;
    if (valid) {
        t = record_tri(fr, j);
        const int pair = fr.pair()[j];
        L = pair_L(lc.pc, lc.pv, pair);
        dA = lc.pc[pair].dA;
    }
    const float y = score_block(S, valid, t, L, dA, bv, lc.iv);
    if (valid) fr.score()[j] = predicted_max(t, y);
}

// selection keys in learned order: descending stored prediction, ties by the
// same order-independent tag as the plain keys (an unscored record, or a NaN
// prediction, falls back to its upper bound)
template <class T>
__global__ void k_sel_keys_learned(FrontierView<T> fr, int64_t n, unsigned long long *__restrict__ keys,
                                   int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float pm = fr.score()[i];
    if (!(pm == pm)) pm = fr.ub()[i];
    uint32_t tag = point_tag(fr.face()[i], fr.lvl()[i], fr.ba(0)[i] ^ (fr.ba(1)[i] << 7) ^ (fr.ba(2)[i] << 14),
                             fr.bb(0)[i] ^ (fr.bb(1)[i] << 7) ^ (fr.bb(2)[i] << 14));
    keys[i] = ((unsigned long long)(~f2ord(pm)) << 32) | tag;
    vals[i] = (int32_t)i;
}

// frontier log: for parents 0..n-1, their features and the label
// (max over the resolution-4 lattice of d(p, B) - max vertex distance) / l,
// into rows base + j of log (17 floats each; rows past cap are dropped, as
// are parents too deep for the lattice)
template <class T>
__global__ void k_log_parents(FrontierView<T> fr, int64_t n, QueryOut<T> lq, LearnCfg lc, BView<T> bv, float *log,
                              int64_t base, int64_t cap) {
    int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || base + j >= cap) return;
    float *o = log + (base + j) * 17;
    const Tri<T> t = record_tri(fr, j);
    const int pair = fr.pair()[j];
    if (fr.lvl()[j] + 2 > 30) {
        for (int k = 0; k < 17; ++k) o[k] = __builtin_nanf("");
        return;
    }
    float f[16];
    tri_features(t, pair_L(lc.pc, lc.pv, pair), lc.pc[pair].dA, bv, lc.iv, f);
    const T dmax = hmax(t.d[0], hmax(t.d[1], t.d[2]));
    T h = dmax;
    for (int k = 0; k < LATTICE_PTS; ++k) h = hmax(h, lq.d[j * LATTICE_PTS + k]);
    const T ell = hmax(hsqrt(norm2(t.v[1] - t.v[0])), hmax(hsqrt(norm2(t.v[2] - t.v[1])), hsqrt(norm2(t.v[0] - t.v[2]))));
    for (int k = 0; k < 16; ++k) o[k] = f[k];
    o[16] = ell > T(0) ? (float)((h - dmax) / ell) : 0.f;
}

// Stage B with the bound policy: a wave scores its 64 records with the
// network (matrix cores); a record whose predicted maximum lies above
// L + eps by more than 2% of its longest edge keeps stage A's bound and
// skips u3 and u4 (its true maximum, hence any bound, almost surely keeps it
// active); the others run stage B as usual.
constexpr float POLICY_MARGIN = 0.02f;

template <class T>
__global__ __launch_bounds__(BLK) void k_stage_b_learned(FrontierView<T> in, ClassifyCfg cc, BView<T> bv, Dest<T> dst,
                                                         Ctl *ctl, LearnCfg lc, const float *__restrict__ params,
                                                         const int *__restrict__ Sb) {
    const int64_t n = (int64_t)ctl->b_next;
    if ((int64_t)blockIdx.x * BLK >= n) return; // no work for this block
    __shared__ ScoreLds S;
    for (int i = threadIdx.x; i < mlp::NPARAM; i += BLK) mlp::set_param(S.W, i, params[i]);
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK) {
        const int64_t j = base + threadIdx.x;
        const bool valid = j < n;
        int list = TO_DISCARD, decider = 0, evals = 0, pair = 0, face = 0, lvl = 0;
        double carry = 0, L = 0, dA = 1;
        Corner<T> cn[3];
        Tri<T> t{};
        if (valid) {
            load_corners(in, j, cn);
            pair = in.pair()[j];
            face = in.face()[j];
            lvl = in.lvl()[j] & 0xff;
            L = pair_L(cc.pc, cc.pv, pair);
            dA = lc.pc[pair].dA;
            t = make_tri(cn);
        }
        const float y = score_block(S, valid, t, L, dA, bv, lc.iv);
        int skipped = 0;
        if (valid) {
            const T ell = hmax(hsqrt(norm2(t.v[1] - t.v[0])),
                               hmax(hsqrt(norm2(t.v[2] - t.v[1])), hsqrt(norm2(t.v[0] - t.v[2]))));
            const double pm = (double)predicted_max(t, y);
            const double eps = cc.pc[pair].eps_abs;
            if (pm > L + eps + (double)POLICY_MARGIN * (double)ell) {
                // stage A's running minimum is already a valid bound
                const double mu = tri_margin(t, margins_of<T>(cc.pc[pair]));
                carry = (double)in.ub()[j];
                decider = in.lvl()[j] >> 8;
                list = decide(carry, L, eps, mu, cc.recheck);
                skipped = 1;
            } else {
                int unsound = 0;
                list = stage_b<T>(cn, pair, cc, bv, (double)in.ub()[j], in.lvl()[j] >> 8, &carry, &decider,
                                  &evals, &unsound, Sb ? Sb[j] : -1);
                if (unsound) ctl->bad = 4;
            }
        }
        int64_t slot = append_slot(valid ? list : TO_DISCARD, ctl);
        if (valid)
            write_to(dst, list, slot, cn, round_up_to_float(carry), face, lvl_field(list, lvl, decider), pair);
        tally(ctl, list, decider, evals, 0, valid, false);
        block_add<1, BLK>({(unsigned long long)skipped}, {&ctl->stat[acc_copy()][ST_SKIPS]});
    }
}

// ---------------------------------------------------------------------------
// record movement and selection
// ---------------------------------------------------------------------------
template <class T>
HD_D void copy_record(const FrontierView<T> &src, int64_t i, const FrontierView<T> &dst, int64_t o) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        dst.v(k)[o] = src.v(k)[i];
        dst.q(k)[o] = src.q(k)[i];
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dst.d(k)[o] = src.d(k)[i];
        dst.I(k)[o] = src.I(k)[i];
        dst.ba(k)[o] = src.ba(k)[i];
        dst.bb(k)[o] = src.bb(k)[i];
    }
    dst.ub()[o] = src.ub()[i];
    dst.face()[o] = src.face()[i];
    dst.lvl()[o] = src.lvl()[i];
    dst.pair()[o] = src.pair()[i];
    dst.score()[o] = src.score()[i];
}

// dst[o] = src[perm[o]] (perm null: src[off + o])
template <class T>
__global__ void k_gather(FrontierView<T> src, const int32_t *__restrict__ perm, int64_t off, int64_t n,
                         FrontierView<T> dst) {
    int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < n) copy_record(src, perm ? perm[o] : off + o, dst, o);
}

// selection keys: descending upper bound, ties by an order-independent tag
template <class T>
__global__ void k_sel_keys(FrontierView<T> fr, int64_t n, unsigned long long *__restrict__ keys,
                           int32_t *__restrict__ vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t tag = point_tag(fr.face()[i], fr.lvl()[i], fr.ba(0)[i] ^ (fr.ba(1)[i] << 7) ^ (fr.ba(2)[i] << 14),
                             fr.bb(0)[i] ^ (fr.bb(1)[i] << 7) ^ (fr.bb(2)[i] << 14));
    keys[i] = ((unsigned long long)(~f2ord(fr.ub()[i])) << 32) | tag;
    vals[i] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// device sub-batch selection
// ---------------------------------------------------------------------------
// Rounds with sub-batches split about K of the active records: those with the
// largest keys (the upper bound: the paper's best-first order; or the
// network's predicted maximum: the learned order). A two-level radix select on
// the 32-bit ordered key finds the threshold without sorting: 4096 bins of the
// key's top 12 bits, then 4096 bins of the next 12 bits inside the boundary
// bin; every record at or above the threshold is selected (about K: the last
// bin is taken whole, and it is 2^-15 of the key's magnitude wide). The
// selected set depends only on the records, not on their order in the list.
// The passes also re-check each record against the current L, which may have
// risen since the record was bounded: below L it is dropped (the paper's stale
// queue entries), within eps of L it is parked.
constexpr int SEL_BINS = 4096;
constexpr unsigned SEL_GRID_MAX = 512;
// SEL_FROZEN: the plan splits nothing (no room, a failure, the budget): every
// record is carried as it is (the park list has no room reserved for it)
enum { SEL_NONE = 0, SEL_ALL = 1, SEL_THRESHOLD = 2, SEL_FROZEN = 3 };

struct SelCfg {
    unsigned *hist1, *hist2; // SEL_BINS counters each, zero between rounds
    int32_t *sel, *rest;     // record indices: the selected parents, the carried records
    int learned;             // the key: the network's prediction (1) or the upper bound (0)
    double budget;           // the paper's face budget (m * nA), less round 0
    int64_t subbatch;        // the sub-batch size
    int64_t two_max, four_max; // a round that splits every live record (SEL_ALL) of at most this many
                               // parents splits two (four) levels deep, as breadth-first rounds do
};

template <class T> HD_D uint32_t sel_key(const FrontierView<T> &f, int64_t j, int learned) {
    float k = f.ub()[j];
    if (learned) {
        const float sc = f.score()[j];
        if (sc == sc) k = sc; // unscored or NaN: the bound
    }
    return f2ord(k);
}

// what the selection does with record j: 0 keep it live, 1 drop it (its bound
// is below L), 2 park it (its bound is within eps of L)
template <class T> HD_D int sel_fate(const FrontierView<T> &f, int64_t j, const PairConst *pc, const PairVar *pv) {
    const int pair = f.pair()[j];
    const double ub = (double)f.ub()[j], L = pair_L(pc, pv, pair);
    if (ub < L) return 1;
    return ub - L <= park_limit(pc[pair].eps_abs) ? 2 : 0;
}

// Run by every thread of one block: the largest bin b of hist with
// sum(hist[b..]) >= want (-1 if the total is smaller); *above receives the sum
// over the bins above b, *at the count of b, *total the sum of all bins. The
// histogram is read with device-scope loads (other blocks filled it with
// atomics) and zeroed for the next round.
__device__ int sel_find_bin(unsigned *hist, unsigned long long want, unsigned long long *above,
                            unsigned long long *at, unsigned long long *total) {
    constexpr int PER = SEL_BINS / BLK;
    static_assert(SEL_BINS % BLK == 0, "bins per thread");
    __shared__ unsigned long long sfx[BLK];
    __shared__ int s_bin;
    __shared__ unsigned long long s_above, s_at;
    const int t = threadIdx.x;
    unsigned v[PER];
    unsigned long long sum = 0;
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        v[k] = __hip_atomic_load(&hist[t * PER + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sum += v[k];
    }
    sfx[t] = sum;
    if (t == 0) {
        s_bin = -1;
        s_above = 0;
        s_at = 0;
    }
    __syncthreads();
    // inclusive suffix sums over the threads' chunks
    for (int off = 1; off < BLK; off <<= 1) {
        const unsigned long long x = t + off < BLK ? sfx[t + off] : 0ull;
        __syncthreads();
        sfx[t] += x;
        __syncthreads();
    }
    unsigned long long run = t + 1 < BLK ? sfx[t + 1] : 0ull; // records in the chunks above
    if (run < want && sfx[t] >= want) {
        // the crossing lies in this thread's chunk: walk it from the top
        for (int k = PER - 1; k >= 0; --k) {
            if (run + v[k] >= want) {
                s_bin = t * PER + k;
                s_above = run;
                s_at = v[k];
                break;
            }
            run += v[k];
        }
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) hist[t * PER + k] = 0;
    __syncthreads();
    *above = s_above;
    *at = s_at;
    *total = sfx[0];
    return s_bin;
}

// block histogram of the live records' keys: level 1 bins the top 12 bits of
// every live record; level 2 the next 12 bits of those in bin b1
template <class T, int LEVEL>
__device__ void sel_histogram(const FrontierView<T> &act, int64_t n, int learned, int learn_off, unsigned b1,
                              const PairConst *pc, const PairVar *pv, unsigned *global_hist,
                              unsigned long long *prom_out) {
    __shared__ unsigned h[SEL_BINS];
    __shared__ unsigned prom;
    for (int i = threadIdx.x; i < SEL_BINS; i += BLK) h[i] = 0;
    if (threadIdx.x == 0) prom = 0;
    __syncthreads();
    for (int64_t j = (int64_t)blockIdx.x * BLK + threadIdx.x; j < n; j += (int64_t)gridDim.x * BLK) {
        if (sel_fate(act, j, pc, pv) != 0) continue;
        const uint32_t key = sel_key(act, j, learned);
        if (LEVEL == 1) {
            atomicAdd(&h[key >> 20], 1u);
            // learned order: a live record whose predicted maximum lies above
            // L + eps may still raise L
            if (learned && !learn_off) {
                const float sc = act.score()[j];
                const int pair = act.pair()[j];
                if (sc == sc && (double)sc > pair_L(pc, pv, pair) + pc[pair].eps_abs) atomicAdd(&prom, 1u);
            }
        } else if ((key >> 20) == b1) {
            atomicAdd(&h[(key >> 8) & (SEL_BINS - 1)], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < SEL_BINS; i += BLK)
        if (h[i]) atomicAdd(&global_hist[i], h[i]);
    if (LEVEL == 1 && threadIdx.x == 0 && prom) atomicAdd(prom_out, (unsigned long long)prom);
}

// first pass: histogram of the live records; the last block finds the
// boundary bin of the target (ctl->plan_K, set by plan_round)
template <class T>
__global__ __launch_bounds__(BLK) void k_sel_hist1(FrontierView<T> act, SelCfg sc, const PairConst *__restrict__ pc,
                                                   const PairVar *pv, Ctl *ctl) {
    const int64_t n = (int64_t)ctl->act_next;
    const unsigned long long want = ctl->plan_K;
    if (want == 0) { // frozen: nothing to count
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            ctl->sel_n = (unsigned long long)n;
            ctl->sel_live = (unsigned long long)n;
            ctl->sel_above1 = 0;
            ctl->sel_b1 = 0;
            ctl->sel_mode = SEL_FROZEN;
        }
        return;
    }
    const int64_t need = (n + BLK - 1) / BLK;
    const unsigned nact = (unsigned)(need < (int64_t)gridDim.x ? need : (int64_t)gridDim.x);
    if (blockIdx.x >= nact && !(nact == 0 && blockIdx.x == 0)) return;
    const int learn_off = ctl->learn_off;
    if (nact > 0) sel_histogram<T, 1>(act, n, sc.learned, learn_off, 0, pc, pv, sc.hist1, &ctl->sel_prom);
    if (nact == 0 || last_block(&ctl->h1_done, nact)) {
        // learned order: the top sub-batch by prediction while some record
        // may still raise L, else every live record (breadth-first), from
        // then on without scoring
        const bool prom = sc.learned && !learn_off &&
                          __hip_atomic_load(&ctl->sel_prom, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0;
        const unsigned long long target =
            prom ? (want < (unsigned long long)sc.subbatch ? want : (unsigned long long)sc.subbatch) : want;
        if (sc.learned && !prom && threadIdx.x == 0) ctl->learn_off = 1;
        unsigned long long above = 0, at = 0, total = 0;
        const int b = sel_find_bin(sc.hist1, target, &above, &at, &total);
        if (threadIdx.x == 0) {
            ctl->sel_n = (unsigned long long)n;
            ctl->sel_live = total;
            ctl->sel_above1 = above;
            ctl->sel_b1 = b < 0 ? 0u : (unsigned)b;
            // every live record, or a threshold the second pass refines inside bin b
            ctl->sel_mode = total <= target ? SEL_ALL : SEL_THRESHOLD;
            ctl->plan_K = target;
        }
    }
}

// second pass: the boundary bin's records by their next 12 bits; the last
// block fixes the threshold and finishes the round's plan
template <class T>
__global__ __launch_bounds__(BLK) void k_sel_hist2(FrontierView<T> act, SelCfg sc, const PairConst *__restrict__ pc,
                                                   const PairVar *pv, Ctl *ctl) {
    const int64_t n = (int64_t)ctl->sel_n;
    const unsigned long long want = ctl->plan_K;
    const bool refine = ctl->sel_mode == SEL_THRESHOLD;
    const int64_t need = refine ? (n + BLK - 1) / BLK : 0;
    const unsigned nact = (unsigned)(need < (int64_t)gridDim.x ? need : (int64_t)gridDim.x);
    if (blockIdx.x >= nact && !(nact == 0 && blockIdx.x == 0)) return;
    if (nact > 0) sel_histogram<T, 2>(act, n, sc.learned, 1, ctl->sel_b1, pc, pv, sc.hist2, nullptr);
    if (!(nact == 0 || last_block(&ctl->h2_done, nact))) return;
    unsigned long long above = 0, at = 0, total = 0;
    int b2 = -1;
    if (refine) b2 = sel_find_bin(sc.hist2, want - ctl->sel_above1, &above, &at, &total);
    if (threadIdx.x != 0) return;
    const unsigned long long live = ctl->sel_live;
    unsigned long long K = 0;
    int mode = SEL_NONE;
    unsigned thr = 0xffffffffu;
    if (ctl->sel_mode == SEL_ALL) {
        K = live;
        mode = SEL_ALL;
    } else if (refine && b2 >= 0) {
        const unsigned b1 = ctl->sel_b1;
        K = ctl->sel_above1 + above + at;
        thr = (b1 << 20) | ((unsigned)b2 << 8);
        mode = SEL_THRESHOLD;
        if (K > ctl->plan_kcap) {
            // the boundary bin does not fit: leave it out (what is above it
            // is fewer than the target, which fits)
            K = ctl->sel_above1 + above;
            thr = b2 + 1 < SEL_BINS ? ((b1 << 20) | ((unsigned)(b2 + 1) << 8)) : ((b1 + 1) << 20);
            if (K == 0) {
                ctl->stall = 1;
                mode = SEL_NONE;
            }
        }
    }
    if (K > 0 && ctl->processed + 4.0 * (double)K > sc.budget) {
        K = 0;
        mode = SEL_NONE;
        ctl->over_budget = 1;
    }
    if (mode == SEL_NONE) K = 0;
    // a round that splits every live record is a breadth-first round: when it
    // is small it goes two or four levels deep (plan_round). plan_kcap counts
    // parents with room for 4 children each; 16 need 5x that room in the
    // active list (15 more records per parent instead of 3) and 4x in the
    // others, 256 need 85x
    int dep = 0;
    const unsigned long long kc = ctl->plan_kcap;
    if (mode == SEL_ALL && K > 0 && K <= (unsigned long long)sc.two_max) {
        if (K <= (unsigned long long)sc.four_max && 85 * K <= kc && ctl->lvl_bound + 4 <= 30 &&
            ctl->processed + 256.0 * (double)K <= sc.budget)
            dep = 4;
        else if (5 * K <= kc && ctl->lvl_bound + 2 <= 30 && ctl->processed + 16.0 * (double)K <= sc.budget)
            dep = 2;
    }
    if (ctl->sel_mode == SEL_FROZEN) mode = SEL_FROZEN;
    ctl->sel_mode = mode;
    ctl->sel_thr = mode == SEL_THRESHOLD ? thr : (mode == SEL_ALL ? 0u : 0xffffffffu);
    ctl->plan_K = K;
    ctl->plan_Q = K * (dep == 4 ? (unsigned long long)LAT16_PTS : (dep == 2 ? 12ull : 3ull));
    ctl->plan_two = dep;
    ctl->plan_rest = live - K;
    ctl->act_next = live - K; // the carried records lead the round's output list
    ctl->processed += (dep == 4 ? 256.0 : (dep == 2 ? 16.0 : 4.0)) * (double)K;
    ctl->subdivided += K;
    if (K > 0) {
        ctl->rounds += 1;
        ctl->lvl_bound += dep ? dep : 1;
    }
    ctl->sel_next = 0;
    ctl->rest_next = 0;
}

// block-aggregated append to one of three counters (list 0..2; -1: none);
// every thread of the block must call it
__device__ int64_t append3(int list, unsigned long long *c0, unsigned long long *c1, unsigned long long *c2) {
    __shared__ int wc[3][NW];
    __shared__ unsigned long long base[3];
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const unsigned long long lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    unsigned long long m[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        m[k] = __ballot(list == k);
        if (lane == 0) wc[k][w] = __popcll(m[k]);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int k = threadIdx.x;
        int tot = 0;
        for (int j = 0; j < NW; ++j) {
            const int c = wc[k][j];
            wc[k][j] = tot;
            tot += c;
        }
        unsigned long long *ctr = k == 0 ? c0 : (k == 1 ? c1 : c2);
        base[k] = tot ? atomicAdd(ctr, (unsigned long long)tot) : 0;
    }
    __syncthreads();
    int64_t slot = -1;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (list == k) slot = (int64_t)(base[k] + wc[k][w] + __popcll(m[k] & lt));
    __syncthreads();
    return slot;
}

// third pass: drop the records below L, park those within eps of it, and list
// the selected parents and the carried records (record indices)
template <class T>
__global__ __launch_bounds__(BLK) void k_sel_compact(FrontierView<T> act, FrontierView<T> park, SelCfg sc,
                                                     const PairConst *__restrict__ pc, const PairVar *pv, Ctl *ctl) {
    const int64_t n = (int64_t)ctl->sel_n;
    const int mode = ctl->sel_mode;
    const unsigned thr = ctl->sel_thr;
    unsigned long long stale = 0;
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK) {
        const int64_t j = base + threadIdx.x;
        int list = -1; // 0 park, 1 selected, 2 carried
        if (j < n && mode == SEL_FROZEN) {
            list = 2;
        } else if (j < n) {
            const int fate = sel_fate(act, j, pc, pv);
            if (fate == 1) ++stale;
            else if (fate == 2) list = 0;
            else list = (mode == SEL_ALL || (mode == SEL_THRESHOLD && sel_key(act, j, sc.learned) >= thr)) ? 1 : 2;
        }
        const int64_t slot = append3(list, &ctl->park_next, &ctl->sel_next, &ctl->rest_next);
        if (list == 0) copy_record(act, j, park, slot);
        else if (list == 1) sc.sel[slot] = (int32_t)j;
        else if (list == 2) sc.rest[slot] = (int32_t)j;
    }
    block_add<1, BLK>({stale}, {&ctl->stat[acc_copy()][ST_STALE]});
}

// learned order in device-planned rounds: the network scores every active
// record that has no score yet (those the previous round appended)
template <class T>
__global__ __launch_bounds__(BLK) void k_score_new(FrontierView<T> fr, const Ctl *ctl, LearnCfg lc, BView<T> bv,
                                                   const float *__restrict__ params) {
    const int64_t n = (int64_t)ctl->act_next;
    if ((int64_t)blockIdx.x * BLK >= n || ctl->learn_off) return;
    __shared__ ScoreLds S;
    bool loaded = false;
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK) {
        const int64_t j = base + threadIdx.x;
        bool valid = false;
        if (j < n) {
            const float sc = fr.score()[j];
            valid = !(sc == sc);
        }
        if (!__syncthreads_or(valid)) continue;
        if (!loaded) {
            for (int i = threadIdx.x; i < mlp::NPARAM; i += BLK) mlp::set_param(S.W, i, params[i]);
            loaded = true;
            __syncthreads();
        }
        Tri<T> t{};
        double L = 0, dA = 1;
        if (valid) {
            t = record_tri(fr, j);
            const int pair = fr.pair()[j];
            L = pair_L(lc.pc, lc.pv, pair);
            dA = lc.pc[pair].dA;
        }
        const float y = score_block(S, valid, t, L, dA, bv, lc.iv);
        if (valid) fr.score()[j] = predicted_max(t, y);
    }
}

// ---------------------------------------------------------------------------
// final FP64 step
// ---------------------------------------------------------------------------
// whether the rounds left the run converged: nothing active or planned, no
// recheck record waiting, no error
__device__ bool run_converged(const Ctl *c) {
    return c->plan_K == 0 && c->act_next == 0 && c->c_next == 0 && c->bad == 0 && c->bad_input == 0 &&
           c->over_budget == 0;
}

// the records of k_final_U (every thread of the block; i >= n: no record)
template <class T>
__device__ void final_U_records(const FrontierView<T> &fr, int64_t i, int64_t n, const AView &a,
                                const BView<double> &bv64, const IdView &iv, const CascadeCtx &c,
                                const PairConst *__restrict__ pc, PairVar *pv, Ctl *ctl) {
    const bool valid = i < n;
    unsigned long long ev = 0;
    int pair = 0;
    double u[2] = {0, 0};
    if (valid) {
        pair = fr.pair()[i];
        int ba[3] = {fr.ba(0)[i], fr.ba(1)[i], fr.ba(2)[i]};
        int bb[3] = {fr.bb(0)[i], fr.bb(1)[i], fr.bb(2)[i]};
        int I[3] = {fr.I(0)[i], fr.I(1)[i], fr.I(2)[i]};
        int evals = 0;
        double u64 = rebound64(a, pair, fr.face()[i], fr.lvl()[i], ba, bb, I, bv64, iv, c, pc[pair].m64, &evals);
        double u32 = (double)fr.ub()[i];
        u[0] = hmin(u64, u32);
        u[1] = u32;
        ev = evals;
    }
    block_pair_minmax<2, 3u, BLK>(pair, valid, u, [&](int p, int k) { return k == 0 ? &pv[p].Uord : &pv[p].Urounds; });
    block_add<1, BLK>({ev}, {&ctl->stat[acc_copy()][ST_EVALS]});
}

// U over the live records of a list (count from cnt). With gated set the
// launch was enqueued ahead of the report of a round that is probably the
// last, and does nothing unless the run has converged.
template <class T>
__global__ __launch_bounds__(BLK) void k_final_U(FrontierView<T> fr, DevCount cnt, int gated, AView a,
                                                 BView<double> bv64, IdView iv, CascadeCtx c,
                                                 const PairConst *__restrict__ pc, PairVar *pv, Ctl *ctl) {
    const int64_t n = gated && !run_converged(ctl) ? 0 : cnt.get();
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK)
        final_U_records(fr, base + threadIdx.x, n, a, bv64, iv, c, pc, pv, ctl);
}

// ---------------------------------------------------------------------------
// test entry: all five bounds of given triangles
// ---------------------------------------------------------------------------
template <class T>
__global__ void k_eval_bounds(const double *v, const double *d, const int32_t *Iorig, const double *q, int64_t n,
                              const int32_t *inv_perm, int64_t nB, BView<T> bv, IdView iv,
                              const PairConst *pc, double *out, int32_t *u3case) {
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
    const double *c = pc[0].ctr;
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

// test entry: the fifth bound of given triangles (uncentred FP64 input),
// their barycenters' closest triangles from a point query (Sb, sorted)
__global__ void k_barycenters(const double *v, int64_t n, double *P) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) P[3 * i + k] = (v[9 * i + k] + v[9 * i + 3 + k] + v[9 * i + 6 + k]) / 3.0;
}

template <class T>
__global__ void k_eval_u5(const double *v, const double *d, const int32_t *Iorig, int64_t n, const int32_t *inv_perm,
                          int64_t nB, const int *Sb, BView<T> bv, const int4 *ids, const PairConst *pc, double *out,
                          int32_t *Sb_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) {
        const int32_t f = Iorig[3 * i + k];
        if (f < 0 || f >= nB) {
            out[i] = __builtin_nan("");
            Sb_out[i] = -1;
            return;
        }
    }
    Tri<T> t;
    const double *c = pc[0].ctr;
    for (int k = 0; k < 3; ++k) {
        t.v[k] = {T(v[9 * i + 3 * k] - c[0]), T(v[9 * i + 3 * k + 1] - c[1]), T(v[9 * i + 3 * k + 2] - c[2])};
        t.q[k] = t.v[k];
        t.d[k] = T(d[3 * i + k]);
        t.I[k] = inv_perm[Iorig[3 * i + k]];
    }
    out[i] = (double)bound_u5(t, bv, Sb[i], nullptr);
    Sb_out[i] = ids[Sb[i]].w;
}

// test entry: the learned proposal's features of given triangles
template <class T>
__global__ void k_tri_features(const double *v, const double *d, const int32_t *Iorig, const double *q, int64_t n,
                               const int32_t *inv_perm, int64_t nB, BView<T> bv, IdView iv, const PairConst *pc,
                               double L, double dA, float *X) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) {
        int32_t f = Iorig[3 * i + k];
        if (f < 0 || f >= nB) {
            for (int j = 0; j < 16; ++j) X[16 * i + j] = __builtin_nanf("");
            return;
        }
    }
    Tri<T> t;
    const double *c = pc[0].ctr;
    for (int k = 0; k < 3; ++k) {
        t.v[k] = {T(v[9 * i + 3 * k] - c[0]), T(v[9 * i + 3 * k + 1] - c[1]), T(v[9 * i + 3 * k + 2] - c[2])};
        t.q[k] = {T(q[9 * i + 3 * k] - c[0]), T(q[9 * i + 3 * k + 1] - c[1]), T(q[9 * i + 3 * k + 2] - c[2])};
        t.d[k] = T(d[3 * i + k]);
        t.I[k] = inv_perm[Iorig[3 * i + k]];
    }
    float f[16];
    tri_features(t, L, dA, bv, iv, f);
    for (int j = 0; j < 16; ++j) X[16 * i + j] = f[j];
}

__global__ void k_inv_perm(const int4 *ids, int64_t n, int32_t *inv) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[ids[i].w] = (int32_t)i;
}

template <class T>
__global__ void k_export_points(const QueryOut<T> r, int64_t n, const int4 *ids, const PairConst *pc, double *d,
                                int32_t *I, double *Q, const Ctl *ctl, int32_t *err) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // the query kernel has finished (stream order): its failure flag is final
    if (err && i == 0) *err = ctl->bad == 2 ? (int32_t)HD_E_INTERNAL : (int32_t)HD_OK;
    if (i >= n) return;
    const double *c = pc[0].ctr;
    d[i] = (double)r.d[i];
    I[i] = ids[r.I[i]].w;
    if (Q) {
        Q[3 * i] = (double)r.q[0][i] + c[0];
        Q[3 * i + 1] = (double)r.q[1][i] + c[1];
        Q[3 * i + 2] = (double)r.q[2][i] + c[2];
    }
}

// round log: every pair's largest live bound after a round
__global__ void k_round_U_reset(PairVar *pv, int npairs) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) pv[p].Uround = d2ord(0.0);
}

template <class T>
__global__ __launch_bounds__(BLK) void k_round_U(FrontierView<T> act, FrontierView<T> park, const Ctl *ctl,
                                                 PairVar *pv) {
    const int64_t na = (int64_t)ctl->act_next, n = na + (int64_t)ctl->park_next;
    for (int64_t base = (int64_t)blockIdx.x * BLK; base < n; base += (int64_t)gridDim.x * BLK) {
        const int64_t i = base + threadIdx.x;
        const bool valid = i < n;
        int pair = 0;
        double u[1] = {0.0};
        if (valid) {
            const bool a = i < na;
            const int64_t j = a ? i : i - na;
            u[0] = (double)(a ? act.ub()[j] : park.ub()[j]);
            pair = a ? act.pair()[j] : park.pair()[j];
        }
        block_pair_minmax<1, 1u, BLK>(pair, valid, u, [&](int p, int) { return &pv[p].Uround; });
    }
}

// ---------------------------------------------------------------------------
// host side: buffers
// ---------------------------------------------------------------------------
template <class T> struct FrontierBuf {
    DBuf mem;
    int64_t cap = 0;
    FrontierView<T> v{};
    // view over p for c records (c a multiple of 64)
    static FrontierView<T> carve(char *p, int64_t c) { return FrontierView<T>{p, c}; }
    // grow to hold c records; the first `live` records are preserved
    void ensure(int64_t c, int64_t live, hipStream_t s) {
        if (c <= cap) return;
        int64_t nc = std::max<int64_t>(c, cap + cap / 2);
        nc = (nc + 63) & ~int64_t(63);
        DBuf nm;
        nm.reserve((size_t)nc * FrontierView<T>::bytes_per_record());
        FrontierView<T> nv = carve(nm.as<char>(), nc);
        if (live > 0)
            k_gather<T><<<grid_for(live, BLK), BLK, 0, s>>>(v, nullptr, 0, live, nv);
        HD_LAUNCH_CHECK();
        HD_HIP(hipStreamSynchronize(s));
        mem.swap(nm);
        cap = nc;
        v = nv;
    }
};

template <class T> void release_fb(FrontierBuf<T> &a) {
    a.mem.release();
    a.cap = 0;
    a.v = FrontierView<T>{};
}

template <class T> void swap_fb(FrontierBuf<T> &a, FrontierBuf<T> &b) {
    a.mem.swap(b.mem);
    std::swap(a.cap, b.cap);
    std::swap(a.v, b.v);
}

// query results for nc queries, one array per field (256-byte aligned)
// carved from p; qout_bytes<T>(nc) bytes
template <class T> constexpr size_t qout_bytes(int64_t nc) {
    return (size_t)nc * (sizeof(T) * 7 + 4 + 8) + 16 * 256;
}
template <class T> QueryOut<T> carve_qout(char *p, int64_t nc) {
    QueryOut<T> o{};
    auto take = [&](size_t sz) {
        char *r = p;
        p += ((size_t)nc * sz + 255) & ~size_t(255);
        return r;
    };
    o.d = (T *)take(sizeof(T));
    o.I = (int *)take(4);
    for (int k = 0; k < 3; ++k) o.q[k] = (T *)take(sizeof(T));
    for (int k = 0; k < 3; ++k) o.p[k] = (T *)take(sizeof(T));
    o.key = (unsigned long long *)take(8);
    return o;
}

template <class T> struct QBuf {
    DBuf mem;
    int64_t cap = 0;
    QueryOut<T> o{};
    // grow to at least n queries (contents are not preserved); on a failed
    // allocation the old buffer stays as it was
    void ensure(int64_t n) {
        if (n <= cap) return;
        int64_t nc = std::max<int64_t>(n, cap + cap / 2);
        DBuf nm;
        nm.reserve(qout_bytes<T>(nc));
        mem.swap(nm);
        o = carve_qout<T>(mem.as<char>(), nc);
        cap = nc;
    }
    void release() {
        mem.release();
        cap = 0;
        o = QueryOut<T>{};
    }
};

// Buffers of the engine, kept between calls on one device (grow-only).
template <class T> struct TypedWs {
    FrontierBuf<T> act, act2, park;
    FrontierBuf<T> pend_b, pend_c; // records between cascade stages (one round's worth)
    QBuf<T> vq, mq, lq, bq; // vertex, midpoint, lattice and barycenter query results
    void release() {
        for (FrontierBuf<T> *f : {&act, &act2, &park, &pend_b, &pend_c}) release_fb(*f);
        for (QBuf<T> *q : {&vq, &mq, &lq, &bq}) q->release();
    }
};
struct Workspace {
    std::mutex mu;
    PinnedBuf host; // mailbox, staged uploads, exported results
    unsigned mb_seq = 0;
    std::vector<hipEvent_t> evpool; // profiling events (kept until the process ends)
    int qvar[2] = {0, 0};           // query launch shape per arithmetic (FP32, FP64)
    bool tuned[2] = {false, false};
    hipEvent_t tune_ev[2] = {nullptr, nullptr};
    DBuf ctl, pc, pv, pbox, params, Vcat, Fcat, fpair, ref, vids, ovf, deep, gstack, scan_tmp, sort_tmp, sortbuf, small;
    DBuf selidx, selhist; // device sub-batch selection: index lists, two histograms
    // what the device copy of the upload holds (the copy is skipped when a
    // call uploads the same bytes to the same buffer)
    std::vector<char> uploaded;
    void *uploaded_to = nullptr;
    TypedWs<float> w32;
    TypedWs<double> w64;
    template <class T> TypedWs<T> &typed();
    // The buffers only grow: after a call that ran out of memory or of
    // capacity (frontier lists sized near the device's memory), they are
    // given back, so that the next call starts from what it needs.
    void trim() {
        w32.release();
        w64.release();
        for (DBuf *b : {&Vcat, &Fcat, &fpair, &ref, &vids, &ovf, &sortbuf, &selidx, &scan_tmp, &sort_tmp})
            b->release();
    }
};
template <> TypedWs<float> &Workspace::typed<float>() { return w32; }
template <> TypedWs<double> &Workspace::typed<double>() { return w64; }

// one workspace per device, created on first use and kept until the process
// ends (never destroyed: the HIP runtime may be gone by static destruction)
std::mutex g_ws_mu;
Workspace *g_ws[64] = {};
Workspace *workspace_for(int dev) {
    std::lock_guard<std::mutex> lk(g_ws_mu);
    Workspace *&w = g_ws[dev & 63];
    if (!w) w = new Workspace();
    return w;
}

// ---- the autotuner's cache file ----------------------------------------------
// One JSON object whose keys name (device, arithmetic, kernel-source hash)
// and whose values hold the chosen launch shape:
//   {"gfx950/256CU/fp32/<hash>": {"variant": 0, "block": 128, "stack": 16}, ...}
// A file that is missing or cannot be parsed counts as empty; it is rewritten
// whole (through a temporary file and a rename) when a choice is added.
#ifndef HD_SOURCE_HASH
#define HD_SOURCE_HASH "unhashed"
#endif

std::string tuner_key(int arith64) {
    int dev = 0;
    HD_HIP(hipGetDevice(&dev));
    hipDeviceProp_t pr;
    HD_HIP(hipGetDeviceProperties(&pr, dev));
    std::string arch(pr.gcnArchName);
    for (char &c : arch)
        if (c == '"' || c == '\\') c = '_';
    return arch + "/" + std::to_string(pr.multiProcessorCount) + "CU/" + (arith64 ? "fp64" : "fp32") + "/" +
           HD_SOURCE_HASH;
}

std::vector<std::pair<std::string, int>> tuner_read(const char *path) {
    std::vector<std::pair<std::string, int>> out;
    FILE *f = std::fopen(path, "rb");
    if (!f) return out;
    std::string txt;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, n);
    std::fclose(f);
    size_t i = txt.find('{');
    while (i != std::string::npos) {
        const size_t k0 = txt.find('"', i + 1);
        if (k0 == std::string::npos) break;
        const size_t k1 = txt.find('"', k0 + 1);
        if (k1 == std::string::npos) break;
        const size_t body = txt.find('{', k1);
        const size_t end = body == std::string::npos ? std::string::npos : txt.find('}', body);
        if (end == std::string::npos) break;
        const size_t v = txt.find("\"variant\"", body);
        if (v != std::string::npos && v < end) {
            const size_t c = txt.find(':', v);
            if (c != std::string::npos && c < end) {
                char *e = nullptr;
                const long val = std::strtol(txt.c_str() + c + 1, &e, 10);
                if (e != txt.c_str() + c + 1) out.emplace_back(txt.substr(k0 + 1, k1 - k0 - 1), (int)val);
            }
        }
        i = end;
    }
    return out;
}

void tuner_write(const char *path, const std::vector<std::pair<std::string, int>> &entries) {
    const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
    FILE *f = std::fopen(tmp.c_str(), "wb");
    if (!f) return; // the cache is an optimisation: an unwritable path only loses it
    std::fputs("{\n", f);
    for (size_t i = 0; i < entries.size(); ++i) {
        const int v = entries[i].second >= 0 && entries[i].second < NQVAR ? entries[i].second : 0;
        std::fprintf(f, "  \"%s\": {\"variant\": %d, \"block\": %d, \"stack\": %d}%s\n", entries[i].first.c_str(), v,
                     QVARIANTS[v].qb, QVARIANTS[v].sd, i + 1 < entries.size() ? "," : "");
    }
    std::fputs("}\n", f);
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0) std::remove(tmp.c_str());
}

// the status of a call whose device state has bad != 0 (see Ctl::bad)
hd_status status_of_bad(int bad) {
    switch (bad) {
    case 3: return HD_E_CAPACITY; // depth exhausted: tolerance below what the arithmetic resolves
    case 5: return HD_E_INVALID;  // plain FP32 with a tolerance below its margin
    default: return HD_E_INTERNAL;
    }
}

int parse_order(int32_t order, int out[5]) {
    if (order <= 0) order = 1234;
    int digits[10], n = 0;
    while (order > 0 && n < 10) {
        digits[n++] = order % 10;
        order /= 10;
    }
    if (order > 0 || n > 5) return -1;
    int used = 0;
    for (int i = 0; i < n; ++i) {
        int k = digits[n - 1 - i];
        if (k < 1 || k > 5 || (used >> k) & 1) return -1;
        used |= 1 << k;
        out[i] = k;
    }
    return n;
}

// Kernel timing with HIP events on the engine's stream (begin/end pairs).
// Events come from a pool kept with the workspace, so that a profiled call
// does not create and destroy events.
struct Profiler {
    hipStream_t s;
    bool on = false;
    bool cascade = true; // also time the cascade kernels
    std::vector<hipEvent_t> *pool = nullptr;
    size_t used = 0;
    std::vector<hipEvent_t> q, c;
    void mark(std::vector<hipEvent_t> &v) {
        if (!on || (&v == &c && !cascade)) return;
        if (used == pool->size()) {
            hipEvent_t e;
            HD_HIP(hipEventCreate(&e));
            pool->push_back(e);
        }
        hipEvent_t e = (*pool)[used++];
        HD_HIP(hipEventRecord(e, s));
        v.push_back(e);
    }
    static double sum(std::vector<hipEvent_t> &v) {
        double ms = 0;
        for (size_t i = 0; i + 1 < v.size(); i += 2) {
            float t = 0;
            if (hipEventElapsedTime(&t, v[i], v[i + 1]) == hipSuccess) ms += t;
        }
        return ms;
    }
};

struct Input {
    int npairs;
    const double *const *VA;
    const int64_t *mA;
    const int32_t *const *FA;
    const int64_t *nA;
    const double *eps; // host: one value, or npairs values
    int eps_per_pair;
    int linked; // pairs 2k and 2k + 1 share their lower bound (the two directions of H)
};

// ---------------------------------------------------------------------------
// the engine
// ---------------------------------------------------------------------------
template <class T>
hd_status run(const Input &in, const Bvh *B, const hd_options &opt, hipStream_t s, Workspace &ws, double *LU,
              hd_stats *stats) {
    auto t0 = std::chrono::steady_clock::now();
    const int np = in.npairs;
    if (np != B->npairs) throw Error{HD_E_INVALID, "pair count differs from the BVH's"};
    if (in.linked && (np % 2) != 0) throw Error{HD_E_INVALID, "linked pairs come in twos"};
    hd_stats S;
    std::memset(&S, 0, sizeof(S));
    CascadeCtx cctx;
    cctx.norder = parse_order(opt.order, cctx.order);
    if (cctx.norder <= 0) throw Error{HD_E_INVALID, "bad cascade order"};
    if (opt.learned < 0 || opt.learned > 2) throw Error{HD_E_INVALID, "learned must be 0, 1 or 2"};
    if (opt.query_shape < 0 || opt.query_shape > NQVAR) throw Error{HD_E_INVALID, "query_shape out of range"};
    if (opt.query_lanes != 0 && opt.query_lanes != 1 && opt.query_lanes != 4)
        throw Error{HD_E_INVALID, "query_lanes must be 0, 1 or 4"};
    if (opt.learned > 0 && !opt.mlp_params) throw Error{HD_E_INVALID, "learned mode needs the network's parameters"};
    if (opt.log_frontier && (!opt.log_out || opt.log_cap <= 0)) throw Error{HD_E_INVALID, "frontier log needs a buffer"};
    for (int p = 0; p < (in.eps_per_pair ? np : 1); ++p)
        if (!(in.eps[p] > 0) || !std::isfinite(in.eps[p])) throw Error{HD_E_INVALID, "eps must be positive"};
    if (opt.eps_relative != 0 && opt.eps_relative != 1) throw Error{HD_E_INVALID, "eps_relative must be 0 or 1"};
    if (!std::isfinite(opt.test_bound_shift)) throw Error{HD_E_INVALID, "test_bound_shift must be finite"};
    if (opt.split_levels < 0) throw Error{HD_E_INVALID, "split_levels must not be negative"};
    if (opt.round_log_cap < 0 || (opt.round_log_cap > 0 && !opt.round_log))
        throw Error{HD_E_INVALID, "round log needs a host array"};
    const bool logging = opt.round_log != nullptr && opt.round_log_cap > 0;
    // plain FP32 rounds: a tolerance below the FP32 margin at L is an input error
    const int check_fp32 = sizeof(T) == 4 && opt.precision == HD_PREC_FP32 ? 1 : 0;
    std::vector<int64_t> foff(np + 1, 0), voff(np + 1, 0);
    for (int p = 0; p < np; ++p) {
        if (in.nA[p] <= 0 || in.mA[p] <= 0 || !in.VA[p] || !in.FA[p]) throw Error{HD_E_INVALID, "empty soup A"};
        foff[p + 1] = foff[p] + in.nA[p];
        voff[p + 1] = voff[p] + in.mA[p];
    }
    const int64_t nA = foff[np], mA = voff[np];
    if (nA >= (int64_t(1) << 30) || mA >= (int64_t(1) << 31)) throw Error{HD_E_INVALID, "soup A too large"};

    TypedWs<T> &tw = ws.typed<T>();
    Profiler prof;
    prof.s = s;
    prof.on = opt.profile != 0;
    prof.cascade = opt.profile == 1;
    prof.pool = &ws.evpool;

    // ---- small tables -----------------------------------------------------
    // Pinned host block: [0, 256) the report ring, [256, 260) the export
    // sequence word, then the packed upload (pair sources, face and vertex
    // offsets, eps) and the result area (control block, pair tables). The upload goes to the
    // device in one asynchronous copy; results come back through one export.
    ws.ctl.reserve(sizeof(Ctl));
    Ctl *ctl = ws.ctl.as<Ctl>();
    ws.pc.reserve(np * sizeof(PairConst));
    ws.pv.reserve(np * sizeof(PairVar));
    PairConst *pc = ws.pc.as<PairConst>();
    PairVar *pv = ws.pv.as<PairVar>();
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    const int neps = in.eps_per_pair ? np : 1;
    const size_t o_src = 0, o_foff = o_src + al(np * sizeof(PairSrcA)), o_voff = o_foff + al((np + 1) * 8),
                 o_eps = o_voff + al((np + 1) * 8), up_bytes = o_eps + al(neps * 8);
    const size_t o_up = HOST_UPLOAD, o_res = o_up + up_bytes;
    const size_t o_rctl = 0, o_rpv = al(sizeof(Ctl)), o_rpc = o_rpv + al(np * sizeof(PairVar)),
                 res_bytes = o_rpc + al(np * sizeof(PairConst));
    ws.host.reserve(o_res + res_bytes);
    Mailbox *mb = ws.host.as<Mailbox>(), *mb_dev = ws.host.dev_as<Mailbox>();
    // Enqueue a report and wait for it by polling the pinned mailbox: far
    // lower latency than a stream synchronisation plus a staged copy.
    auto report_async = [&]() -> unsigned {
        const unsigned seq = ++ws.mb_seq;
        k_report<<<1, 64, 0, s>>>(ctl, pv, mb_dev, seq);
        HD_LAUNCH_CHECK();
        return seq;
    };
    auto wait_report = [&](unsigned seq) -> Mailbox {
        const Mailbox *slot = mb + seq % MB_SLOTS;
        wait_host_seq(&slot->seq, seq, s);
        Mailbox m = *slot;
        if (m.bad_input) {
            // the ingest made the input safe to run on (indices and values
            // replaced), and the rounds already enqueued finish first
            HD_HIP(hipStreamSynchronize(s));
            throw Error{HD_E_INVALID, "soup A has an out-of-range index or a non-finite coordinate"};
        }
        return m;
    };
    auto report = [&]() -> Mailbox { return wait_report(report_async()); };
    {
        char *up = ws.host.as<char>(o_up);
        PairSrcA *hs = (PairSrcA *)(up + o_src);
        for (int p = 0; p < np; ++p) hs[p] = PairSrcA{in.VA[p], in.FA[p], in.mA[p]};
        std::memcpy(up + o_foff, foff.data(), (np + 1) * 8);
        std::memcpy(up + o_voff, voff.data(), (np + 1) * 8);
        std::memcpy(up + o_eps, in.eps, neps * 8);
    }
    if (up_bytes > ws.params.bytes) ws.uploaded_to = nullptr; // a new allocation may reuse the address
    ws.params.reserve(up_bytes);
    {
        const char *up = ws.host.as<char>(o_up);
        if (ws.uploaded_to != ws.params.p || ws.uploaded.size() != up_bytes ||
            std::memcmp(ws.uploaded.data(), up, up_bytes) != 0) {
            HD_HIP(hipMemcpyAsync(ws.params.p, up, up_bytes, hipMemcpyHostToDevice, s));
            ws.uploaded.assign(up, up + up_bytes);
            ws.uploaded_to = ws.params.p;
        }
    }
    const PairSrcA *dsrc = (const PairSrcA *)(ws.params.as<char>() + o_src);
    int64_t *dfoff = (int64_t *)(ws.params.as<char>() + o_foff);
    int64_t *dvoff = (int64_t *)(ws.params.as<char>() + o_voff);
    double *deps = (double *)(ws.params.as<char>() + o_eps);

    // ---- ingest A ---------------------------------------------------------
    ws.Vcat.reserve(mA * 3 * sizeof(double));
    ws.Fcat.reserve(nA * 3 * sizeof(int32_t));
    ws.fpair.reserve(nA * sizeof(int32_t));
    ws.ref.reserve(2 * mA * sizeof(int32_t) + 512);
    int32_t *ref = ws.ref.as<int32_t>();
    int32_t *refpos = ref + ((mA + 63) / 64) * 64;
    ws.small.reserve(4096);
    int32_t *d_total = ws.small.as<int32_t>();
    const int pstride = pbox_stride(np);
    ws.pbox.reserve((size_t)ACC_COPIES * pstride * sizeof(PairBox));
    PairBox *pbox = ws.pbox.as<PairBox>();
    k_bound_init<<<grid_for(std::max<int64_t>(mA, (int64_t)np * ACC_COPIES), BLK), BLK, 0, s>>>(
        ctl, pc, pv, pbox, pstride, B->pairs.as<BvhPair>(), np, ref, mA, logging ? 1 : 0, in.linked);
    const unsigned ingest_grid = np == 1 ? std::min(grid_for(nA, BLK), INGEST_ONE_PAIR_GRID) : grid_for(nA, BLK);
    k_ingest<<<ingest_grid, BLK, 0, s>>>(dsrc, dfoff, dvoff, np, nA, ws.Fcat.as<int32_t>(), ws.Vcat.as<double>(),
                                         ws.fpair.as<int32_t>(), ref, pc, pbox, pstride, ctl);
    scan_exclusive_i32(ref, refpos, mA, d_total, ws.scan_tmp, s);
    HD_LAUNCH_CHECK();
    // The count of referenced vertices stays on the device (round 0's
    // launches read it; their grids are sized for all mA vertices), and an
    // invalid input is reported with the first round's report: no wait here.
    ws.vids.reserve(mA * sizeof(int32_t));
    k_ingest_post<<<grid_for(std::max<int64_t>(mA, np), BLK), BLK, 0, s>>>(
        ref, refpos, mA, d_total, ws.vids.as<int32_t>(), pc, pbox, pstride, B->pairs.as<BvhPair>(), np, deps,
        in.eps_per_pair, opt.eps_relative ? 1 : 0, ctl);
    const DevCount nref_dev{&ctl->nref, 1, 0};

    const BView<T> bv = [&] {
        if constexpr (sizeof(T) == 4) return BView<float>{B->frames32.as<float4>()};
        else return BView<double>{B->frames64.as<double2>()};
    }();
    const BView<double> bv64{B->frames64.as<double2>()};
    const IdView iv{B->ids.as<int4>()};
    const AView av{ws.Vcat.as<double>(), ws.Fcat.as<int32_t>(), pc};
    // a single-pair BVH with an internal root has its top levels tabled
    const WideNode *top = np == 1 && B->npairs == 1 && !B->hpairs.empty() && B->hpairs[0].root >= 0
                              ? B->top.as<WideNode>()
                              : nullptr;
    const QueryCfg qcfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 1, top};
    ws.gstack.reserve((size_t)np * DEEP_STACK * sizeof(int2));
    ws.deep.reserve((size_t)DEEP_SLOTS * DEEP_STACK * sizeof(int2));
    const bool small_stack = opt.stack_depth > 0 && opt.stack_depth < QSTACK;
    int &qvar = ws.qvar[sizeof(T) == 4 ? 0 : 1];
    if (qvar < 0 || qvar >= NQVAR) qvar = 0;
    int qsel = 0; // the launch shape this call uses (set after the autotuner)
    // launches of at most qmax queries run a quad of lanes per query
    const int64_t qmax =
        opt.query_lanes == 1 ? -1 : (opt.query_lanes == 4 ? INT64_MAX : QUAD_MAX_DEFAULT);

    // queries: n_max bounds the count (host count, or the device-planned one),
    // the grid covers it up to a persistent cap and loops beyond
    auto run_queries = [&](const QueryIn<T> &qi, DevCount cnt, int64_t n_max, const QueryOut<T> &out) {
        if (n_max <= 0) return;
        ws.ovf.reserve((size_t)n_max * sizeof(int32_t));
        prof.mark(prof.q);
        launch_query<T>(qsel, n_max, qmax, qi, cnt, qcfg, bv, out, pc, pv, ctl, ws.ovf.as<int32_t>(),
                        ws.deep.as<int2>(), s);
        prof.mark(prof.q);
        const L64Cfg l64{B->nodes.as<WideNode>(), bv64, iv.ids, pc, np, ws.gstack.as<int2>(), check_fp32};
        k_argmax_finalize<T><<<std::min<unsigned>(grid_for(n_max, BLK), GRID_MAX), BLK, 0, s>>>(qi, cnt, out.key,
                                                                                               out.I, pv, l64, ctl);
        if (np > ARGMAX_LAST_BLOCK_PAIRS) k_argmax_pairs<<<grid_for((int64_t)np * 4, BLK), BLK, 0, s>>>(pv, l64, ctl);
        HD_LAUNCH_CHECK();
    };

    // ---- autotuner: the query kernel's launch shape -------------------------
    // Times every variant on this call's vertex queries (best of three; no
    // effect on L: the trial queries do not raise it) and keeps the fastest
    // for this device and arithmetic, or the default when it is within 5% of
    // the fastest; later calls reuse the choice. With a cache file, a choice
    // kept there for this device, arithmetic and kernel source is taken
    // without tuning, and a new choice is added to it.
    tw.vq.ensure(mA);
    const int arith = sizeof(T) == 4 ? 0 : 1;
    std::string tkey;
    if (opt.autotune == 1 && !ws.tuned[arith] && opt.tuner_cache) {
        tkey = tuner_key(arith);
        for (const auto &e : tuner_read(opt.tuner_cache))
            if (e.first == tkey && e.second >= 0 && e.second < NQVAR) {
                qvar = e.second;
                ws.tuned[arith] = true;
                S.tuned = 2;
            }
    }
    if ((opt.autotune == 1 && !ws.tuned[arith]) || opt.autotune == 2) {
        QueryIn<T> qi{};
        qi.mode = Q_VERTICES;
        qi.npairs = np;
        qi.vids = ws.vids.as<int32_t>();
        qi.voff = dvoff;
        qi.a = av;
        qi.pc = pc;
        const QueryCfg tcfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 0, top};
        ws.ovf.reserve((size_t)mA * sizeof(int32_t));
        if (ws.tune_ev[0] == nullptr)
            for (auto &e : ws.tune_ev) HD_HIP(hipEventCreate(&e));
        float best = 0, t_default = 0;
        int pick = 0;
        for (int v = 0; v < NQVAR; ++v) {
            float t = 1e30f;
            for (int rep = 0; rep < 3; ++rep) {
                k_zero_query_stats<<<1, 64, 0, s>>>(ctl);
                HD_HIP(hipEventRecord(ws.tune_ev[0], s));
                launch_query<T>(v, mA, -1, qi, nref_dev, tcfg, bv, tw.vq.o, pc, pv, ctl,
                                ws.ovf.as<int32_t>(), ws.deep.as<int2>(), s);
                HD_HIP(hipEventRecord(ws.tune_ev[1], s));
                HD_HIP(hipEventSynchronize(ws.tune_ev[1]));
                float ms = 0;
                HD_HIP(hipEventElapsedTime(&ms, ws.tune_ev[0], ws.tune_ev[1]));
                t = std::min(t, ms);
            }
            if (v == 0) t_default = t;
            if (v == 0 || t < best) {
                best = t;
                pick = v;
            }
        }
        // keep the default unless another shape is clearly faster (timings
        // of one launch vary by a few percent)
        if (t_default <= 1.05f * best) pick = 0;
        k_zero_query_stats<<<1, 64, 0, s>>>(ctl);
        qvar = pick;
        ws.tuned[arith] = true;
        S.tuned = 1;
        if (opt.tuner_cache) {
            if (tkey.empty()) tkey = tuner_key(arith);
            auto entries = tuner_read(opt.tuner_cache);
            bool found = false;
            for (auto &e : entries)
                if (e.first == tkey) {
                    e.second = pick;
                    found = true;
                }
            if (!found) entries.emplace_back(tkey, pick);
            tuner_write(opt.tuner_cache, entries);
        }
    }
    qsel = small_stack ? -1 : (opt.query_shape > 0 ? opt.query_shape - 1 : qvar);
    S.query_block = qsel < 0 ? 128 : QVARIANTS[qsel].qb;
    S.query_stack = qsel < 0 ? SMALL_STACK : QVARIANTS[qsel].sd;
    S.query_lanes = opt.query_lanes;
    S.query_quad_max = qmax < 0 ? 0 : (qmax == INT64_MAX ? -1 : qmax);

    // ---- round 0: vertex queries ------------------------------------------
    {
        QueryIn<T> qi{};
        qi.mode = Q_VERTICES;
        qi.npairs = np;
        qi.vids = ws.vids.as<int32_t>();
        qi.voff = dvoff;
        qi.a = av;
        qi.pc = pc;
        run_queries(qi, nref_dev, mA, tw.vq.o); // counters set by k_ingest_post
    }

    // ---- frontier buffers ---------------------------------------------------
    int64_t cap0 = opt.capacity > 0 ? opt.capacity : std::max<int64_t>(int64_t(1) << 20, 4 * nA);
    cap0 = std::max<int64_t>(cap0, nA);
    tw.act.ensure(cap0, 0, s);
    tw.act2.ensure(cap0, 0, s);
    tw.park.ensure(cap0, 0, s);
    int64_t cap_limit = opt.capacity > 0 ? std::max<int64_t>(opt.capacity, nA) : (int64_t(1) << 30);

    ClassifyCfg cc;
    cc.c = cctx;
    cc.recheck = (opt.precision == HD_PREC_FP32_RECHECK) && sizeof(T) == 4;
    cc.shift = opt.test_bound_shift;
    bool has_u5 = false; // the order has the fifth bound (barycenter queries before stage B)
    for (int i = 0; i < cctx.norder; ++i) has_u5 = has_u5 || cctx.order[i] == 5;
    // stage B inside the vertex round's and the one-level planned rounds'
    // kernels (FP32, no barycenter queries, no learned bound policy)
    const bool fuse_b = sizeof(T) == 4 && !has_u5 && opt.learned != 2 && FUSE_STAGE_B;
    cc.a = av;
    cc.bv64 = bv64;
    cc.iv = iv;
    cc.pc = pc;
    cc.pv = pv;

    // stages B and C over what one round's stage A produced (at most n records)
    const LearnCfg lc{pc, pv, iv};
    // (defer: device-planned rounds may leave the recheck band to accumulate)
    const double budget = (opt.budget_m > 0 ? opt.budget_m : 1e7) * (double)nA;
    // The device plans each round itself (the sub-batch too, when there is
    // one) and the host enqueues one round ahead of the report it waits for:
    // the GPU never idles between rounds. The host-driven loop below handles
    // the frontier log and the round log.
    const bool planned = !opt.log_frontier && !logging;
    // device-planned rounds with sub-batches: the device selects each round's
    // sub-batch (k_sel_hist1, k_sel_hist2, k_sel_compact)
    const bool sel_round = planned && opt.subbatch > 0;
    // device-planned rounds: the stage lists follow the active lists (keep_c:
    // records waiting for stage C, kept when its list grows), and the
    // capacities each plan works with
    auto size_round = [&](int64_t keep_c) {
        const int64_t c = std::min(tw.act.cap, tw.act2.cap);
        tw.mq.ensure(c);
        tw.pend_b.ensure(c, 0, s);
        if (cc.recheck) tw.pend_c.ensure(c, keep_c, s);
        if (sel_round) ws.selidx.reserve(2 * (size_t)std::max(tw.act.cap, tw.act2.cap) * sizeof(int32_t));
    };
    auto caps = [&]() {
        PlanCaps c;
        c.act = std::min(tw.act.cap, tw.act2.cap);
        c.park = tw.park.cap;
        c.pend = tw.pend_b.cap;
        c.pend_c = cc.recheck ? tw.pend_c.cap : c.pend;
        c.mq = tw.mq.cap;
        c.budget = budget - (double)nA;
        c.grow_act = c.act < cap_limit;
        c.grow_park = c.park < cap_limit;
        c.subbatch = sel_round ? opt.subbatch : 0;
        c.learned = sel_round && opt.learned > 0 ? 1 : 0;
        // (sub-batched rounds: only a round that splits every live record,
        // a breadth-first round, goes deeper; the selection decides)
        c.two_max = opt.split_levels == 1
                        ? 0
                        : (opt.split_levels == 0 || opt.split_levels == 2 ? TWO_LEVEL_MAX : opt.split_levels);
        c.four_max = c.two_max > 0 && opt.split_levels != 2 ? FOUR_LEVEL_MAX : 0;
        return c;
    };
    // plan_seq != 0: the stages end a device-planned round (report under
    // that sequence number, plan the next), in stage C's last block when
    // there is a stage C, else in a kernel of their own
    auto later_stages = [&](int64_t n, const FrontierView<T> &act_out, int defer, unsigned plan_seq) {
        Dest<T> d{act_out, tw.park.v, tw.pend_b.v, tw.pend_c.v};
        const unsigned g = std::max(1u, std::min<unsigned>(grid_for(n, BLK), GRID_MAX));
        const int *Sb = nullptr;
        if (has_u5) {
            // the fifth bound: the closest B triangle of each waiting record's
            // barycenter (one point query each; they do not raise L)
            tw.bq.ensure(tw.pend_b.cap);
            QueryIn<T> qi{};
            qi.mode = Q_BARYCENTERS;
            qi.npairs = np;
            qi.a = av;
            qi.par = tw.pend_b.v;
            qi.pc = pc;
            const QueryCfg bcfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 0, top};
            ws.ovf.reserve((size_t)n * sizeof(int32_t));
            launch_query<T>(qsel, n, qmax, qi, DevCount{&ctl->b_next, 1, 0}, bcfg, bv, tw.bq.o, pc, pv, ctl,
                            ws.ovf.as<int32_t>(), ws.deep.as<int2>(), s);
            Sb = tw.bq.o.I;
        }
        // (with stage B in the kernels that create the triangles, nothing
        // is left for it: every such kernel of this run is the FUSE form)
        if (opt.learned == 2)
            k_stage_b_learned<T><<<g, BLK, 0, s>>>(tw.pend_b.v, cc, bv, d, ctl, lc, opt.mlp_params, Sb);
        else if (!(fuse_b && sizeof(T) == 4))
            k_stage_b<T><<<g, BLK, 0, s>>>(tw.pend_b.v, cc, bv, d, ctl, Sb);
        // (stage C's records are the few within the FP32 margin of a
        // decision: a grid of one block per CU, striding, suffices)
        if (cc.recheck)
            k_stage_c<T><<<std::min(g, C_GRID_MAX), BLK, 0, s>>>(tw.pend_c.v, cc, d, ctl, defer, mb_dev, plan_seq,
                                                                 plan_seq ? caps() : PlanCaps{});
        else if (plan_seq)
            k_report_plan<<<1, 64, 0, s>>>(ctl, pv, mb_dev, plan_seq, caps());
        HD_LAUNCH_CHECK();
    };

    // the results (control block, pair tables) to pinned host memory; returns
    // the sequence number the host waits for
    auto enqueue_export = [&]() -> unsigned {
        Export ex{};
        ex.n = 3;
        ex.src[0] = ctl;
        ex.dst[0] = ws.host.dev_as<char>(o_res + o_rctl);
        ex.bytes[0] = CTL_HOST_BYTES;
        ex.src[1] = pv;
        ex.dst[1] = ws.host.dev_as<char>(o_res + o_rpv);
        ex.bytes[1] = np * sizeof(PairVar);
        ex.src[2] = pc;
        ex.dst[2] = ws.host.dev_as<char>(o_res + o_rpc);
        ex.bytes[2] = np * sizeof(PairConst);
        const unsigned seq = ++ws.mb_seq;
        export_to_host(ex, ws.host.dev_as<unsigned>(HOST_EXPORT_SEQ), seq, s);
        return seq;
    };
    // round log: each pair's largest live bound (active and parked lists,
    // counts on the device) into PairVar::Uround before the round's report,
    // and one record per report
    Mailbox hm{}; // the latest report read
    auto round_U = [&](const FrontierView<T> &act_out) {
        if (!logging) return;
        k_round_U_reset<<<grid_for(np, 64), 64, 0, s>>>(pv, np);
        k_round_U<T><<<std::min<unsigned>(grid_for(tw.act.cap + tw.park.cap, BLK), GRID_MAX), BLK, 0, s>>>(
            act_out, tw.park.v, ctl, pv);
        HD_LAUNCH_CHECK();
    };
    auto log_round = [&](int r, int64_t split) {
        if (!logging || S.round_records >= opt.round_log_cap) return;
        hd_round_record &R = opt.round_log[S.round_records++];
        std::memset(&R, 0, sizeof(R));
        R.round = r;
        R.split = split;
        R.active = hm.act;
        R.parked = hm.park;
        R.bounded = hm.bounded;
        for (int k = 0; k < 5; ++k) R.discards[k] = hm.discards[k];
        R.L = hm.L0;
        R.U = hm.U0;
        R.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    };
    // a final step and export enqueued ahead of the last round's report
    // (used when that report shows the run converged)
    bool spec = false;
    unsigned spec_seq = 0;

    // ---- round 0: bound every face ------------------------------------------
    // (planned rounds: the stage lists get the active lists' size now, so that
    // recheck records deferred from round 0 are never moved by a resize)
    const int64_t pend0 = planned ? std::max<int64_t>(nA, std::min(tw.act.cap, tw.act2.cap)) : nA;
    tw.pend_b.ensure(pend0, 0, s);
    if (cc.recheck) tw.pend_c.ensure(pend0, 0, s);
    // planned rounds: round 0's stages also report it and plan round 1
    unsigned seq0 = 0;
    if (planned) {
        size_round(0); // no resize here (round 0 sized the stage lists): deferred records stay
        seq0 = ++ws.mb_seq;
    }
    if (sel_round) {
        ws.selhist.reserve(2 * SEL_BINS * sizeof(unsigned));
        k_zero_u32<<<grid_for(2 * SEL_BINS, BLK), BLK, 0, s>>>(ws.selhist.as<unsigned>(), 2 * SEL_BINS);
        HD_LAUNCH_CHECK();
    }
    prof.mark(prof.c);
    {
        const Dest<T> d0{tw.act.v, tw.park.v, tw.pend_b.v, tw.pend_c.v};
        bool fused = false;
        if constexpr (sizeof(T) == 4) {
            if (fuse_b) {
                k_round0<T, 1><<<grid_for(nA, BLK), BLK, 0, s>>>(nA, ws.Fcat.as<int32_t>(), ws.fpair.as<int32_t>(),
                                                                 tw.vq.o, cc, d0, ctl, bv);
                fused = true;
            }
        }
        if (!fused)
            k_round0<T><<<grid_for(nA, BLK), BLK, 0, s>>>(nA, ws.Fcat.as<int32_t>(), ws.fpair.as<int32_t>(), tw.vq.o,
                                                          cc, d0, ctl, bv);
    }
    HD_LAUNCH_CHECK();
    later_stages(nA, tw.act.v, planned ? 1 : 0, seq0);
    prof.mark(prof.c);
    double processed = (double)nA;
    int64_t subdivided = 0, logged = 0, nAct = 0, nPark = 0;
    int rounds = 0;
    hd_status status = HD_OK;
    if (planned) {
        // report the state after a round and plan the next one
        auto report_plan_async = [&]() -> unsigned {
            const unsigned seq = ++ws.mb_seq;
            k_report_plan<<<1, 64, 0, s>>>(ctl, pv, mb_dev, seq, caps());
            HD_LAUNCH_CHECK();
            return seq;
        };
        // a round as planned by the report before it
        auto enqueue_round = [&]() {
            const PlanCaps c = caps();
            const int64_t kmax = std::min<int64_t>(c.mq / 3, c.act);
            const int32_t *selp = nullptr, *restp = nullptr;
            if (sel_round) {
                // the sub-batch: score the new records (learned order), then
                // select by key, dropping and parking what the current L
                // decides (the counts are on the device)
                const int64_t cap_act = tw.act.cap;
                SelCfg sc{ws.selhist.as<unsigned>(), ws.selhist.as<unsigned>() + SEL_BINS,
                          ws.selidx.as<int32_t>(), ws.selidx.as<int32_t>() + std::max(tw.act.cap, tw.act2.cap),
                          opt.learned > 0 ? 1 : 0, c.budget, (int64_t)opt.subbatch, c.two_max, c.four_max};
                const unsigned gs = std::max(1u, std::min<unsigned>(grid_for(cap_act, BLK), SEL_GRID_MAX));
                if (opt.learned > 0)
                    k_score_new<T><<<std::min<unsigned>(grid_for(cap_act, BLK), GRID_MAX), BLK, 0, s>>>(
                        tw.act.v, ctl, lc, bv, opt.mlp_params);
                k_sel_hist1<T><<<gs, BLK, 0, s>>>(tw.act.v, sc, pc, pv, ctl);
                k_sel_hist2<T><<<gs, BLK, 0, s>>>(tw.act.v, sc, pc, pv, ctl);
                k_sel_compact<T><<<std::min<unsigned>(grid_for(cap_act, BLK), GRID_MAX), BLK, 0, s>>>(
                    tw.act.v, tw.park.v, sc, pc, pv, ctl);
                HD_LAUNCH_CHECK();
                selp = sc.sel;
                restp = sc.rest;
            }
            QueryIn<T> qi{};
            qi.mode = Q_MIDPOINTS;
            qi.npairs = np;
            qi.a = av;
            qi.par = tw.act.v;
            qi.pc = pc;
            qi.sel = selp;
            qi.two = &ctl->plan_two;
            // (the plan keeps the round's queries, 3 or 12 per parent, within
            // 3 * kmax: two-level rounds need room for 16 children per parent)
            run_queries(qi, DevCount{&ctl->plan_Q, 1, 0}, 3 * kmax, tw.mq.o);
            prof.mark(prof.c);
            bool fused = false;
            if constexpr (sizeof(T) == 4) {
                if (fuse_b) {
                    k_children<T, 0, 1><<<std::min<unsigned>(grid_for(4 * kmax, BLK), GRID_MAX), BLK, 0, s>>>(
                        DevCount{&ctl->plan_K, 1, 0}, tw.act.v, tw.mq.o, cc,
                        Dest<T>{tw.act2.v, tw.park.v, tw.pend_b.v, tw.pend_c.v}, ctl, 1, selp, restp, bv);
                    fused = true;
                }
            }
            if (!fused)
                k_children<T, 0><<<std::min<unsigned>(grid_for(4 * kmax, BLK), GRID_MAX), BLK, 0, s>>>(
                    DevCount{&ctl->plan_K, 1, 0}, tw.act.v, tw.mq.o, cc,
                    Dest<T>{tw.act2.v, tw.park.v, tw.pend_b.v, tw.pend_c.v}, ctl, 1, selp, restp, bv);
            if (c.two_max > 0) {
                const unsigned g2 = std::min<unsigned>(grid_for(16 * std::min(kmax, c.two_max), BLK), GRID_MAX);
                const Dest<T> d2{tw.act2.v, tw.park.v, tw.pend_b.v, tw.pend_c.v};
                bool fused2 = false;
                if constexpr (sizeof(T) == 4) {
                    if (fused) {
                        k_children<T, 1, 1><<<g2, BLK, 0, s>>>(DevCount{&ctl->plan_K, 1, 0}, tw.act.v, tw.mq.o, cc,
                                                               d2, ctl, 1, selp, restp, bv);
                        fused2 = true;
                    }
                }
                if (!fused2)
                    k_children<T, 1><<<g2, BLK, 0, s>>>(DevCount{&ctl->plan_K, 1, 0}, tw.act.v, tw.mq.o, cc, d2, ctl,
                                                        1, selp, restp, bv);
            }
            HD_LAUNCH_CHECK();
            const unsigned seq = ++ws.mb_seq;
            later_stages(4 * kmax, tw.act2.v, 1, seq);
            prof.mark(prof.c);
            swap_fb(tw.act, tw.act2);
            return seq;
        };
        unsigned seq_prev = seq0; // state after round 0 (the latest report not yet read)
        int enqueued = 0;
        int64_t peak = 0;
        int64_t last_act = -1; // active count of the last report read (-1: none yet)
        while (true) {
            const bool more = !(opt.max_rounds > 0 && enqueued >= opt.max_rounds);
            // The next round goes in ahead of the pending report, unless the
            // last report read left so few active triangles that the pending
            // round is likely the last: an empty round costs its five
            // launches, a missed look-ahead one host reaction.
            const bool ahead = more && !(last_act >= 0 && last_act <= LOOKAHEAD_MIN);
            unsigned seq_new = 0;
            if (ahead) {
                seq_new = enqueue_round();
                ++enqueued;
            } else if (more) {
                // the pending round is probably the last: its final step and
                // export go in ahead of its report, and do nothing on the
                // device unless the run has converged
                prof.mark(prof.c);
                k_final_U<T><<<std::min<unsigned>(grid_for(tw.park.cap, BLK), GRID_MAX), BLK, 0, s>>>(
                    tw.park.v, DevCount{&ctl->park_next, 1, 0}, 1, av, bv64, iv, cctx, pc, pv, ctl);
                HD_LAUNCH_CHECK();
                prof.mark(prof.c);
                spec_seq = enqueue_export();
                spec = true;
            }
            hm = wait_report(seq_prev);
            peak = std::max<int64_t>(peak, hm.act + hm.park);
            last_act = hm.act;
            const bool done = hm.act == 0 || hm.bad || hm.over_budget || hm.stall;
            if (ahead) {
                seq_prev = seq_new;
                if (!done) continue;
                // the round enqueued ahead found nothing to do (or stopped too)
                hm = wait_report(seq_new);
                peak = std::max<int64_t>(peak, hm.act + hm.park);
                last_act = hm.act;
            } else if (more && !done) {
                spec = false;
                seq_prev = enqueue_round();
                ++enqueued;
                continue;
            }
            if (!(hm.stall && !hm.bad && !hm.over_budget && hm.act > 0)) break;
            // out of list capacity: grow (the stalled rounds left the lists in
            // place) and go on, or give up at the limit
            const int64_t cur = std::min(tw.act.cap, tw.act2.cap);
            if (cur >= cap_limit && tw.park.cap >= cap_limit) break;
            const int64_t grow = std::min<int64_t>(cap_limit, std::max<int64_t>(2 * cur, 4 * hm.act));
            try {
                tw.act.ensure(grow, hm.act, s);
                tw.act2.ensure(grow, 0, s);
                tw.park.ensure(std::min<int64_t>(cap_limit, std::max<int64_t>(2 * tw.park.cap, hm.park + 4 * hm.act)), hm.park, s);
                size_round(hm.pend_c);
            } catch (const Error &e) {
                if (e.st != HD_E_NOMEM) throw;
                // out of device memory: the lists stay as they are and the
                // rounds split what fits (sub-batches)
                cap_limit = std::min(std::min(tw.act.cap, tw.act2.cap), tw.park.cap);
                size_round(hm.pend_c);
            }
            spec = false;
            k_clear_stall<<<1, 64, 0, s>>>(ctl);
            seq_prev = report_plan_async();
            enqueued = (int)hm.rounds; // stalled rounds split nothing and do not count
        }
        if (cc.recheck && hm.pend_c > 0 && !hm.bad) {
            // the rounds stopped early (round limit, budget, capacity) with
            // records still waiting for stage C: decide them now, so that the
            // final U covers them (the lists have room: plans reserve it)
            tw.act.ensure(hm.act + hm.pend_c, hm.act, s);
            tw.park.ensure(hm.park + hm.pend_c, hm.park, s);
            k_set_counts<<<1, 64, 0, s>>>(ctl, (unsigned long long)hm.act, (unsigned long long)hm.park);
            k_stage_c<T><<<std::min<unsigned>(grid_for(hm.pend_c, BLK), GRID_MAX), BLK, 0, s>>>(
                tw.pend_c.v, cc, Dest<T>{tw.act.v, tw.park.v, tw.pend_b.v, tw.pend_c.v}, ctl, 0, nullptr, 0u,
                PlanCaps{});
            HD_LAUNCH_CHECK();
            spec = false;
            const Mailbox hf = report();
            hm.act = hf.act;
            hm.park = hf.park;
            hm.bad = hf.bad;
        }
        nAct = hm.act;
        nPark = hm.park;
        rounds = (int)hm.rounds;
        subdivided = hm.subdivided;
        S.max_frontier = peak;
        if (hm.bad) status = status_of_bad(hm.bad);
        else if (hm.over_budget || (hm.stall && hm.act > 0)) status = HD_E_CAPACITY;
    } else {
        round_U(tw.act.v);
        hm = report();
        nAct = hm.act;
        nPark = hm.park;
        S.max_frontier = nAct + nPark;
        if (hm.bad) status = status_of_bad(hm.bad);
        log_round(0, 0);
    }
    // learned order: every record is scored once, when it joins the active
    // list (only needed when sub-batches are selected)
    const bool scoring = opt.learned > 0 && opt.subbatch > 0;
    auto score_new = [&](int64_t from, int64_t to) {
        if (!scoring || to <= from) return;
        k_score<T><<<grid_for(to - from, BLK), BLK, 0, s>>>(tw.act.v, from, to - from, lc, bv, opt.mlp_params);
        HD_LAUNCH_CHECK();
    };
    if (!planned) score_new(0, nAct);

    while (!planned && status == HD_OK && nAct > 0) {
        if (opt.max_rounds > 0 && rounds >= opt.max_rounds) break;
        // how many to split this round, growing the lists when allowed
        int64_t K = nAct;
        if (opt.subbatch > 0) K = std::min<int64_t>(K, opt.subbatch);
        auto fits = [&](int64_t k) {
            return nAct + 3 * k <= std::min(tw.act.cap, tw.act2.cap) && nPark + 4 * k <= tw.park.cap;
        };
        if (!fits(K)) {
            int64_t need_act = std::min(cap_limit, nAct + 3 * K), need_park = std::min(cap_limit, nPark + 4 * K);
            try {
                tw.act.ensure(need_act, nAct, s);
                tw.act2.ensure(need_act, 0, s);
                tw.park.ensure(need_park, nPark, s);
            } catch (const Error &e) {
                if (e.st != HD_E_NOMEM) throw;
            }
            K = std::min<int64_t>(K, std::min((std::min(tw.act.cap, tw.act2.cap) - nAct) / 3,
                                              (tw.park.cap - nPark) / 4));
        }
        if (K <= 0) {
            status = HD_E_CAPACITY;
            break;
        }
        if (processed + 4.0 * (double)K > budget) {
            status = HD_E_CAPACITY;
            break;
        }
        if (K < nAct) {
            // largest upper bounds first (the paper's priority-queue order)
            ws.sortbuf.reserve((size_t)nAct * 24 + 1024);
            unsigned long long *keys = ws.sortbuf.as<unsigned long long>();
            unsigned long long *keys2 = keys + nAct;
            int32_t *vals = (int32_t *)(keys2 + nAct);
            int32_t *vals2 = vals + nAct;
            if (opt.learned > 0) {
                // the network's predicted maximum distance (scored when each
                // record joined the active list) orders the frontier
                k_sel_keys_learned<T><<<grid_for(nAct, BLK), BLK, 0, s>>>(tw.act.v, nAct, keys, vals);
            } else {
                k_sel_keys<T><<<grid_for(nAct, BLK), BLK, 0, s>>>(tw.act.v, nAct, keys, vals);
            }
            radix_sort_u64(keys, vals, keys2, vals2, nAct, 64, ws.sort_tmp, s);
            k_gather<T><<<grid_for(nAct, BLK), BLK, 0, s>>>(tw.act.v, vals, 0, nAct, tw.act2.v);
            HD_LAUNCH_CHECK();
            swap_fb(tw.act, tw.act2);
        }
        const int64_t rest = nAct - K;
        k_round_setup<<<1, 1, 0, s>>>(ctl, (unsigned long long)rest, (unsigned long long)nPark);
        if (opt.log_frontier && logged < opt.log_cap) {
            // the parents' features and labels: 12 lattice queries each (they do
            // not raise L, so the logged run follows the plain one)
            tw.lq.ensure(LATTICE_PTS * K);
            QueryIn<T> li{};
            li.mode = Q_LATTICE;
            li.npairs = np;
            li.a = av;
            li.par = tw.act.v;
            li.pc = pc;
            const QueryCfg lcfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 0, top};
            const int64_t nq = LATTICE_PTS * K;
            ws.ovf.reserve((size_t)nq * sizeof(int32_t));
            launch_query<T>(qsel, nq, qmax, li, host_count(nq), lcfg, bv, tw.lq.o, pc, pv, ctl, ws.ovf.as<int32_t>(),
                            ws.deep.as<int2>(), s);
            k_log_parents<T><<<grid_for(K, BLK), BLK, 0, s>>>(tw.act.v, K, tw.lq.o, lc, bv, opt.log_out, logged,
                                                              opt.log_cap);
            HD_LAUNCH_CHECK();
            logged += std::min<int64_t>(K, opt.log_cap - logged);
            k_round_setup<<<1, 1, 0, s>>>(ctl, (unsigned long long)rest, (unsigned long long)nPark);
        }
        // midpoints of the K selected parents
        tw.mq.ensure(3 * K);
        QueryIn<T> qi{};
        qi.mode = Q_MIDPOINTS;
        qi.npairs = np;
        qi.a = av;
        qi.par = tw.act.v;
        qi.pc = pc;
        run_queries(qi, host_count(3 * K), 3 * K, tw.mq.o);
        // the unselected remainder first, then the active children
        if (rest > 0) k_gather<T><<<grid_for(rest, BLK), BLK, 0, s>>>(tw.act.v, nullptr, K, rest, tw.act2.v);
        tw.pend_b.ensure(4 * K, 0, s);
        if (cc.recheck) tw.pend_c.ensure(4 * K, 0, s);
        prof.mark(prof.c);
        {
            const unsigned gk = std::min<unsigned>(grid_for(4 * K, BLK), GRID_MAX);
            const Dest<T> dk{tw.act2.v, tw.park.v, tw.pend_b.v, tw.pend_c.v};
            bool fusedk = false;
            if constexpr (sizeof(T) == 4) {
                if (fuse_b) {
                    k_children<T, 0, 1><<<gk, BLK, 0, s>>>(host_count(K), tw.act.v, tw.mq.o, cc, dk, ctl, 0, nullptr,
                                                           nullptr, bv);
                    fusedk = true;
                }
            }
            if (!fusedk)
                k_children<T, 0><<<gk, BLK, 0, s>>>(host_count(K), tw.act.v, tw.mq.o, cc, dk, ctl, 0, nullptr, nullptr,
                                                    bv);
        }
        HD_LAUNCH_CHECK();
        later_stages(4 * K, tw.act2.v, 0, 0);
        prof.mark(prof.c);
        round_U(tw.act2.v);
        hm = report();
        swap_fb(tw.act, tw.act2);
        nAct = hm.act;
        nPark = hm.park;
        score_new(rest, nAct);
        subdivided += K;
        processed += 4.0 * (double)K;
        ++rounds;
        S.max_frontier = std::max<int64_t>(S.max_frontier, nAct + nPark);
        if (hm.bad) status = status_of_bad(hm.bad);
        log_round(rounds, K);
    }

    // ---- final FP64 step: U over every live triangle --------------------------

    // the final step enqueued ahead stands when the rounds converged (its
    // launch then did the work below)
    const bool use_spec = spec && status == HD_OK && nAct == 0 && hm.pend_c == 0;
    if (status == HD_OK && !use_spec) {
        prof.mark(prof.c);
        if (nPark > 0)
            k_final_U<T><<<std::min<unsigned>(grid_for(nPark, BLK), GRID_MAX), BLK, 0, s>>>(
                tw.park.v, host_count(nPark), 0, av, bv64, iv, cctx, pc, pv, ctl);
        if (nAct > 0)
            k_final_U<T><<<std::min<unsigned>(grid_for(nAct, BLK), GRID_MAX), BLK, 0, s>>>(
                tw.act.v, host_count(nAct), 0, av, bv64, iv, cctx, pc, pv, ctl);
        HD_LAUNCH_CHECK();
        prof.mark(prof.c);
    }
    {
        const unsigned seq = use_spec ? spec_seq : enqueue_export();
        wait_host_seq(ws.host.as<unsigned>(HOST_EXPORT_SEQ), seq, s);
    }
    const Ctl &hc = *ws.host.as<Ctl>(o_res + o_rctl);
    auto stat = [&](int k) {
        unsigned long long t = 0;
        for (int c = 0; c < ACC_COPIES; ++c) t += hc.stat[c][k];
        return t;
    };
    const PairVar *hp = ws.host.as<PairVar>(o_res + o_rpv);
    const PairConst *hc_ = ws.host.as<PairConst>(o_res + o_rpc);
    if (status == HD_OK && hc.bad) status = status_of_bad(hc.bad);
    if (status == HD_OK) {
        for (int p = 0; p < np; ++p) {
            // a pair's own lower bound, and the (shared) one its decisions used
            const double L = ord2d(hp[p].Lord);
            const double Ld = std::max(L, ord2d(hp[hc_[p].link].Lord));
            const double U = std::max(Ld, ord2d(hp[p].Uord));
            LU[2 * p] = L;
            LU[2 * p + 1] = U;
            if (nAct == 0 && U - Ld > hc_[p].eps_abs) status = HD_E_INTERNAL;
        }
        if (nAct > 0 && opt.max_rounds <= 0) status = HD_E_INTERNAL;
    }
    S.rounds = rounds;
    S.status = status;
    S.nodes_bounded = (int64_t)stat(ST_BOUNDED);
    S.subdivided = subdivided;
    S.queries = (int64_t)stat(ST_QUERIES);
    S.pt_tri_evals = (int64_t)(stat(ST_EVALS) + stat(ST_QLEAVES));
    S.box_tests = (int64_t)stat(ST_BOXES);
    for (int k = 0; k < 5; ++k) S.discards[k] = (int64_t)stat(ST_DISCARDS + k);
    S.discards_u5 = (int64_t)stat(ST_DISCARDS + 5);
    S.device_flag = hc.bad;
    S.rechecked64 = (int64_t)stat(ST_RECHECKED);
    S.parked_final = nPark;
    S.query_leaf_evals = (int64_t)stat(ST_QLEAVES);
    S.query_box_tests = (int64_t)stat(ST_BOXES);
    S.logged = logged;
    S.learned_skips = (int64_t)stat(ST_SKIPS);
    S.stale = (int64_t)stat(ST_STALE);
    S.stack_overflows = (int64_t)stat(ST_OVERFLOWS);
    S.dA = hc_[0].dA;
    S.eps_abs = hc_[0].eps_abs;
    S.mu_coef_d = margins_of<T>(hc_[0]).mu_d;
    S.mu_coef_0 = margins_of<T>(hc_[0]).mu_0;
    S.L_rounds = ord2d(hp[0].Lord);
    S.U_rounds = std::max(S.L_rounds, ord2d(hp[0].Urounds));
    if (prof.on) {
        S.ms_query_kernels = Profiler::sum(prof.q);
        S.ms_cascade_kernels = Profiler::sum(prof.c);
        S.query_launches = (int64_t)prof.q.size() / 2;
        S.cascade_launches = (int64_t)prof.c.size() / 2;
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

// ---- scratch of hd_point_distances_noalloc --------------------------------
// Callers that cannot allocate get their scratch (the control block, the pair
// tables, the overflow list, the deep stack and the query results) from one
// static device array per GPU, held until the process ends. Host code never
// uses the array's name as an address: the device address comes from
// hipGetSymbolAddress, once per device, and is kept in g_scratch_dev.
namespace {
constexpr size_t al256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t NA_CTL = 0;
constexpr size_t NA_PC = NA_CTL + al256(sizeof(Ctl));
constexpr size_t NA_PV = NA_PC + al256(sizeof(PairConst));
constexpr size_t NA_OVF = NA_PV + al256(sizeof(PairVar));
constexpr size_t NA_DEEP = NA_OVF + al256((size_t)HD_NOALLOC_MAX_POINTS * sizeof(int32_t));
constexpr size_t NA_Q = NA_DEEP + al256((size_t)DEEP_SLOTS * DEEP_STACK * sizeof(int2));
constexpr size_t NA_BYTES = NA_Q + qout_bytes<double>(HD_NOALLOC_MAX_POINTS); // FP64 results are the larger
static_assert(qout_bytes<double>(1) >= qout_bytes<float>(1), "FP64 query results need more room");
} // namespace

static __device__ __align__(256) unsigned char scratch[NA_BYTES];

static std::mutex g_scratch_mu;
static void *g_scratch_dev[64] = {};

// the device address of `scratch` on the current device (looked up once per device)
static char *scratch_on_current_device() {
    int dev = 0;
    HD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) throw Error{HD_E_DEVICE, "device index out of range"};
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        HD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_dev[dev] = p;
    }
    return static_cast<char *>(g_scratch_dev[dev]);
}

namespace hd {
namespace {
__global__ void k_write_status(int32_t *err, int32_t v) {
    if (threadIdx.x == 0) *err = v;
}
} // namespace
} // namespace hd

static hd_status guard(const std::function<hd_status()> &fn) {
    try {
        return fn();
    } catch (const Error &e) {
        return e.st;
    } catch (...) {
        return HD_E_INTERNAL;
    }
}

// the calling thread's device workspace, or a private one if another call
// holds it
struct WsLease {
    Workspace *ws = nullptr;
    Workspace *owned = nullptr;
    std::unique_lock<std::mutex> lk;
    WsLease() {
        int dev = 0;
        (void)hipGetDevice(&dev);
        Workspace *w = workspace_for(dev);
        lk = std::unique_lock<std::mutex>(w->mu, std::try_to_lock);
        if (lk.owns_lock()) {
            ws = w;
        } else {
            owned = new Workspace();
            ws = owned;
        }
    }
    ~WsLease() { delete owned; }
};

static hd_status bound_any(const Input &in, hd_bvh Bh, const hd_options *opt, hd_stream_t stream, double *LU,
                           hd_stats *stats) {
    hd_options o;
    hd_default_options(&o);
    if (opt) o = *opt;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    return guard([&] {
        WsLease lease;
        std::vector<double> lu(2 * (size_t)in.npairs, NAN);
        hd_status r = HD_E_INVALID;
        auto trim = [&] {
            // the work already enqueued may still use the buffers
            (void)hipStreamSynchronize((hipStream_t)stream);
            (void)hipGetLastError();
            lease.ws->trim();
        };
        try {
            if (o.precision == HD_PREC_FP64)
                r = run<double>(in, B, o, (hipStream_t)stream, *lease.ws, lu.data(), stats);
            else if (o.precision == HD_PREC_FP32 || o.precision == HD_PREC_FP32_RECHECK)
                r = run<float>(in, B, o, (hipStream_t)stream, *lease.ws, lu.data(), stats);
            else
                return HD_E_INVALID;
        } catch (const Error &e) {
            if (e.st == HD_E_NOMEM) trim();
            throw;
        }
        if (r == HD_E_NOMEM || r == HD_E_CAPACITY) trim();
        if (r == HD_OK) std::copy(lu.begin(), lu.end(), LU);
        return r;
    });
}

extern "C" {

const char *hd_status_str(hd_status s) {
    switch (s) {
    case HD_OK: return "ok";
    case HD_E_INVALID: return "invalid argument";
    case HD_E_CAPACITY: return "capacity, face budget or subdivision depth exceeded";
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
    return hd_build_bvh_batched(1, &VB, &mB, &FB, &nB, stream, out);
}

hd_status hd_build_bvh_batched(int32_t npairs, const double *const *VB, const int64_t *mB, const int32_t *const *FB,
                               const int64_t *nB, hd_stream_t stream, hd_bvh *out) {
    if (!out) return HD_E_INVALID;
    *out = nullptr;
    if (npairs <= 0 || !VB || !mB || !FB || !nB) return HD_E_INVALID;
    return guard([&] {
        Bvh *b = build_bvh(npairs, VB, mB, FB, nB, (hipStream_t)stream);
        *out = reinterpret_cast<hd_bvh>(b);
        return HD_OK;
    });
}

void hd_free_bvh(hd_bvh b) { recycle_bvh(reinterpret_cast<Bvh *>(b)); }

int32_t hd_build_graphs(int32_t enable) { return set_build_graphs(enable); }

hd_status hd_bound(const double *VA, int64_t mA, const int32_t *FA, int64_t nA, hd_bvh Bh, double eps,
                   const hd_options *opt, hd_stream_t stream, double LU_out[2], hd_stats *stats) {
    if (LU_out) LU_out[0] = LU_out[1] = NAN;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->status = HD_E_INVALID;
    }
    if (!LU_out || !Bh || !VA || !FA || mA <= 0 || nA <= 0) return HD_E_INVALID;
    Input in{1, &VA, &mA, &FA, &nA, &eps, 0};
    hd_status st = bound_any(in, Bh, opt, stream, LU_out, stats);
    if (stats) stats->status = st;
    return st;
}

hd_status hd_bound_batched(int32_t npairs, const double *const *VA, const int64_t *mA, const int32_t *const *FA,
                           const int64_t *nA, hd_bvh Bh, const double *eps, int32_t eps_per_pair,
                           const hd_options *opt, hd_stream_t stream, double *LU_out, hd_stats *stats) {
    if (LU_out)
        for (int p = 0; p < npairs; ++p) LU_out[2 * p] = LU_out[2 * p + 1] = NAN;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->status = HD_E_INVALID;
    }
    if (npairs <= 0 || !LU_out || !Bh || !VA || !mA || !FA || !nA || !eps) return HD_E_INVALID;
    Input in{npairs, VA, mA, FA, nA, eps, eps_per_pair ? 1 : 0};
    hd_status st = bound_any(in, Bh, opt, stream, LU_out, stats);
    if (stats) stats->status = st;
    return st;
}

hd_status hd_hausdorff(const double *VA, int64_t mA, const int32_t *FA, int64_t nA, const double *VB, int64_t mB,
                       const int32_t *FB, int64_t nB, double eps, const hd_options *opt, hd_stream_t stream,
                       double LU_out[2], double LU_dir[4], hd_stats *stats) {
    if (LU_out) LU_out[0] = LU_out[1] = NAN;
    if (LU_dir)
        for (int k = 0; k < 4; ++k) LU_dir[k] = NAN;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->status = HD_E_INVALID;
    }
    if (!LU_out || !VA || !FA || !VB || !FB || mA <= 0 || nA <= 0 || mB <= 0 || nB <= 0) return HD_E_INVALID;
    hipStream_t s = (hipStream_t)stream;
    hd_status st = guard([&] {
        // one BVH over both soups: pair 0 queries B (for h(A,B)), pair 1 queries A (for h(B,A))
        const double *Vt[2] = {VB, VA};
        const int32_t *Ft[2] = {FB, FA};
        const int64_t mt[2] = {mB, mA}, nt[2] = {nB, nA};
        Bvh *b = build_bvh(2, Vt, mt, Ft, nt, s);
        struct Release {
            Bvh *b;
            ~Release() { recycle_bvh(b); }
        } release{b};
        const double *Vs[2] = {VA, VB};
        const int32_t *Fs[2] = {FA, FB};
        const int64_t ms[2] = {mA, mB}, ns[2] = {nA, nB};
        Input in{2, Vs, ms, Fs, ns, &eps, 0, 1};
        double lu[4];
        const hd_status r = bound_any(in, reinterpret_cast<hd_bvh>(b), opt, stream, lu, stats);
        if (r != HD_OK) return r;
        // H = max(h(A,B), h(B,A)): the larger lower bound, the larger upper bound
        LU_out[0] = std::max(lu[0], lu[2]);
        LU_out[1] = std::max(lu[1], lu[3]);
        if (LU_dir)
            for (int k = 0; k < 4; ++k) LU_dir[k] = lu[k];
        return HD_OK;
    });
    if (stats) stats->status = st;
    return st;
}

hd_status hd_point_distances(const double *P, int64_t nP, hd_bvh Bh, int32_t precision, int32_t lanes, double *d,
                             int32_t *I, double *Q, hd_stream_t stream) {
    if (!Bh || nP < 0 || (nP > 0 && (!P || !d || !I))) return HD_E_INVALID;
    if (lanes != 0 && lanes != 1 && lanes != 4) return HD_E_INVALID;
    if (nP == 0) return HD_OK;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard([&] {
        DBuf ctlb, pcb, pvb, ovf, deep;
        ctlb.reserve(sizeof(Ctl));
        pcb.reserve(sizeof(PairConst));
        pvb.reserve(sizeof(PairVar));
        ovf.reserve((size_t)nP * sizeof(int32_t));
        deep.reserve((size_t)DEEP_SLOTS * DEEP_STACK * sizeof(int2));
        Ctl *ctl = ctlb.as<Ctl>();
        PairConst *pc = pcb.as<PairConst>();
        PairVar *pv = pvb.as<PairVar>();
        k_ctl_init<<<1, 256, 0, s>>>(ctl);
        k_pairs_init<<<1, 64, 0, s>>>(pc, pv, B->pairs.as<BvhPair>(), 1);
        const WideNode *top = B->npairs == 1 && !B->hpairs.empty() && B->hpairs[0].root >= 0
                                  ? B->top.as<WideNode>()
                                  : nullptr;
        const QueryCfg cfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 0, top};
        auto go = [&](auto tag) {
            using T = decltype(tag);
            QBuf<T> qb;
            qb.ensure(nP);
            QueryIn<T> qi{};
            qi.mode = Q_POINTS;
            qi.npairs = 1;
            qi.P = P;
            qi.pc = pc;
            BView<T> bv;
            if constexpr (sizeof(T) == 4) bv = BView<float>{B->frames32.as<float4>()};
            else bv = BView<double>{B->frames64.as<double2>()};
            launch_query<T>(0, nP, lanes == 4 ? INT64_MAX : -1, qi, host_count(nP), cfg, bv, qb.o, pc, pv, ctl,
                            ovf.as<int32_t>(), deep.as<int2>(), s);
            k_export_points<T><<<grid_for(nP, BLK), BLK, 0, s>>>(qb.o, nP, B->ids.as<int4>(), pc, d, I, Q, ctl,
                                                                 nullptr);
            HD_LAUNCH_CHECK();
            HD_HIP(hipStreamSynchronize(s));
        };
        if (precision == HD_PREC_FP64) go(double{});
        else go(float{});
        Ctl hc;
        HD_HIP(hipMemcpy(&hc, ctl, CTL_HOST_BYTES, hipMemcpyDeviceToHost));
        if (hc.bad == 2) return HD_E_INTERNAL;
        return HD_OK;
    });
}

hd_status hd_point_distances_noalloc(const double *P, int64_t nP, hd_bvh Bh, int32_t precision, int32_t lanes,
                                     double *d, int32_t *I, double *Q, int32_t *err, hd_stream_t stream) {
    if (!Bh || !err || nP < 0 || (nP > 0 && (!P || !d || !I))) return HD_E_INVALID;
    if (lanes != 0 && lanes != 1 && lanes != 4) return HD_E_INVALID;
    if (precision != HD_PREC_FP64 && precision != HD_PREC_FP32 && precision != HD_PREC_FP32_RECHECK)
        return HD_E_INVALID;
    if (nP > HD_NOALLOC_MAX_POINTS) return HD_E_CAPACITY;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard([&] {
        char *sc = scratch_on_current_device();
        if (nP == 0) {
            k_write_status<<<1, 64, 0, s>>>(err, HD_OK);
            HD_LAUNCH_CHECK();
            return HD_OK;
        }
        Ctl *ctl = reinterpret_cast<Ctl *>(sc + NA_CTL);
        PairConst *pc = reinterpret_cast<PairConst *>(sc + NA_PC);
        PairVar *pv = reinterpret_cast<PairVar *>(sc + NA_PV);
        int32_t *ovf = reinterpret_cast<int32_t *>(sc + NA_OVF);
        int2 *deep = reinterpret_cast<int2 *>(sc + NA_DEEP);
        // the previous call's contents stay in the array: zero the control
        // block and rebuild the pair table (kernels, no memset)
        k_ctl_init<<<1, 256, 0, s>>>(ctl);
        k_pairs_init<<<1, 64, 0, s>>>(pc, pv, B->pairs.as<BvhPair>(), 1);
        const WideNode *top = B->npairs == 1 && !B->hpairs.empty() && B->hpairs[0].root >= 0
                                  ? B->top.as<WideNode>()
                                  : nullptr;
        const QueryCfg cfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 0, top};
        auto go = [&](auto tag) {
            using T = decltype(tag);
            const QueryOut<T> qo = carve_qout<T>(sc + NA_Q, nP);
            QueryIn<T> qi{};
            qi.mode = Q_POINTS;
            qi.npairs = 1;
            qi.P = P;
            qi.pc = pc;
            BView<T> bv;
            if constexpr (sizeof(T) == 4) bv = BView<float>{B->frames32.as<float4>()};
            else bv = BView<double>{B->frames64.as<double2>()};
            launch_query<T>(0, nP, lanes == 4 ? INT64_MAX : -1, qi, host_count(nP), cfg, bv, qo, pc, pv, ctl, ovf,
                            deep, s);
            k_export_points<T><<<grid_for(nP, BLK), BLK, 0, s>>>(qo, nP, B->ids.as<int4>(), pc, d, I, Q, ctl, err);
            HD_LAUNCH_CHECK();
        };
        if (precision == HD_PREC_FP64) go(double{});
        else go(float{});
        return HD_OK;
    });
}

hd_status hd_eval_bounds(const double *v, const double *dd, const int32_t *I, const double *q, int64_t n, hd_bvh Bh,
                         int32_t precision, double *out, int32_t *u3_case, hd_stream_t stream) {
    if (!Bh || n < 0 || (n > 0 && (!v || !dd || !I || !q || !out || !u3_case))) return HD_E_INVALID;
    if (n == 0) return HD_OK;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard([&] {
        DBuf inv, pcb, pvb;
        inv.reserve((size_t)B->nB * sizeof(int32_t));
        pcb.reserve(sizeof(PairConst));
        pvb.reserve(sizeof(PairVar));
        PairConst *pc = pcb.as<PairConst>();
        k_pairs_init<<<1, 64, 0, s>>>(pc, pvb.as<PairVar>(), B->pairs.as<BvhPair>(), 1);
        k_inv_perm<<<grid_for(B->nB, BLK), BLK, 0, s>>>(B->ids.as<int4>(), B->nB, inv.as<int32_t>());
        IdView iv{B->ids.as<int4>()};
        if (precision == HD_PREC_FP64)
            k_eval_bounds<double><<<grid_for(n, BLK), BLK, 0, s>>>(v, dd, I, q, n, inv.as<int32_t>(), B->nB,
                                                                   BView<double>{B->frames64.as<double2>()}, iv, pc,
                                                                   out, u3_case);
        else
            k_eval_bounds<float><<<grid_for(n, BLK), BLK, 0, s>>>(v, dd, I, q, n, inv.as<int32_t>(), B->nB,
                                                                  BView<float>{B->frames32.as<float4>()}, iv, pc,
                                                                  out, u3_case);
        HD_LAUNCH_CHECK();
        HD_HIP(hipStreamSynchronize(s));
        return HD_OK;
    });
}

hd_status hd_eval_bound_u5(const double *v, const double *dd, const int32_t *I, int64_t n, hd_bvh Bh,
                           int32_t precision, double *out, int32_t *Sb_out, hd_stream_t stream) {
    if (!Bh || n < 0 || (n > 0 && (!v || !dd || !I || !out || !Sb_out))) return HD_E_INVALID;
    if (n == 0) return HD_OK;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard([&] {
        DBuf inv, ctlb, pcb, pvb, ovf, deep, P;
        inv.reserve((size_t)B->nB * sizeof(int32_t));
        ctlb.reserve(sizeof(Ctl));
        pcb.reserve(sizeof(PairConst));
        pvb.reserve(sizeof(PairVar));
        ovf.reserve((size_t)n * sizeof(int32_t));
        deep.reserve((size_t)DEEP_SLOTS * DEEP_STACK * sizeof(int2));
        P.reserve((size_t)n * 3 * sizeof(double));
        Ctl *ctl = ctlb.as<Ctl>();
        PairConst *pc = pcb.as<PairConst>();
        PairVar *pv = pvb.as<PairVar>();
        k_ctl_init<<<1, 256, 0, s>>>(ctl);
        k_pairs_init<<<1, 64, 0, s>>>(pc, pv, B->pairs.as<BvhPair>(), 1);
        k_inv_perm<<<grid_for(B->nB, BLK), BLK, 0, s>>>(B->ids.as<int4>(), B->nB, inv.as<int32_t>());
        k_barycenters<<<grid_for(n, BLK), BLK, 0, s>>>(v, n, P.as<double>());
        const QueryCfg cfg{B->nodes.as<WideNode>(), B->ids.as<int4>(), 0, nullptr};
        auto go = [&](auto tag) {
            using T = decltype(tag);
            QBuf<T> qb;
            qb.ensure(n);
            QueryIn<T> qi{};
            qi.mode = Q_POINTS;
            qi.npairs = 1;
            qi.P = P.as<double>();
            qi.pc = pc;
            BView<T> bv;
            if constexpr (sizeof(T) == 4) bv = BView<float>{B->frames32.as<float4>()};
            else bv = BView<double>{B->frames64.as<double2>()};
            launch_query<T>(0, n, -1, qi, host_count(n), cfg, bv, qb.o, pc, pv, ctl, ovf.as<int32_t>(),
                            deep.as<int2>(), s);
            k_eval_u5<T><<<grid_for(n, BLK), BLK, 0, s>>>(v, dd, I, n, inv.as<int32_t>(), B->nB, qb.o.I, bv,
                                                          B->ids.as<int4>(), pc, out, Sb_out);
            HD_LAUNCH_CHECK();
            HD_HIP(hipStreamSynchronize(s));
        };
        if (precision == HD_PREC_FP64) go(double{});
        else go(float{});
        return HD_OK;
    });
}

hd_status hd_frontier_features(const double *v, const double *dd, const int32_t *I, const double *q, int64_t n,
                               hd_bvh Bh, double L, double dA, float *X, hd_stream_t stream) {
    if (!Bh || n < 0 || (n > 0 && (!v || !dd || !I || !q || !X)) || !(dA > 0)) return HD_E_INVALID;
    if (n == 0) return HD_OK;
    const Bvh *B = reinterpret_cast<const Bvh *>(Bh);
    hipStream_t s = (hipStream_t)stream;
    return guard([&] {
        DBuf inv, pcb, pvb;
        inv.reserve((size_t)B->nB * sizeof(int32_t));
        pcb.reserve(sizeof(PairConst));
        pvb.reserve(sizeof(PairVar));
        PairConst *pc = pcb.as<PairConst>();
        k_pairs_init<<<1, 64, 0, s>>>(pc, pvb.as<PairVar>(), B->pairs.as<BvhPair>(), 1);
        k_inv_perm<<<grid_for(B->nB, BLK), BLK, 0, s>>>(B->ids.as<int4>(), B->nB, inv.as<int32_t>());
        k_tri_features<float><<<grid_for(n, BLK), BLK, 0, s>>>(v, dd, I, q, n, inv.as<int32_t>(), B->nB,
                                                               BView<float>{B->frames32.as<float4>()},
                                                               IdView{B->ids.as<int4>()}, pc, L, dA, X);
        HD_LAUNCH_CHECK();
        HD_HIP(hipStreamSynchronize(s));
        return HD_OK;
    });
}

} // extern "C"
