// hd_reduce.hpp -- per-pair min/max reductions over a workgroup.
//
// Device-scope atomics on one address serialise at the memory side (about
// 10 ns each on a multi-XCD part), so a kernel where every thread folds a
// value into its pair's slot would spend its time in atomics. Here a block
// reduces in registers and LDS first: one atomic per value per block when the
// whole block belongs to one pair (the common case, since a pair's elements
// are contiguous), one per wave when a block straddles pairs, one per lane
// only in a wave that itself mixes pairs.
#pragma once
#include "hd_math.hpp"

namespace hd {

// Accumulators that every block of a large grid updates are kept in
// ACC_COPIES copies, 256 bytes apart, block b updating copy b % ACC_COPIES:
// atomics on one 256-byte region serialise at the memory side, so sixteen
// copies take sixteen times the rate. Whoever reads the value folds the copies.
constexpr int ACC_COPIES = 16;
__device__ __forceinline__ int acc_copy() { return (int)(blockIdx.x & (ACC_COPIES - 1)); }

// Fold ordered bits x into *a with max (mx) or min, for the paths where
// several pairs share a wave or a block: there every lane or wave has an
// atomic of its own, and a batch of pairs can queue thousands of them on one
// pair's line. The slot only moves one way while a launch runs, so an atomic
// that cannot change it is skipped: a plain read (possibly an older copy in
// this XCD's L2, never past the current value) decides. (The one atomic of a
// block that holds a single pair is left as it is: there the read only
// lengthens the path.)
__device__ __forceinline__ void fold_ord(unsigned long long *a, unsigned long long x, bool mx) {
    const unsigned long long cur = __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (mx ? x > cur : x < cur) {
        if (mx) atomicMax(a, x);
        else atomicMin(a, x);
    }
}

// v[k] is reduced with max when bit k of MAXMASK is set, else with min.
// Threads with valid == false must pass neutral values (+inf for min, -inf
// for max, or anything with valid == false: they are masked out). addr(p, k)
// returns the ordered-bits slot of value k of pair p. Every thread of the
// block must call this (it contains barriers).
template <int K, unsigned MAXMASK, int BLOCK, class Addr>
__device__ __forceinline__ void block_pair_minmax(int p, bool valid, const double (&v)[K], Addr addr) {
    constexpr int NW = BLOCK / 64;
    __shared__ double sv[NW][K];
    __shared__ int sp[NW];
    const int w = threadIdx.x >> 6, lane = __lane_id();
    const unsigned long long vm = __ballot(valid);
    int p0 = vm ? __shfl(p, __ffsll(vm) - 1, 64) : -1;
    const bool wave_uni = __ballot(valid && p != p0) == 0;
    double r[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const bool mx = (MAXMASK >> k) & 1u;
        double x = valid ? v[k] : (mx ? -__builtin_inf() : __builtin_inf());
        if (wave_uni) {
            for (int o = 32; o >= 1; o >>= 1) {
                double y = __shfl_xor(x, o, 64);
                x = mx ? fmax(x, y) : fmin(x, y);
            }
        } else if (valid) {
            fold_ord(addr(p, k), d2ord(x), mx);
        }
        r[k] = x;
    }
    if (lane == 0) {
        sp[w] = (vm && wave_uni) ? p0 : -1;
#pragma unroll
        for (int k = 0; k < K; ++k) sv[w][k] = r[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int q = -1;
        bool uni = true;
        for (int i = 0; i < NW; ++i) {
            if (sp[i] < 0) continue;
            if (q < 0) q = sp[i];
            else if (sp[i] != q) uni = false;
        }
        if (q >= 0 && uni) {
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const bool mx = (MAXMASK >> k) & 1u;
                double x = mx ? -__builtin_inf() : __builtin_inf();
                for (int i = 0; i < NW; ++i)
                    if (sp[i] >= 0) x = mx ? fmax(x, sv[i][k]) : fmin(x, sv[i][k]);
                unsigned long long *a = addr(q, k);
                if (mx) atomicMax(a, d2ord(x));
                else atomicMin(a, d2ord(x));
            }
        } else if (q >= 0) {
            for (int i = 0; i < NW; ++i) {
                if (sp[i] < 0) continue;
#pragma unroll
                for (int k = 0; k < K; ++k) fold_ord(addr(sp[i], k), d2ord(sv[i][k]), (MAXMASK >> k) & 1u);
            }
        }
    }
    __syncthreads();
}

// Statistics counters: the block sums v[k] (wave shuffles, then LDS) and one
// thread adds each nonzero sum to *dst[k]. Every thread of the block must call
// this (it contains barriers).
template <int N, int BLOCK>
__device__ __forceinline__ void block_add(const unsigned long long (&v)[N], unsigned long long *const (&dst)[N]) {
    __shared__ unsigned long long s[N];
    if (threadIdx.x < N) s[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
        unsigned long long x = v[k];
        for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
        if (__lane_id() == 0 && x) atomicAdd(&s[k], x);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (threadIdx.x == k && s[k]) atomicAdd(dst[k], s[k]);
}

} // namespace hd
