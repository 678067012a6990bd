// hd_prims.hip -- device-wide exclusive scan and stable LSD radix sort,
// written for wave64: lane prefixes from ballot/popcount and 64-lane shuffles,
// block results combined in LDS.
#include "hd_internal.hpp"

namespace hd {

namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// inclusive scan across the 64 lanes of a wave
__device__ __forceinline__ int wave_inclusive_scan(int v) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int t = __shfl_up(v, o, 64);
        if ((int)__lane_id() >= o) v += t;
    }
    return v;
}

// exclusive scan across a block of SCAN_BLOCK threads; returns the block total
__device__ __forceinline__ int block_exclusive_scan(int v, int *total) {
    __shared__ int wsum[SCAN_BLOCK / 64];
    int inc = wave_inclusive_scan(v);
    int w = threadIdx.x >> 6;
    if (__lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < SCAN_BLOCK / 64; ++i) {
        if (i < w) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ void k_scan_reduce(const int32_t *__restrict__ in, int64_t n, int32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) s += in[base + i];
    int tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// single block: exclusive scan of the per-tile partial sums, in place
__global__ void k_scan_partials(int32_t *part, int64_t n, int32_t *d_total) {
    int carry = 0;
    for (int64_t b = 0; b < n; b += SCAN_BLOCK) {
        int64_t i = b + threadIdx.x;
        int v = i < n ? part[i] : 0;
        int tot;
        int ex = block_exclusive_scan(v, &tot);
        if (i < n) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && d_total) *d_total = carry;
}

__global__ void k_scan_down(const int32_t *__restrict__ in, int32_t *__restrict__ out, int64_t n,
                            const int32_t *__restrict__ part) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int tot;
    int ex = block_exclusive_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) out[base + i] = ex;
        ex += v[i];
    }
}

__global__ void k_zero_i32(int32_t *p) { *p = 0; }

// Exclusive scan of a short array (n <= SMALL_SCAN_MAX, 16-byte aligned) in
// one block of SMALL_SCAN_BLOCK threads. The array is cut into tiles of
// SMALL_SCAN_BLOCK x 4 values; thread t loads values 4t..4t+3 of every tile
// (one coalesced 16-byte load per tile, all in flight at once) and keeps only
// their sums. Each wave scans its sums per tile; one wave then scans the
// 16 x 16 wave totals in (tile, wave) order, which is the order of the values,
// so every thread finds its offset in one LDS read per tile; it then reads
// its four values again (from the L2) to write their offsets. One launch
// instead of three, up to 64 Ki values (the digit table of a radix sort of
// 800 k keys).
constexpr int SMALL_SCAN_BLOCK = 1024;
constexpr int SMALL_SCAN_TILES = 16;
constexpr int64_t SMALL_SCAN_TILE = (int64_t)SMALL_SCAN_BLOCK * 4;
constexpr int64_t SMALL_SCAN_MAX = SMALL_SCAN_TILE * SMALL_SCAN_TILES;
__device__ __forceinline__ int4 load4_tail(const int32_t *__restrict__ in, int i, int n) {
    if (i + 3 < n) return *reinterpret_cast<const int4 *>(in + i);
    int4 v;
    v.x = i < n ? in[i] : 0;
    v.y = i + 1 < n ? in[i + 1] : 0;
    v.z = i + 2 < n ? in[i + 2] : 0;
    v.w = 0;
    return v;
}
__global__ __launch_bounds__(SMALL_SCAN_BLOCK) void k_scan_small(const int32_t *in, int32_t *out, int64_t n,
                                                                 int32_t *d_total) {
    constexpr int NW = SMALL_SCAN_BLOCK / 64;
    static_assert(SMALL_SCAN_TILES * NW == 4 * 64, "one wave scans the wave totals, four per lane");
    __shared__ int wsum[SMALL_SCAN_TILES][NW]; // wave totals, then their exclusive prefix
    __shared__ int s_total;
    const int w = threadIdx.x >> 6;
    const int m = (int)n; // n <= SMALL_SCAN_MAX
    int exc[SMALL_SCAN_TILES]; // the thread's exclusive offset inside its wave, per tile
#pragma unroll
    for (int k = 0; k < SMALL_SCAN_TILES; ++k) {
        const int4 v = load4_tail(in, k * (int)SMALL_SCAN_TILE + 4 * (int)threadIdx.x, m);
        exc[k] = v.x + v.y + v.z + v.w;
    }
#pragma unroll
    for (int k = 0; k < SMALL_SCAN_TILES; ++k) {
        const int inc = wave_inclusive_scan(exc[k]);
        if (__lane_id() == 63) wsum[k][w] = inc;
        exc[k] = inc - exc[k];
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        int *flat = &wsum[0][0];
        const int l = threadIdx.x;
        const int t0 = flat[4 * l], t1 = flat[4 * l + 1], t2 = flat[4 * l + 2], t3 = flat[4 * l + 3];
        const int tot = t0 + t1 + t2 + t3;
        const int inc = wave_inclusive_scan(tot);
        const int ex = inc - tot;
        flat[4 * l] = ex;
        flat[4 * l + 1] = ex + t0;
        flat[4 * l + 2] = ex + t0 + t1;
        flat[4 * l + 3] = ex + t0 + t1 + t2;
        if (l == 63) s_total = inc;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < SMALL_SCAN_TILES; ++k) {
        const int i = k * (int)SMALL_SCAN_TILE + 4 * (int)threadIdx.x;
        const int4 v = load4_tail(in, i, m);
        int4 o;
        o.x = wsum[k][w] + exc[k];
        o.y = o.x + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        if (i + 3 < m) {
            *reinterpret_cast<int4 *>(out + i) = o;
        } else {
            if (i < m) out[i] = o.x;
            if (i + 1 < m) out[i + 1] = o.y;
            if (i + 2 < m) out[i + 2] = o.z;
        }
    }
    if (threadIdx.x == 0 && d_total) *d_total = s_total;
}

inline bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

// ---------------------------------------------------------------------------
// radix sort: 8-bit digits, one tile of RS_BLOCK * items keys per block
// (items: RS_ITEMS_MAX for long arrays; fewer for short ones, so that they
// still spread over many blocks, each with a short serial loop)
// ---------------------------------------------------------------------------
constexpr int RS_BLOCK = 256;
constexpr int RS_ITEMS_MAX = 16;
constexpr int RS_WAVES = RS_BLOCK / 64;

// digit counts of each block's tile: hist[d * nblocks + b] (digit-major, for
// the device-wide scan), or hist[b * 256 + d] when block_major (for the
// scatter that derives its own offsets)
template <class K>
__global__ void k_radix_hist(const K *__restrict__ keys, int64_t n, int shift, int nblocks, int items,
                             int block_major, int32_t *__restrict__ hist) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RS_BLOCK * items;
    for (int r = 0; r < items; ++r) {
        int64_t i = base + (int64_t)r * RS_BLOCK + threadIdx.x;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[block_major ? (int64_t)blockIdx.x * 256 + threadIdx.x : (int64_t)threadIdx.x * nblocks + blockIdx.x] =
        h[threadIdx.x];
}

// Offset of digit d (= thread) for this block, from the block-major counts
// of all nblocks blocks: the count of smaller digits in all blocks plus the
// count of digit d in earlier blocks. Every block reads the whole table
// (nblocks x 1 KB, coalesced), which replaces a separate scan launch when
// the table is small.
__device__ int radix_block_offset(const int32_t *__restrict__ hist, int nblocks) {
    static_assert(RS_BLOCK == 256, "one thread per digit");
    const int d = threadIdx.x;
    // rows in batches of 32 loads in flight (the table was written by blocks
    // on every XCD, so each load has the latency of memory beyond L2)
    constexpr int RB = 32;
    int total = 0, before = 0;
    for (int b0 = 0; b0 < nblocks; b0 += RB) {
        int hv[RB];
#pragma unroll
        for (int k = 0; k < RB; ++k) hv[k] = b0 + k < nblocks ? hist[(int64_t)(b0 + k) * 256 + d] : 0;
#pragma unroll
        for (int k = 0; k < RB; ++k) {
            total += hv[k];
            before += b0 + k < (int)blockIdx.x ? hv[k] : 0;
        }
    }
    // exclusive scan of the totals over the 256 digits
    __shared__ int wsum[RS_WAVES];
    const int inc = wave_inclusive_scan(total);
    const int w = d >> 6;
    if (__lane_id() == 63) wsum[w] = inc;
    __syncthreads();
    int off = 0;
#pragma unroll
    for (int i = 0; i < RS_WAVES; ++i)
        if (i < w) off += wsum[i];
    return off + inc - total + before;
}

// Stable scatter: within a round of RS_BLOCK keys, a key's rank among equal
// digits of its wave comes from eight ballots (one per digit bit); waves are
// then ordered through per-digit counters in LDS. The block's digit offsets
// come from offs (digit-major, scanned), or, with offs null, from the
// block-major counts in hist.
template <class K>
__global__ void k_radix_scatter(const K *__restrict__ kin, const int32_t *__restrict__ vin, K *__restrict__ kout,
                                int32_t *__restrict__ vout, int64_t n, int shift, int nblocks, int items,
                                const int32_t *__restrict__ offs, const int32_t *__restrict__ hist) {
    __shared__ int goff[256];
    __shared__ int wcnt[RS_WAVES][256];
    __shared__ int woff[RS_WAVES][256];
    goff[threadIdx.x] = offs ? offs[(int64_t)threadIdx.x * nblocks + blockIdx.x] : radix_block_offset(hist, nblocks);
    const int w = threadIdx.x >> 6;
    const int lane = __lane_id();
    const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    int64_t base = (int64_t)blockIdx.x * RS_BLOCK * items;
    for (int r = 0; r < items; ++r) {
        for (int k = 0; k < RS_WAVES; ++k) wcnt[k][threadIdx.x] = 0;
        __syncthreads();
        int64_t i = base + (int64_t)r * RS_BLOCK + threadIdx.x;
        bool act = i < n;
        K key = act ? kin[i] : K(0);
        int32_t val = act ? vin[i] : 0;
        uint32_t dg = (uint32_t)(key >> shift) & 255u;
        unsigned long long peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            unsigned long long m = __ballot((dg >> b) & 1u);
            peers &= ((dg >> b) & 1u) ? m : ~m;
        }
        int rank = __popcll(peers & lt);
        if (act && rank == 0) wcnt[w][dg] = __popcll(peers);
        __syncthreads();
        {
            int d = threadIdx.x;
            int run = goff[d];
            for (int k = 0; k < RS_WAVES; ++k) {
                woff[k][d] = run;
                run += wcnt[k][d];
            }
            goff[d] = run;
        }
        __syncthreads();
        if (act) {
            int64_t o = woff[w][dg] + rank;
            kout[o] = key;
            vout[o] = val;
        }
        __syncthreads();
    }
}

// launch plan of a radix sort of n keys: the fewest items per block that
// keep the digit histogram small (at most RS_FUSED_MAX blocks x 256 digits:
// then each scatter block derives its own offsets), at most RS_ITEMS_MAX
constexpr int RS_FUSED_MAX = 128;
struct RadixPlan {
    int items, nb;
    int64_t hn, scan_parts;
    explicit RadixPlan(int64_t n) {
        items = (int)std::min<int64_t>(
            RS_ITEMS_MAX, std::max<int64_t>(1, (n + RS_FUSED_MAX * RS_BLOCK - 1) / (RS_FUSED_MAX * RS_BLOCK)));
        const int64_t tile = (int64_t)RS_BLOCK * items;
        nb = (int)((n + tile - 1) / tile);
        hn = 256LL * nb;
        scan_parts = (hn + SCAN_TILE - 1) / SCAN_TILE;
    }
    size_t tmp_bytes() const { return (size_t)(2 * hn + scan_parts + 64) * sizeof(int32_t); }
};

template <class K>
void radix_sort_impl(K *keys, int32_t *vals, K *keys_alt, int32_t *vals_alt, int64_t n, int bits, DBuf &tmp,
                     hipStream_t s) {
    if (n <= 1) return;
    const RadixPlan rp(n);
    const int items = rp.items, nb = rp.nb;
    const int64_t hn = rp.hn, scan_parts = rp.scan_parts;
    tmp.reserve(rp.tmp_bytes());
    int32_t *hist = tmp.as<int32_t>();
    int32_t *offs = hist + hn;
    int32_t *part = offs + hn;
    K *ka = keys, *kb = keys_alt;
    int32_t *va = vals, *vb = vals_alt;
    int passes = (bits + 7) / 8;
    const bool fused = nb <= RS_FUSED_MAX;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        k_radix_hist<K><<<nb, RS_BLOCK, 0, s>>>(ka, n, shift, nb, items, fused ? 1 : 0, hist);
        if (fused) {
            k_radix_scatter<K><<<nb, RS_BLOCK, 0, s>>>(ka, va, kb, vb, n, shift, nb, items, nullptr, hist);
            HD_LAUNCH_CHECK();
            std::swap(ka, kb);
            std::swap(va, vb);
            continue;
        }
        if (hn <= SMALL_SCAN_MAX && aligned16(hist) && aligned16(offs)) {
            k_scan_small<<<1, SMALL_SCAN_BLOCK, 0, s>>>(hist, offs, hn, nullptr);
        } else {
            k_scan_reduce<<<(unsigned)scan_parts, SCAN_BLOCK, 0, s>>>(hist, hn, part);
            k_scan_partials<<<1, SCAN_BLOCK, 0, s>>>(part, scan_parts, nullptr);
            k_scan_down<<<(unsigned)scan_parts, SCAN_BLOCK, 0, s>>>(hist, offs, hn, part);
        }
        k_radix_scatter<K><<<nb, RS_BLOCK, 0, s>>>(ka, va, kb, vb, n, shift, nb, items, offs, nullptr);
        HD_LAUNCH_CHECK();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        HD_HIP(hipMemcpyAsync(keys, ka, n * sizeof(K), hipMemcpyDeviceToDevice, s));
        HD_HIP(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
}

__global__ __launch_bounds__(256) void k_export(Export e, unsigned *seq_dev, unsigned seq) {
    for (int r = 0; r < e.n; ++r) {
        const uint32_t *src = (const uint32_t *)e.src[r];
        uint32_t *dst = (uint32_t *)e.dst[r];
        const int64_t w = e.bytes[r] / 4;
        for (int64_t i = threadIdx.x; i < w; i += blockDim.x) dst[i] = src[i];
    }
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0) __hip_atomic_store(seq_dev, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

} // namespace

void export_to_host(const Export &e, unsigned *seq_dev, unsigned seq, hipStream_t s) {
    k_export<<<1, 256, 0, s>>>(e, seq_dev, seq);
    HD_LAUNCH_CHECK();
}

void wait_host_seq(const unsigned *seq_host, unsigned seq, hipStream_t s) {
    for (unsigned long it = 1;; ++it) {
        if (__atomic_load_n(seq_host, __ATOMIC_ACQUIRE) == seq) return;
        if ((it & 4095) == 0) {
            hipError_t e = hipStreamQuery(s);
            if (e != hipSuccess && e != hipErrorNotReady) throw Error{HD_E_DEVICE, hipGetErrorString(e)};
            if (e == hipSuccess) {
                __atomic_thread_fence(__ATOMIC_SEQ_CST);
                if (__atomic_load_n(seq_host, __ATOMIC_ACQUIRE) == seq) return;
                throw Error{HD_E_INTERNAL, "device report not visible after the stream drained"};
            }
        }
        __builtin_ia32_pause();
    }
}

size_t radix_sort_tmp_bytes(int64_t n) { return n <= 1 ? 0 : RadixPlan(n).tmp_bytes(); }

void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *d_total, DBuf &tmp,
                        hipStream_t s) {
    if (n <= 0) {
        if (d_total) k_zero_i32<<<1, 1, 0, s>>>(d_total);
        return;
    }
    if (n <= SMALL_SCAN_MAX && aligned16(in) && aligned16(out)) {
        k_scan_small<<<1, SMALL_SCAN_BLOCK, 0, s>>>(in, out, n, d_total);
        HD_LAUNCH_CHECK();
        return;
    }
    int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    tmp.reserve(nb * sizeof(int32_t));
    int32_t *part = tmp.as<int32_t>();
    k_scan_reduce<<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, n, part);
    k_scan_partials<<<1, SCAN_BLOCK, 0, s>>>(part, nb, d_total);
    k_scan_down<<<(unsigned)nb, SCAN_BLOCK, 0, s>>>(in, out, n, part);
    HD_LAUNCH_CHECK();
}

void radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt, int64_t n, int bits,
                    DBuf &tmp, hipStream_t s) {
    radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s);
}

void radix_sort_u64(unsigned long long *keys, int32_t *vals, unsigned long long *keys_alt, int32_t *vals_alt,
                    int64_t n, int bits, DBuf &tmp, hipStream_t s) {
    radix_sort_impl<unsigned long long>(keys, vals, keys_alt, vals_alt, n, bits, tmp, s);
}

} // namespace hd
