// hd_internal.hpp -- host-side declarations shared by the library's
// translation units: the (multi-pair) BVH handle, device-buffer helpers,
// error handling and the data-parallel primitives (scan, radix sort).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <cstring>
#include <string>
#include <vector>

#include "../../include/hd.h"
#include "hd_math.hpp"

namespace hd {

// Thrown inside the library only; converted to hd_status at the ABI.
struct Error {
    hd_status st;
    std::string what;
};

#define HD_HIP(call)                                                                            \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            throw ::hd::Error{e_ == hipErrorOutOfMemory ? HD_E_NOMEM : HD_E_DEVICE,            \
                              std::string(#call) + ": " + hipGetErrorString(e_)};               \
    } while (0)

#define HD_LAUNCH_CHECK() HD_HIP(hipGetLastError())

// Owning device buffer (freed with hipFree on destruction).
struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // grow to at least n bytes (contents are not preserved)
    void reserve(size_t n) {
        if (n <= bytes) return;
        release();
        size_t b = n < 256 ? 256 : n;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw Error{HD_E_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
        }
        bytes = b;
    }
    void swap(DBuf &o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
    }
    template <class X> X *as() const { return static_cast<X *>(p); }
};

// Per-pair BVH facts (device array, host copy).
struct BvhPair {
    double ctr[3];        // centre subtracted from this pair's coordinates
    double coord_max;     // largest |coordinate| of the pair's B after centring
    double edge_max;      // longest edge of the pair's B triangles
    int64_t tri_begin;    // sorted-leaf range of the pair
    int64_t tri_end;
    int32_t root;         // >= 0 internal node, < 0 the single leaf ~root
    int32_t nB;
};

// Device-resident BVH over one or more soups B_p (one subtree per pair).
// Arrays indexed by "sorted index" follow the (pair, Morton) order.
struct Bvh {
    int device = 0;
    int npairs = 0;
    int64_t nB = 0;
    DBuf nodes;    // four-wide nodes x 128 B (at most nB - 1 of them)
    DBuf top;      // TOP_NODES x 128 B: the top levels of pair 0 (single-pair BVHs with an internal root)
    DBuf frames32; // nB x 64 B
    DBuf frames64; // nB x 128 B
    DBuf ids;      // nB x int4: corner vertex ids (frame order), original face index in its pair
    DBuf pairs;    // npairs x BvhPair
    std::vector<BvhPair> hpairs;
};

// Owning pinned host buffer (hipHostMalloc, mapped and coherent), used to
// stage small uploads and to receive results written by the device. Grows
// only; contents are not preserved on growth.
struct PinnedBuf {
    void *p = nullptr;
    void *dev = nullptr; // the same memory as seen by the device
    size_t bytes = 0;
    PinnedBuf() = default;
    PinnedBuf(const PinnedBuf &) = delete;
    PinnedBuf &operator=(const PinnedBuf &) = delete;
    ~PinnedBuf() {
        if (p) (void)hipHostFree(p);
    }
    void reserve(size_t n) {
        if (n <= bytes) return;
        if (p) (void)hipHostFree(p);
        p = dev = nullptr;
        bytes = 0;
        size_t b = n < 4096 ? 4096 : n;
        HD_HIP(hipHostMalloc(&p, b, hipHostMallocMapped | hipHostMallocCoherent));
        HD_HIP(hipHostGetDevicePointer(&dev, p, 0));
        bytes = b;
        std::memset(p, 0, b);
    }
    template <class X> X *as(size_t off = 0) const { return (X *)((char *)p + off); }
    template <class X> X *dev_as(size_t off = 0) const { return (X *)((char *)dev + off); }
};

// Device -> pinned host copy of up to four regions (sizes in bytes, multiples
// of 4), followed by a store of `seq` to *seq_dev that the host can poll: one
// kernel instead of staged copies and a stream synchronisation.
struct Export {
    const void *src[4];
    void *dst[4]; // device view of pinned memory
    int64_t bytes[4];
    int n;
};
void export_to_host(const Export &e, unsigned *seq_dev, unsigned seq, hipStream_t s);
// Wait until *seq_host == seq. Polls the pinned word; queries the stream now
// and then so that a failed launch or a device error ends the wait.
void wait_host_seq(const unsigned *seq_host, unsigned seq, hipStream_t s);

// --- learned proposal network (hd_mlp.hip) --------------------------------
hd_status mlp_forward(const float *X, int64_t n, const float *params, float *y, hipStream_t s);

// --- primitives (hd_prims.hip) -------------------------------------------
// Scratch bytes (the tmp buffer) the radix sort below needs for n values:
// reserved up front, it adds no allocation to a call.
size_t radix_sort_tmp_bytes(int64_t n);
// Exclusive scan of n int32 values; total in *d_total (device, may be null).
void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *d_total, DBuf &tmp,
                        hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys. Results land in keys/vals (the alt buffers are scratch).
void radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt, int64_t n,
                    int bits, DBuf &tmp, hipStream_t s);
void radix_sort_u64(unsigned long long *keys, int32_t *vals, unsigned long long *keys_alt, int32_t *vals_alt,
                    int64_t n, int bits, DBuf &tmp, hipStream_t s);

// --- BVH (hd_bvh.hip) ------------------------------------------------------
// VB[p], FB[p]: device pointers of pair p (host arrays of npairs pointers).
Bvh *build_bvh(int npairs, const double *const *VB, const int64_t *mB, const int32_t *const *FB,
               const int64_t *nB, hipStream_t s);
// Release a BVH (waits for the device; its buffers may serve a later build).
void recycle_bvh(Bvh *b);
// whether BVH builds are captured into (and replayed from) HIP graphs;
// returns the previous setting
int set_build_graphs(int enable);

// Four-wide BVH node, one 128-byte line: the boxes of up to four children
// (structure of arrays: component c of child k at lo*/hi*[k]) and their
// references. A reference >= 0 is a wide node, WIDE_EMPTY an unused slot, any
// other negative value the leaf ~ref (sorted triangle index).
constexpr int32_t WIDE_EMPTY = INT32_MIN;
struct alignas(128) WideNode {
    float4 lox, loy, loz, hix, hiy, hiz;
    int4 child;
    int4 meta; // (number of used slots, 0, 0, 0)
};
static_assert(sizeof(WideNode) == 128, "one cache line per node");
constexpr int WIDE_WORDS = 28; // the words a traversal reads (boxes and references)

// The top levels of a single-pair BVH (its root, the root's children and
// their children: at most 1 + 4 + 16 nodes), copied into a table that query
// kernels stage in LDS (the first WIDE_WORDS words of each): entry 0 the root, 1 + k its child slot k, 5 + 4k + m
// slot m of that child (entries for empty or leaf slots unused). Inside the
// table a child that is itself tabled is referenced as TOP_REF + its entry;
// other references are unchanged.
constexpr int TOP_NODES = 21;
constexpr int32_t TOP_REF = 1 << 30; // wide-node indices stay below it

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

} // namespace hd
