// hd_internal.hpp -- host-side declarations shared by the library's
// translation units: the (multi-pair) BVH handle, device-buffer helpers,
// error handling and the data-parallel primitives (scan, radix sort).
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

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
    DBuf nodes;    // internal nodes x 64 B: child boxes + child refs
    DBuf frames32; // nB x 64 B
    DBuf frames64; // nB x 128 B
    DBuf ids;      // nB x int4: corner vertex ids (frame order), original face index in its pair
    DBuf pairs;    // npairs x BvhPair
    std::vector<BvhPair> hpairs;
    float ms_build = 0;
};

// --- primitives (hd_prims.hip) -------------------------------------------
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

// Node record: a = (lo_L.xyz, child_L), b = (hi_L.xyz, child_R),
// c = (lo_R.xyz, 0), d = (hi_R.xyz, 0). A child >= 0 is an internal node,
// a child < 0 the leaf ~child (sorted triangle index).
struct NodeRec {
    float4 a, b, c, d;
};

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

} // namespace hd
