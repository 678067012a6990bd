// hd_internal.hpp -- host-side declarations shared by the library's
// translation units: the BVH handle, device-buffer helpers, error handling
// and the data-parallel primitives (scan, radix sort).
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
            throw Error{HD_E_NOMEM, "hipMalloc of " + std::to_string(b) + " bytes failed"};
        }
        bytes = b;
    }
    template <class X> X *as() const { return static_cast<X *>(p); }
};

// Device-resident BVH over soup B with everything the queries and the
// bounds need. Arrays indexed by "sorted index" follow the Morton order of
// the leaves.
struct Bvh {
    int device = 0;
    int64_t nB = 0, mB = 0;
    double center[3] = {0, 0, 0}; // subtracted from every coordinate (A's too)
    double coord_max = 0;         // max |coordinate| of B after centering
    double edge_max = 0;          // longest edge of any B triangle
    DBuf nodes;                   // (nB-1 or 1) x 64 B: child boxes + child refs
    DBuf frames32;                // nB x 64 B
    DBuf frames64;                // nB x 128 B
    DBuf ids;                     // nB x int4: corner vertex ids (frame order), original face id
    DBuf scratch;                 // build temporaries
    float ms_build = 0;
};

// --- primitives (hd_prims.hip) -------------------------------------------
// Exclusive scan of n int32 values in place-out; returns nothing; total in
// *d_total (device, may be null).
void scan_exclusive_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *d_total, DBuf &tmp,
                        hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys. Results land in keys/vals (the alt buffers are scratch).
void radix_sort_u32(uint32_t *keys, int32_t *vals, uint32_t *keys_alt, int32_t *vals_alt, int64_t n,
                    int bits, DBuf &tmp, hipStream_t s);

// --- BVH (hd_bvh.hip) ------------------------------------------------------
Bvh *build_bvh(const double *VB, int64_t mB, const int32_t *FB, int64_t nB, hipStream_t s);

// Node record: a = (lo_L.xyz, child_L), b = (hi_L.xyz, child_R),
// c = (lo_R.xyz, 0), d = (hi_R.xyz, 0). A child >= 0 is an internal node,
// a child < 0 the leaf ~child (sorted triangle index).
struct NodeRec {
    float4 a, b, c, d;
};

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

} // namespace hd
