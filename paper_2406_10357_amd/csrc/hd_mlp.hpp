// hd_mlp.hpp -- device pieces of the learned proposal's network shared by the
// network's own kernels and the engine's cascade kernels: parameter layout,
// BF16 weights in LDS, and the forward pass of a 16-row tile on the matrix
// cores (v_mfma_f32_16x16x16_bf16).
//
// Operand layouts of the 16x16x16 MFMA (lane l, g = l / 16, c = l % 16): A
// holds A[c][4g + j], B holds B[4g + j][c], the result holds D[4g + j][c],
// j = 0..3. A layer's result (rows by lane group) feeds the next layer's A
// operand (rows by lane) through a per-wave LDS tile.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {
namespace mlp {

constexpr int NIN = 16, NH = 64;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH, NPARAM = OFF_B3 + 1;
constexpr int MBLK = 256, MWAVES = MBLK / 64;
static_assert(NPARAM == 5313, "16-64-64-1 network");

typedef short v4s __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// round to nearest even BF16 (bit pattern)
__device__ __forceinline__ unsigned short to_bf16(float x) {
    unsigned u = __builtin_bit_cast(unsigned, x);
    u = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
    return __builtin_bit_cast(float, (unsigned)h << 16);
}
__device__ __forceinline__ v4s pack4(unsigned short a, unsigned short b, unsigned short c, unsigned short d) {
    v4s r;
    r.x = (short)a;
    r.y = (short)b;
    r.z = (short)c;
    r.w = (short)d;
    return r;
}
__device__ __forceinline__ v4s pack4f(float a, float b, float c, float d) {
    return pack4(to_bf16(a), to_bf16(b), to_bf16(c), to_bf16(d));
}
__device__ __forceinline__ v4f mfma(v4s a, v4s b, v4f c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// BF16 weights in the layouts the operands read with one 8-byte access:
// w1t[o][k] and w2t[o][k] (output-major) for the forward B operands, w2[k][o]
// (input-major) for the backward product dZ2 * W2^T.
struct alignas(16) Weights {
    alignas(16) unsigned short w1t[NH * NIN];
    alignas(16) unsigned short w2t[NH * NH];
    alignas(16) unsigned short w2[NH * NH];
    float w3[NH]; // BF16-rounded values, kept as float for the dot product
    float b1[NH], b2[NH], b3;
};

// the BF16 forms of parameter i (value x); called by its owner
__device__ inline void set_param(Weights &W, int i, float x) {
    if (i < OFF_B1) {
        int k = i / NH, o = i % NH;
        W.w1t[o * NIN + k] = to_bf16(x);
    } else if (i < OFF_W2) {
        W.b1[i - OFF_B1] = x;
    } else if (i < OFF_B2) {
        int j = i - OFF_W2, k = j / NH, o = j % NH;
        unsigned short h = to_bf16(x);
        W.w2t[o * NH + k] = h;
        W.w2[k * NH + o] = h;
    } else if (i < OFF_W3) {
        W.b2[i - OFF_B2] = x;
    } else if (i < OFF_B3) {
        W.w3[i - OFF_W3] = from_bf16(to_bf16(x));
    } else {
        W.b3 = x;
    }
}

// Activations of one tile, in result layout (rows 4g + j, column 16c + lane%16).
struct Tile {
    v4f z1[4], z2[4];
    float y[4]; // output of rows 4g + j (same in all lanes of group g)
};

// Forward pass of rows r0 .. r0+15 (rows >= n are zero inputs). s1 is the
// wave's 16 x 64 BF16 staging tile.
__device__ inline void tile_forward(const float *__restrict__ X, const int32_t *rows, int64_t r0, int64_t n,
                             const Weights &W, unsigned short *s1, Tile &T) {
    const int l = __lane_id(), g = l >> 4, c = l & 15;
    // A operand of layer 1: X[row c][4g .. 4g+3]
    v4s a1 = pack4(0, 0, 0, 0);
    {
        int64_t r = r0 + c;
        if (r < n) {
            int64_t src = rows ? rows[r] : r;
            const float4 x = *reinterpret_cast<const float4 *>(X + src * NIN + 4 * g);
            a1 = pack4f(x.x, x.y, x.z, x.w);
        }
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int o = 16 * cb + c;
        const v4s b = *reinterpret_cast<const v4s *>(&W.w1t[o * NIN + 4 * g]);
        v4f z = mfma(a1, b, v4f{0.f, 0.f, 0.f, 0.f});
        const float bias = W.b1[o];
        z += bias;
        T.z1[cb] = z;
        // H1 (BF16) into the staging tile: row 4g + j, column o
#pragma unroll
        for (int j = 0; j < 4; ++j) s1[(4 * g + j) * NH + o] = to_bf16(fmaxf(z[j], 0.f));
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    v4s a2[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) a2[kb] = *reinterpret_cast<const v4s *>(&s1[c * NH + 16 * kb + 4 * g]);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int o = 16 * cb + c;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const v4s b = *reinterpret_cast<const v4s *>(&W.w2t[o * NH + 16 * kb + 4 * g]);
            acc = mfma(a2[kb], b, acc);
        }
        acc += W.b2[o];
        T.z2[cb] = acc;
        const float w = W.w3[o];
#pragma unroll
        for (int j = 0; j < 4; ++j) part[j] += fmaxf(acc[j], 0.f) * w;
    }
    // sum over the 16 columns held by the lanes of a group
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        float v = part[j];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        T.y[j] = v + W.b3;
    }
    __builtin_amdgcn_wave_barrier();
}


} // namespace mlp
} // namespace hd
