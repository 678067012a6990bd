// hd_mlp.hip -- the learned proposal's network on the matrix cores.
//
// 16 inputs -> 64 ReLU -> 64 ReLU -> 1. The two hidden layers are BF16 x BF16
// matrix products with FP32 accumulation (v_mfma_f32_16x16x16_bf16); the output
// layer is an FP32 dot product with BF16 weights. Parameters are an FP32
// vector (the master copy): W1 [16][64] input-major, b1 [64], W2 [64][64],
// b2 [64], w3 [64], b3.
//
// A wave works on tiles of 16 rows. Operand layouts of the 16x16x16 MFMA
// (lane l, g = l / 16, c = l % 16): A holds A[c][4g + j], B holds
// B[4g + j][c], the result holds D[4g + j][c], j = 0..3. A layer's result
// (rows by lane group) feeds the next layer's A operand (rows by lane)
// through a per-wave LDS tile; the weight gradients need no transpose: the
// result layout of a forward product is exactly the A or B layout of the
// backward product over the batch rows.
//
// Training runs in one workgroup of four waves: each step takes a minibatch
// (row indices given by the caller), accumulates the gradient in registers,
// folds it into LDS, and applies Adam (Kingma and Ba) to the FP32 master
// weights in global memory; every thread owns a fixed set of parameters, so
// the update needs no communication beyond the workgroup barrier.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "hd_internal.hpp"
#include "hd_mlp.hpp"

namespace hd {

namespace {

using namespace mlp;

// -------------------------------------------------------------------------
// inference
// -------------------------------------------------------------------------
__global__ __launch_bounds__(MBLK) void k_mlp_forward(const float *__restrict__ X, int64_t n,
                                                      const float *__restrict__ params, float *__restrict__ y) {
    __shared__ Weights W;
    __shared__ alignas(16) unsigned short stage[MWAVES][16 * NH];
    for (int i = threadIdx.x; i < NPARAM; i += MBLK) set_param(W, i, params[i]);
    __syncthreads();
    const int wave = threadIdx.x >> 6, l = __lane_id(), g = l >> 4, c = l & 15;
    const int64_t tiles = (n + 15) / 16;
    for (int64_t t = (int64_t)blockIdx.x * MWAVES + wave; t < tiles; t += (int64_t)gridDim.x * MWAVES) {
        Tile T;
        tile_forward(X, nullptr, 16 * t, n, W, stage[wave], T);
        if (c == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int64_t r = 16 * t + 4 * g + j;
                if (r < n) y[r] = T.y[j];
            }
        }
    }
}

// -------------------------------------------------------------------------
// training / gradient
// -------------------------------------------------------------------------
struct Grads {
    v4f w2[16]; // block (a, cb): hidden 16a + 4g + j, output 16cb + lane%16
    v4f w1[4];  // block cb: input 4g + j, hidden 16cb + lane%16
    float w3[4], b2[4], b1[4], b3; // per column 16cb + lane%16 (summed over rows later)
    float loss;
};

__device__ void zero(Grads &G) {
#pragma unroll
    for (int k = 0; k < 16; ++k) G.w2[k] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        G.w1[k] = v4f{0.f, 0.f, 0.f, 0.f};
        G.w3[k] = G.b2[k] = G.b1[k] = 0.f;
    }
    G.b3 = G.loss = 0.f;
}

// Gradient contribution of one tile to the loss sum_rows (y - t)^2 * scale.
__device__ void tile_backward(const float *__restrict__ X, const float *__restrict__ tgt, const int32_t *rows,
                              int64_t r0, int64_t n, float scale, const Weights &W, unsigned short *s1,
                              unsigned short *s2, Grads &G) {
    const int l = __lane_id(), g = l >> 4, c = l & 15;
    Tile T;
    tile_forward(X, rows, r0, n, W, s1, T);
    // dy of rows 4g + j (zero for rows past the end)
    float dy[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t r = r0 + 4 * g + j;
        float e = 0.f;
        if (r < n) e = T.y[j] - tgt[rows ? rows[r] : r];
        dy[j] = 2.f * e * scale;
        if (c == 0) G.loss += e * e * scale;
        if (c == 0) G.b3 += dy[j];
    }
    // output layer and dZ2 (result layout), staged as BF16 rows for dH1
    v4f dz2[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int o = 16 * cb + c;
        const float w = W.w3[o];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float h2 = fmaxf(T.z2[cb][j], 0.f);
            G.w3[cb] += h2 * dy[j];
            const float d = T.z2[cb][j] > 0.f ? dy[j] * w : 0.f;
            dz2[cb][j] = d;
            G.b2[cb] += d;
            s2[(4 * g + j) * NH + o] = to_bf16(d);
        }
    }
    // dW2[k][o] += sum_rows H1[row][k] dZ2[row][o]: A = H1^T (result layout
    // of layer 1, block a), B = dZ2 (result layout, block cb)
    v4s h1t[4], dz2b[4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
        h1t[a] = pack4f(fmaxf(T.z1[a][0], 0.f), fmaxf(T.z1[a][1], 0.f), fmaxf(T.z1[a][2], 0.f),
                        fmaxf(T.z1[a][3], 0.f));
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) dz2b[cb] = pack4f(dz2[cb][0], dz2[cb][1], dz2[cb][2], dz2[cb][3]);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) G.w2[a * 4 + cb] = mfma(h1t[a], dz2b[cb], G.w2[a * 4 + cb]);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dH1 = dZ2 W2^T: A = dZ2 rows (staged), B[o][k] = W2[k][o]
    v4s a2[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) a2[kb] = *reinterpret_cast<const v4s *>(&s2[c * NH + 16 * kb + 4 * g]);
    v4s dz1b[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        const int k = 16 * cb + c;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            const v4s b = *reinterpret_cast<const v4s *>(&W.w2[k * NH + 16 * kb + 4 * g]);
            acc = mfma(a2[kb], b, acc);
        }
        v4f dz1;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            dz1[j] = T.z1[cb][j] > 0.f ? acc[j] : 0.f;
            G.b1[cb] += dz1[j];
        }
        dz1b[cb] = pack4f(dz1[0], dz1[1], dz1[2], dz1[3]);
    }
    // dW1[i][k] += sum_rows X[row][i] dZ1[row][k]: A = X^T (A[i = lane%16][row 4g + j])
    v4s xt;
    {
        float xv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t r = r0 + 4 * g + j;
            xv[j] = r < n ? X[(rows ? rows[r] : r) * NIN + c] : 0.f;
        }
        xt = pack4f(xv[0], xv[1], xv[2], xv[3]);
    }
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) G.w1[cb] = mfma(xt, dz1b[cb], G.w1[cb]);
    __builtin_amdgcn_wave_barrier();
}

// fold a wave's gradient registers into the LDS gradient vector
__device__ void fold(const Grads &G, float *gsum) {
    const int l = __lane_id(), g = l >> 4, c = l & 15;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int cb = 0; cb < 4; ++cb)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                atomicAdd(&gsum[OFF_W2 + (16 * a + 4 * g + j) * NH + 16 * cb + c], G.w2[a * 4 + cb][j]);
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int j = 0; j < 4; ++j) atomicAdd(&gsum[OFF_W1 + (4 * g + j) * NH + 16 * cb + c], G.w1[cb][j]);
    // per-column sums: reduce over the four lane groups first
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
        float w3 = G.w3[cb], b2 = G.b2[cb], b1 = G.b1[cb];
        w3 += __shfl_xor(w3, 16, 64);
        w3 += __shfl_xor(w3, 32, 64);
        b2 += __shfl_xor(b2, 16, 64);
        b2 += __shfl_xor(b2, 32, 64);
        b1 += __shfl_xor(b1, 16, 64);
        b1 += __shfl_xor(b1, 32, 64);
        if (g == 0) {
            atomicAdd(&gsum[OFF_W3 + 16 * cb + c], w3);
            atomicAdd(&gsum[OFF_B2 + 16 * cb + c], b2);
            atomicAdd(&gsum[OFF_B1 + 16 * cb + c], b1);
        }
    }
    float b3 = G.b3, ls = G.loss;
    for (int o = 32; o >= 1; o >>= 1) {
        b3 += __shfl_xor(b3, o, 64);
        ls += __shfl_xor(ls, o, 64);
    }
    if (l == 0) {
        atomicAdd(&gsum[OFF_B3], b3);
        atomicAdd(&gsum[NPARAM], ls);
    }
}

struct AdamCfg {
    float lr, beta1, beta2, eps;
    int64_t step0; // Adam steps already taken
};

// mode 0: nsteps Adam steps over minibatches rows[s * batch ..]; mode 1: one
// gradient (and loss) of rows 0..batch-1 written to grad_out, no update.
__global__ __launch_bounds__(MBLK) void k_mlp_train(const float *__restrict__ X, const float *__restrict__ tgt,
                                                    const int32_t *__restrict__ rows, int64_t nsteps, int batch,
                                                    float *params, float *adam_m, float *adam_v, AdamCfg cfg,
                                                    float *loss_out, float *grad_out, int mode) {
    __shared__ Weights W;
    __shared__ alignas(16) unsigned short stage1[MWAVES][16 * NH];
    __shared__ alignas(16) unsigned short stage2[MWAVES][16 * NH];
    __shared__ float gsum[NPARAM + 1];
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < NPARAM; i += MBLK) set_param(W, i, params[i]);
    const float scale = 1.f / (float)batch;
    const int tiles = (batch + 15) / 16;
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int i = threadIdx.x; i <= NPARAM; i += MBLK) gsum[i] = 0.f;
        __syncthreads();
        Grads G;
        zero(G);
        const int32_t *rs = rows ? rows + s * (int64_t)batch : nullptr;
        for (int t = wave; t < tiles; t += MWAVES)
            tile_backward(X, tgt, rs, 16 * (int64_t)t, batch, scale, W, stage1[wave], stage2[wave], G);
        fold(G, gsum);
        __syncthreads();
        if (mode == 1) {
            for (int i = threadIdx.x; i < NPARAM; i += MBLK) grad_out[i] = gsum[i];
            if (threadIdx.x == 0 && loss_out) loss_out[0] = gsum[NPARAM];
            return;
        }
        if (threadIdx.x == 0 && loss_out) loss_out[s] = gsum[NPARAM];
        const float t = (float)(cfg.step0 + s + 1);
        const float c1 = 1.f - powf(cfg.beta1, t), c2 = 1.f - powf(cfg.beta2, t);
        for (int i = threadIdx.x; i < NPARAM; i += MBLK) {
            const float gi = gsum[i];
            const float m = cfg.beta1 * adam_m[i] + (1.f - cfg.beta1) * gi;
            const float v = cfg.beta2 * adam_v[i] + (1.f - cfg.beta2) * gi * gi;
            adam_m[i] = m;
            adam_v[i] = v;
            const float p = params[i] - cfg.lr * (m / c1) / (sqrtf(v / c2) + cfg.eps);
            params[i] = p;
            set_param(W, i, p);
        }
        __syncthreads();
    }
}

} // namespace

// -------------------------------------------------------------------------
// host side
// -------------------------------------------------------------------------
constexpr int NPARAM_PUBLIC = NPARAM;
hd_status mlp_forward(const float *X, int64_t n, const float *params, float *y, hipStream_t s) {
    if (n <= 0) return HD_OK;
    const int64_t tiles = (n + 15) / 16;
    const unsigned grid = (unsigned)std::min<int64_t>((tiles + MWAVES - 1) / MWAVES, 4096);
    k_mlp_forward<<<grid, MBLK, 0, s>>>(X, n, params, y);
    HD_LAUNCH_CHECK();
    return HD_OK;
}

hd_status mlp_grad(const float *X, const float *t, int64_t n, const float *params, float *grad, float *loss,
                   hipStream_t s) {
    AdamCfg cfg{0.f, 0.f, 0.f, 0.f, 0};
    k_mlp_train<<<1, MBLK, 0, s>>>(X, t, nullptr, 1, (int)n, const_cast<float *>(params), nullptr, nullptr, cfg,
                                   loss, grad, 1);
    HD_LAUNCH_CHECK();
    return HD_OK;
}

hd_status mlp_train(const float *X, const float *t, const int32_t *rows, int64_t nsteps, int batch, float *params,
                    float *m, float *v, int64_t step0, float lr, float beta1, float beta2, float eps, float *loss,
                    hipStream_t s) {
    AdamCfg cfg{lr, beta1, beta2, eps, step0};
    k_mlp_train<<<1, MBLK, 0, s>>>(X, t, rows, nsteps, batch, params, m, v, cfg, loss, nullptr, 0);
    HD_LAUNCH_CHECK();
    return HD_OK;
}

} // namespace hd

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
namespace {
template <class F> hd_status mlp_guard(F &&f) {
    try {
        return f();
    } catch (const hd::Error &e) {
        return e.st;
    } catch (...) {
        return HD_E_INTERNAL;
    }
}
} // namespace

extern "C" {

int32_t hd_mlp_nparams(void) { return hd::NPARAM_PUBLIC; }

hd_status hd_mlp_forward(const float *X, int64_t n, const float *params, float *y, hd_stream_t stream) {
    if (n < 0 || (n > 0 && (!X || !params || !y))) return HD_E_INVALID;
    return mlp_guard([&] { return hd::mlp_forward(X, n, params, y, (hipStream_t)stream); });
}

hd_status hd_mlp_grad(const float *X, const float *t, int64_t n, const float *params, float *grad, float *loss,
                      hd_stream_t stream) {
    if (n <= 0 || n > (int64_t(1) << 30) || !X || !t || !params || !grad) return HD_E_INVALID;
    return mlp_guard([&] { return hd::mlp_grad(X, t, n, params, grad, loss, (hipStream_t)stream); });
}

hd_status hd_mlp_train(const float *X, const float *t, const int32_t *rows, int64_t nsteps, int32_t batch,
                       float *params, float *adam_m, float *adam_v, int64_t step0, float lr, float *loss,
                       hd_stream_t stream) {
    if (nsteps < 0 || batch <= 0 || !X || !t || !rows || !params || !adam_m || !adam_v || !(lr > 0))
        return HD_E_INVALID;
    if (nsteps == 0) return HD_OK;
    return mlp_guard([&] {
        return hd::mlp_train(X, t, rows, nsteps, batch, params, adam_m, adam_v, step0, lr, 0.9f, 0.999f, 1e-8f,
                             loss, (hipStream_t)stream);
    });
}

} // extern "C"
