// cs_mlp.hip -- kernels of the sampler network (2 -> 64 x4 (SiLU) -> 2).
//
// FP32 engine (training, FP32 inference, calibration): one workgroup of 256
// lanes holds 64 samples; its four waves split every layer's 64 output
// neurons (wave w computes neurons 16w..16w+15 for all 64 samples), reading
// the sample's input row from LDS (128-bit loads) and the weights as
// wave-uniform scalar loads.  Backward keeps SiLU'(z) in registers (the lane
// that produced z consumes it), the layer outputs in LDS for the weight
// gradients, and writes one partial gradient per workgroup; a second kernel
// sums the partials in a fixed order (bitwise reproducible) and applies Adam.
//
// MFMA engine (BF16 / FP8 inference): the tile evaluator of cs_net.h on
// grid-strided 16-sample tiles, the fragments and small parameters in LDS.
// Preparation kernels build the fragments (BF16 rounding, or per-layer FP8
// scales from the weight amax and a calibration pass of the FP32 engine).
#include <hip/hip_runtime.h>

#include <cmath>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_net.h"

namespace cs {

constexpr int kMlpThreads = 256;
constexpr int kMlpSamples = 64;  // samples per FP32 workgroup
constexpr int kRow = 68;         // LDS row stride (floats), 16-byte aligned rows

__device__ __forceinline__ float silu_grad_f32(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// ---------------------------------------------------------------------------
// FP32 engine pieces
// ---------------------------------------------------------------------------
// Layer 1 (2 -> 64) for this lane's 16 neurons [16w, 16w+16) of sample s.
__device__ __forceinline__ void fwd_first(const float* P, int w, float f1, float f2, float z[16]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int j = 16 * w + i;
        z[i] = fmaf(P[kOffW1 + 2 * j + 1], f2, fmaf(P[kOffW1 + 2 * j], f1, P[kOffB1 + j]));
    }
}

// Hidden layer (64 -> 64): z_j = b_j + sum_k W[j][k] h[k], k ascending.
__device__ __forceinline__ void fwd_hidden(const float* W, const float* b, int w, const float* hrow, float z[16]) {
#pragma unroll
    for (int i = 0; i < 16; ++i) z[i] = b[16 * w + i];
#pragma unroll 4
    for (int k = 0; k < kMlpHidden; k += 4) {
        const float4 hv = *(const float4*)(hrow + k);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float* wr = W + (16 * w + i) * kMlpHidden + k;
            float a = z[i];
            a = fmaf(wr[0], hv.x, a);
            a = fmaf(wr[1], hv.y, a);
            a = fmaf(wr[2], hv.z, a);
            a = fmaf(wr[3], hv.w, a);
            z[i] = a;
        }
    }
}

// Output layer (64 -> 2) for one sample, k ascending.
__device__ __forceinline__ void fwd_out(const float* P, const float* hrow, float& y0, float& y1) {
    float a0 = P[kOffB5], a1 = P[kOffB5 + 1];
#pragma unroll 8
    for (int k = 0; k < kMlpHidden; ++k) {
        a0 = fmaf(P[kOffW5 + k], hrow[k], a0);
        a1 = fmaf(P[kOffW5 + kMlpHidden + k], hrow[k], a1);
    }
    y0 = a0;
    y1 = a1;
}

__device__ __forceinline__ uint32_t float_bits(float f) { return __float_as_uint(f); }

// Forward pass of one FP32 workgroup; the last hidden output ends in H[1]
// (ping-pong buffers H[0], H[1]).  amax (nullable): running max |h| of the
// inputs of hidden layers 2..4, as float bits.
__device__ __forceinline__ void fwd_block_f32(const float* P, float f1, float f2, bool active, float (*H)[kMlpSamples][kRow],
                                              uint32_t* amax) {
    const int tid = threadIdx.x;
    const int w = wave_uniform(tid >> 6);
    const int s = tid & 63;
    float z[16];
    fwd_first(P, w, f1, f2, z);
    float m = 0.0f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const float h = silu_f32(z[i]);
        H[0][s][16 * w + i] = h;
        m = fmaxf(m, fabsf(h));
    }
    if (amax && active) atomicMax(&amax[0], float_bits(m));
    __syncthreads();
    const float* Ws[3] = {P + kOffW2, P + kOffW3, P + kOffW4};
    const float* Bs[3] = {P + kOffB2, P + kOffB3, P + kOffB4};
#pragma unroll 1
    for (int L = 0; L < 3; ++L) {
        const int src = L & 1, dst = src ^ 1;
        fwd_hidden(Ws[L], Bs[L], w, H[src][s], z);
        __syncthreads();  // all reads of H[src] done before it is overwritten next layer
        m = 0.0f;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float h = silu_f32(z[i]);
            H[dst][s][16 * w + i] = h;
            m = fmaxf(m, fabsf(h));
        }
        if (amax && active && L < 2) atomicMax(&amax[L + 1], float_bits(m));
        __syncthreads();
    }
}

struct FwdArgs {
    const float* P;
    const float *x, *u;
    int64_t n;
    float* y;      // nullable, 2n
    float* mu;     // nullable
    float* ratio;  // nullable
    uint8_t* mask; // nullable
    uint32_t* amax;  // nullable: calibration
};


// Sampler reading of the outputs (shared by every precision): inside the
// network's domain cos(theta) = clamp(y0, -1, 1) and the energy ratio follows
// from it by the Compton relation; outside it the plain sampler answers.
__device__ __forceinline__ void net_out(const FwdArgs& a, int64_t i, float x, float y0) {
    const float mu = fminf(fmaxf(y0, -1.0f), 1.0f);
    if (a.mu) a.mu[i] = mu;
    if (a.ratio) a.ratio[i] = 1.0f / (1.0f + x * (1.0f - mu));
    if (a.mask) a.mask[i] = 0;
}
__device__ __forceinline__ void fallback_out(const FwdArgs& a, int64_t i, float x, float u) {
    const double v = angle_icdf_v((double)u, (double)x);
    if (a.mu) a.mu[i] = (float)(1.0 - v);
    if (a.ratio) a.ratio[i] = (float)(1.0 / (1.0 + (double)x * v));
    if (a.mask) a.mask[i] = 1;
}
__device__ __forceinline__ void sampler_out(const FwdArgs& a, int64_t i, float x, float u, float y0) {
    if (in_range(x))
        net_out(a, i, x, y0);
    else
        fallback_out(a, i, x, u);
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_fwd_f32(const FwdArgs a) {
    __shared__ float H[2][kMlpSamples][kRow];
    const int s = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * kMlpSamples + s;
    const bool active = i < a.n;
    const float x = active ? a.x[i] : 1.0f, u = active ? a.u[i] : 0.5f;
    float f1, f2;
    features(x, u, f1, f2);
    fwd_block_f32(a.P, f1, f2, active, H, a.amax);
    if (threadIdx.x < 64 && active) {
        float y0, y1;
        fwd_out(a.P, H[1][s], y0, y1);
        if (a.y) {
            a.y[2 * i] = y0;
            a.y[2 * i + 1] = y1;
        }
        if (a.mu || a.ratio || a.mask) sampler_out(a, i, x, u, y0);
    }
}

// ---------------------------------------------------------------------------
// training: forward + backward per workgroup, partial gradients
// ---------------------------------------------------------------------------
struct GradArgs {
    const float* P;
    const float *x, *u, *mu_t, *r_t;
    int64_t n;
    int loss;         // 0 MSE, 1 MAE
    float* partials;  // [blocks][kMlpParams]
    float* loss_partials;  // [blocks]
};

// A workgroup walks the 64-sample tiles blockIdx.x, blockIdx.x + gridDim.x,
// ...; each element of its partial gradient is always produced by the same
// lane, which adds the tiles in that order (no atomics, reproducible).
__global__ __launch_bounds__(kMlpThreads) void k_mlp_grad_block(const GradArgs a) {
    __shared__ float H[4][kMlpSamples][kRow];  // h1..h4
    __shared__ float D[2][kMlpSamples][kRow];  // delta ping-pong
    __shared__ float F[kMlpSamples][2];        // features
    __shared__ float DY[kMlpSamples][2];       // output delta
    __shared__ float s_loss[kMlpSamples];
    const int tid = threadIdx.x;
    const int w = wave_uniform(tid >> 6);
    const int s = tid & 63;
    const int64_t n_tiles = (a.n + kMlpSamples - 1) / kMlpSamples;
    float* out = a.partials + (int64_t)blockIdx.x * kMlpParams;
    // out[idx] = first tile ? v : out[idx] + v (always the same lane for idx)
    auto put = [&](int64_t idx, float v, bool first) { out[idx] = first ? v : out[idx] + v; };
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const bool first = tile == (int64_t)blockIdx.x;
        __syncthreads();  // the previous tile's LDS reads are done
        const int64_t i = tile * kMlpSamples + s;
        const bool active = i < a.n;
        const float* P = a.P;
        float f1 = 0.0f, f2 = 0.0f;
        if (active) features(a.x[i], a.u[i], f1, f2);
        if (w == 0) {
            F[s][0] = f1;
            F[s][1] = f2;
        }
        // forward; SiLU'(z) of this lane's 16 neurons of every layer in registers
        float g[4][16];
        float z[16];
        fwd_first(P, w, f1, f2, z);
    #pragma unroll
        for (int k = 0; k < 16; ++k) {
            H[0][s][16 * w + k] = silu_f32(z[k]);
            g[0][k] = silu_grad_f32(z[k]);
        }
        __syncthreads();
        fwd_hidden(P + kOffW2, P + kOffB2, w, H[0][s], z);
    #pragma unroll
        for (int k = 0; k < 16; ++k) {
            H[1][s][16 * w + k] = silu_f32(z[k]);
            g[1][k] = silu_grad_f32(z[k]);
        }
        __syncthreads();
        fwd_hidden(P + kOffW3, P + kOffB3, w, H[1][s], z);
    #pragma unroll
        for (int k = 0; k < 16; ++k) {
            H[2][s][16 * w + k] = silu_f32(z[k]);
            g[2][k] = silu_grad_f32(z[k]);
        }
        __syncthreads();
        fwd_hidden(P + kOffW4, P + kOffB4, w, H[2][s], z);
    #pragma unroll
        for (int k = 0; k < 16; ++k) {
            H[3][s][16 * w + k] = silu_f32(z[k]);
            g[3][k] = silu_grad_f32(z[k]);
        }
        __syncthreads();
        // output layer and loss gradient
        if (w == 0) {
            float y0, y1;
            fwd_out(P, H[3][s], y0, y1);
            float d0 = 0.0f, d1 = 0.0f, l = 0.0f;
            if (active) {
                const float e0 = y0 - a.mu_t[i], e1 = y1 - a.r_t[i];
                const float inv_n = 1.0f / (float)a.n;
                if (a.loss == 0) {
                    d0 = e0 * inv_n;
                    d1 = e1 * inv_n;
                    l = 0.5f * (e0 * e0 + e1 * e1) * inv_n;
                } else {
                    d0 = (e0 > 0.0f ? 0.5f : (e0 < 0.0f ? -0.5f : 0.0f)) * inv_n;
                    d1 = (e1 > 0.0f ? 0.5f : (e1 < 0.0f ? -0.5f : 0.0f)) * inv_n;
                    l = 0.5f * (fabsf(e0) + fabsf(e1)) * inv_n;
                }
            }
            DY[s][0] = d0;
            DY[s][1] = d1;
            s_loss[s] = l;
        }
        __syncthreads();
        // layer 5 gradients: dW5[o][k] = sum_s DY[s][o] h4[s][k], db5[o] = sum_s DY[s][o]
        if (tid < 128) {
            const int o = tid >> 6, k = tid & 63;
            float acc = 0.0f;
            for (int q = 0; q < kMlpSamples; ++q) acc = fmaf(DY[q][o], H[3][q][k], acc);
            put(kOffW5 + o * kMlpHidden + k, acc, first);
        } else if (tid < 130) {
            const int o = tid - 128;
            float acc = 0.0f;
            for (int q = 0; q < kMlpSamples; ++q) acc += DY[q][o];
            put(kOffB5 + o, acc, first);
        } else if (tid == 130) {
            float acc = 0.0f;
            for (int q = 0; q < kMlpSamples; ++q) acc += s_loss[q];
            a.loss_partials[blockIdx.x] = first ? acc : a.loss_partials[blockIdx.x] + acc;
        }
        // delta4 = (W5^T DY) * g4
    #pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int j = 16 * w + k;
            D[0][s][j] = (P[kOffW5 + j] * DY[s][0] + P[kOffW5 + kMlpHidden + j] * DY[s][1]) * g[3][k];
        }
        __syncthreads();
        // hidden layers 4, 3, 2: weight gradient from D[cur] and H[L-1], delta of
        // the layer below into D[cur ^ 1]
        const int offW[3] = {kOffW4, kOffW3, kOffW2};
        const int offB[3] = {kOffB4, kOffB3, kOffB2};
        int cur = 0;
    #pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int hin = 2 - m;  // H index of the layer input (h3, h2, h1)
            {
                // dW[j][k] = sum_s D[s][j] H[s][k] for j = tid%64, k in [16 w, 16 w + 16)
                const int j = s;
                float acc[16];
    #pragma unroll
                for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
                float db = 0.0f;
                for (int q = 0; q < kMlpSamples; ++q) {
                    const float d = D[cur][q][j];
                    db += d;
                    const float* hr = &H[hin][q][16 * w];
    #pragma unroll
                    for (int k = 0; k < 16; k += 4) {
                        const float4 hv = *(const float4*)(hr + k);
                        acc[k] = fmaf(d, hv.x, acc[k]);
                        acc[k + 1] = fmaf(d, hv.y, acc[k + 1]);
                        acc[k + 2] = fmaf(d, hv.z, acc[k + 2]);
                        acc[k + 3] = fmaf(d, hv.w, acc[k + 3]);
                    }
                }
    #pragma unroll
                for (int k = 0; k < 16; ++k) put(offW[m] + j * kMlpHidden + 16 * w + k, acc[k], first);
                if (w == 0) put(offB[m] + j, db, first);
            }
            {
                // delta of the layer below: (W^T D[cur])[s][j] * g, j in this lane's range
                const float* W = P + offW[m];
                float acc[16];
    #pragma unroll
                for (int k = 0; k < 16; ++k) acc[k] = 0.0f;
    #pragma unroll 4
                for (int o = 0; o < kMlpHidden; o += 4) {
                    const float4 dv = *(const float4*)(&D[cur][s][o]);
    #pragma unroll
                    for (int k = 0; k < 16; ++k) {
                        const int j = 16 * w + k;
                        float t = acc[k];
                        t = fmaf(W[(o + 0) * kMlpHidden + j], dv.x, t);
                        t = fmaf(W[(o + 1) * kMlpHidden + j], dv.y, t);
                        t = fmaf(W[(o + 2) * kMlpHidden + j], dv.z, t);
                        t = fmaf(W[(o + 3) * kMlpHidden + j], dv.w, t);
                        acc[k] = t;
                    }
                }
    #pragma unroll
                for (int k = 0; k < 16; ++k) D[cur ^ 1][s][16 * w + k] = acc[k] * g[hin][k];
            }
            __syncthreads();
            cur ^= 1;
        }
        // layer 1: dW1[j][i] = sum_s D[s][j] F[s][i], db1[j] = sum_s D[s][j]
        if (tid < 64) {
            const int j = tid;
            float a0 = 0.0f, a1 = 0.0f, db = 0.0f;
            for (int q = 0; q < kMlpSamples; ++q) {
                const float d = D[cur][q][j];
                a0 = fmaf(d, F[q][0], a0);
                a1 = fmaf(d, F[q][1], a1);
                db += d;
            }
            put(kOffW1 + 2 * j, a0, first);
            put(kOffW1 + 2 * j + 1, a1, first);
            put(kOffB1 + j, db, first);
        }
    }
}

// Fixed-order sum of the per-workgroup partials; then either write the
// gradient or apply Adam (FP32 state, bias corrections from the host).
struct ReduceArgs {
    const float* partials;
    const float* loss_partials;
    int64_t blocks;
    float* grad_out;  // nullable
    float* loss_out;  // nullable
    float* params;    // nullable: apply Adam
    float *m, *v;
    float lr, bc1, bc2;
};

__global__ __launch_bounds__(256) void k_mlp_reduce(const ReduceArgs a) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p < kMlpParams) {
        float g = 0.0f;
        for (int64_t b = 0; b < a.blocks; ++b) g += a.partials[b * kMlpParams + p];
        if (a.grad_out) a.grad_out[p] = g;
        if (a.params) {
            const float m = 0.9f * a.m[p] + 0.1f * g;
            const float v = 0.999f * a.v[p] + 0.001f * g * g;
            a.m[p] = m;
            a.v[p] = v;
            const float mh = m / a.bc1, vh = v / a.bc2;
            a.params[p] -= a.lr * mh / (sqrtf(vh) + 1e-8f);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.loss_out) {
        float l = 0.0f;
        for (int64_t b = 0; b < a.blocks; ++b) l += a.loss_partials[b];
        *a.loss_out = l;
    }
}

__global__ void k_mlp_adam_only(float* params, float* m_, float* v_, const float* grad, float lr, float bc1,
                                float bc2) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float m = 0.9f * m_[p] + 0.1f * g;
    const float v = 0.999f * v_[p] + 0.001f * g * g;
    m_[p] = m;
    v_[p] = v;
    params[p] -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
}

// ---------------------------------------------------------------------------
// MFMA engine
// ---------------------------------------------------------------------------

// Build fragments: thread per (layer, tile_out, kstep, lane, e).
__global__ void k_mlp_build_frag(const float* P, const float* scales, int prec, __bf16* fb, uint8_t* f8) {
    const int idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= kFragCount * 8) return;
    const int e = idx & 7, lane = (idx >> 3) & 63, s = (idx >> 9) & 1, t = (idx >> 10) & 3, L = idx >> 12;
    const int offW[3] = {kOffW2, kOffW3, kOffW4};
    const int row = 16 * t + (lane & 15);
    const int col = frag_in_neuron(s, lane >> 4, e);
    const float wv = P[offW[L] + row * kMlpHidden + col];
    if (prec == CS_SAMPLER_MLP_BF16)
        fb[idx] = (__bf16)wv;
    else
        f8[idx] = to_e4m3(wv / scales[L]);
}

// Per-layer weight amax -> scale (one workgroup per hidden layer).
__global__ __launch_bounds__(256) void k_mlp_weight_scale(const float* P, float* scales) {
    __shared__ float s_m[256];
    const int offW[3] = {kOffW2, kOffW3, kOffW4};
    float m = 0.0f;
    for (int i = threadIdx.x; i < kMlpHidden * kMlpHidden; i += 256) m = fmaxf(m, fabsf(P[offW[blockIdx.x] + i]));
    s_m[threadIdx.x] = m;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) s_m[threadIdx.x] = fmaxf(s_m[threadIdx.x], s_m[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) scales[blockIdx.x] = fmaxf(s_m[0], 1e-30f) / kE4M3Max;
}

__global__ void k_mlp_zero_amax(uint32_t* amax) {
    if (threadIdx.x < 3) amax[threadIdx.x] = 0u;
}

__global__ void k_mlp_act_scale(float* scales) {
    if (threadIdx.x < 3) {
        const float m = __uint_as_float(((const uint32_t*)scales)[6 + threadIdx.x]);
        scales[3 + threadIdx.x] = fmaxf(m, 1e-30f) / kE4M3Max;
    }
}

constexpr int kMfmaThreads = 256;
// Register budget and tiles in flight of the inference kernel: with all four
// tiles of a group side by side and at most 168 registers (three waves per
// SIMD) it needs no spills; measured on 2^22 samples this was the fastest of
// {2, 4} tiles x {2, 3, 4} waves per SIMD (all of which give the same bits).
constexpr int kMfmaWavesPerSimd = 3;
constexpr int kMfmaTilesAtOnce = 4;
constexpr int kFbCap = 128;  // deferred samples one wave can hold (it flushes at 64)

// The plain sampler for the first `cnt` (<= 64) deferred samples of a wave's
// queue, one per lane.  Called by the whole wave.
__device__ __forceinline__ void fallback_pass(const FwdArgs& a, const int64_t* q, int cnt) {
    const int lane = lane_id();
    const bool act = lane < cnt;
    const int64_t i = act ? q[lane] : 0;
    const float x = act ? a.x[i] : 0.0f, u = act ? a.u[i] : 0.5f;
    const double v = angle_icdf_v((double)u, (double)x);
    if (act) {
        if (a.mu) a.mu[i] = (float)(1.0 - v);
        if (a.ratio) a.ratio[i] = (float)(1.0 / (1.0 + (double)x * v));
        if (a.mask) a.mask[i] = 1;
    }
}

// Each wave walks groups of 64 consecutive samples (wave-strided over the
// grid): lane l reads sample l and forms its features once, the four
// 16-sample tiles are evaluated side by side, and lane
// l takes its own sample's outputs back and writes them (whole-line stores).
// Samples outside the network's domain are answered afterwards, in a second
// walk over the same groups: they are queued per wave in LDS, in order, and
// the plain sampler takes them in dense passes of 64, so that its Newton
// iteration never runs on a mostly idle wave (and its registers are not
// live while the network runs).  No workgroup barrier after the set-up.
template <int PREC>
__global__ __launch_bounds__(kMfmaThreads, kMfmaWavesPerSimd) void k_mlp_mfma(const FwdArgs a, const MlpDev m) {
    __shared__ NetLds<PREC> s_net;
    __shared__ int64_t s_fb[kMfmaThreads / 64][kFbCap];
    net_load<PREC>(s_net, m);
    __syncthreads();
    const int lane = lane_id();
    const int wave = wave_uniform((int)threadIdx.x >> 6);
    const bool sampling = a.mu || a.ratio || a.mask;
    const int64_t n_groups = (a.n + 63) / 64;
    const int64_t first = (int64_t)blockIdx.x * (kMfmaThreads / 64) + wave;
    const int64_t stride = (int64_t)gridDim.x * (kMfmaThreads / 64);
    for (int64_t grp = first; grp < n_groups; grp += stride) {
        const int64_t i = grp * 64 + lane;
        const bool active = i < a.n;
        const float x = active ? a.x[i] : 1.0f, u = active ? a.u[i] : 0.5f;
        float f1, f2;
        features(x, u, f1, f2);
        // the network's LDS copy is re-read for every group: an opaque
        // (wave-uniform, zero) offset keeps the compiler from hoisting all of
        // it into registers, which would cost occupancy
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        const auto* frag = s_net.frag + opaque;
        const float* P = s_net.P + opaque;
        const float* sc = s_net.sc + opaque;
        float o0 = 0.0f, o1 = 0.0f;
#pragma unroll
        for (int t0 = 0; t0 < 4; t0 += kMfmaTilesAtOnce) {
            float g1[kMfmaTilesAtOnce], g2[kMfmaTilesAtOnce], y0[kMfmaTilesAtOnce], y1[kMfmaTilesAtOnce];
#pragma unroll
            for (int k = 0; k < kMfmaTilesAtOnce; ++k) {
                const int src = 16 * (t0 + k) + (lane & 15);
                g1[k] = __shfl(f1, src, 64);
                g2[k] = __shfl(f2, src, 64);
            }
            mlp_tiles<PREC, kMfmaTilesAtOnce>(frag, P, sc, g1, g2, y0, y1);
#pragma unroll
            for (int k = 0; k < kMfmaTilesAtOnce; ++k)
                if ((lane >> 4) == t0 + k) {
                    o0 = y0[k];
                    o1 = y1[k];
                }
        }
        if (active && a.y) *(float2*)(a.y + 2 * i) = make_float2(o0, o1);
        if (sampling && active && in_range(x)) net_out(a, i, x, o0);
    }
    if (!sampling) return;
    int64_t* fb = s_fb[wave];
    int nfb = 0;  // wave-uniform
    for (int64_t grp = first; grp < n_groups; grp += stride) {
        const int64_t i = grp * 64 + lane;
        const bool defer = i < a.n && !in_range(a.x[i]);
        const uint64_t msk = __ballot(defer);
        if (msk == 0) continue;
        if (defer) fb[nfb + __popcll(msk & ((1ull << lane) - 1ull))] = i;
        nfb += __popcll(msk);
        // the queue's writes precede the pass's reads (one wave, in order)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (nfb >= 64) {
            fallback_pass(a, fb, 64);
            const int64_t rest = lane < nfb - 64 ? fb[64 + lane] : 0;
            __builtin_amdgcn_wave_barrier();
            if (lane < nfb - 64) fb[lane] = rest;
            nfb -= 64;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (nfb > 0) fallback_pass(a, fb, nfb);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
constexpr int64_t kMaxGradBlocks = 1024;

int64_t mlp_grad_blocks(int64_t n) {
    const int64_t t = (n + kMlpSamples - 1) / kMlpSamples;
    return t < kMaxGradBlocks ? t : kMaxGradBlocks;
}

hipError_t launch_mlp_forward(const MlpDev& m, cs_sampler prec, const float* x, const float* u, int64_t n, float* y,
                              float* mu, float* ratio, uint8_t* mask, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    FwdArgs a = {m.params, x, u, n, y, mu, ratio, mask, nullptr};
    if (prec == CS_SAMPLER_MLP_F32) {
        k_mlp_fwd_f32<<<(unsigned)((n + kMlpSamples - 1) / kMlpSamples), kMlpThreads, 0, st>>>(a);
    } else {
        // one 64-sample group per wave and step of the loop; 2048 workgroups
        // (8 per compute unit) cover the chip
        const int64_t groups = (n + 63) / 64;
        int64_t blocks = (groups + kMfmaThreads / 64 - 1) / (kMfmaThreads / 64);
        if (blocks > 2048) blocks = 2048;
        if (prec == CS_SAMPLER_MLP_BF16)
            k_mlp_mfma<CS_SAMPLER_MLP_BF16><<<(unsigned)blocks, kMfmaThreads, 0, st>>>(a, m);
        else
            k_mlp_mfma<CS_SAMPLER_MLP_FP8><<<(unsigned)blocks, kMfmaThreads, 0, st>>>(a, m);
    }
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev& m, const float* x, const float* u, const float* mu_t, const float* r_t,
                           int64_t n, int loss, float* partials, float* loss_partials, float* grad_out,
                           float* loss_out, float* adam_m, float* adam_v, float* params_rw, float lr, int64_t t,
                           hipStream_t st) {
    const int64_t blocks = mlp_grad_blocks(n);
    GradArgs g = {m.params, x, u, mu_t, r_t, n, loss, partials, loss_partials};
    k_mlp_grad_block<<<(unsigned)blocks, kMlpThreads, 0, st>>>(g);
    ReduceArgs r = {};
    r.partials = partials;
    r.loss_partials = loss_partials;
    r.blocks = blocks;
    r.grad_out = grad_out;
    r.loss_out = loss_out;
    if (params_rw) {
        r.params = params_rw;
        r.m = adam_m;
        r.v = adam_v;
        r.lr = lr;
        r.bc1 = (float)(1.0 - std::pow(0.9, (double)t));
        r.bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    }
    k_mlp_reduce<<<(kMlpParams + 255) / 256, 256, 0, st>>>(r);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, int64_t t, hipStream_t st) {
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    k_mlp_adam_only<<<(kMlpParams + 255) / 256, 256, 0, st>>>(params, m, v, grad, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_quantize(float* params, void* frag_bf16, void* frag_fp8, float* scales, cs_sampler prec,
                               const float* cx, const float* cu, int64_t n, hipStream_t st) {
    const unsigned nb = (kFragCount * 8 + 255) / 256;
    if (prec == CS_SAMPLER_MLP_BF16) {
        k_mlp_build_frag<<<nb, 256, 0, st>>>(params, scales, CS_SAMPLER_MLP_BF16, (__bf16*)frag_bf16, nullptr);
    } else {
        k_mlp_zero_amax<<<1, 64, 0, st>>>((uint32_t*)scales + 6);
        FwdArgs a = {params, cx, cu, n, nullptr, nullptr, nullptr, nullptr, (uint32_t*)scales + 6};
        k_mlp_fwd_f32<<<(unsigned)((n + kMlpSamples - 1) / kMlpSamples), kMlpThreads, 0, st>>>(a);
        k_mlp_act_scale<<<1, 64, 0, st>>>(scales);
        k_mlp_weight_scale<<<3, 256, 0, st>>>(params, scales);
        k_mlp_build_frag<<<nb, 256, 0, st>>>(params, scales, CS_SAMPLER_MLP_FP8, nullptr, (uint8_t*)frag_fp8);
    }
    return hipGetLastError();
}

}  // namespace cs
