// cs_net.h -- device-side evaluation of the sampler network (2 -> 64 x4
// (SiLU) -> 2), shared by the network kernels and by the collision phase of
// the step kernels so that both give the same bits for the same inputs.
//
// Inputs are FP32: f1 maps log10 x linearly from the network's x range onto
// [-1, 1] (by default x in [1e-4, 1e2]), f2 = 2u - 1.  Output 0 is
// cos(theta), output 1 the energy ratio.
//
// Two evaluators:
//   * FP32: either a workgroup-wide engine (cs_mlp.hip) or, inside the step,
//     one lane per sample (mlp_lane_f32) with the layer outputs in LDS.  Both
//     accumulate b + sum_k W[j][k] h[k] with k ascending and fmaf, so they
//     agree bitwise.
//   * MFMA (BF16 / FP8 E4M3): a wave evaluates 16 samples per tile with
//     v_mfma_f32_16x16x32_{bf16,fp8}.  Lane l owns sample l%16 and, in group
//     g = l/16, the neurons 16t + 4g + r (t, r = 0..3): exactly the rows of
//     the accumulator fragment it holds, so a layer's output stays in
//     registers and becomes the next layer's B operand once the weight
//     fragments list the input neurons in the same order (k-slot 8g + e of
//     k-step s <-> neuron 16(2s + e/4) + 4g + e%4, i.e. the lane's neurons
//     0..7 form k-step 0 and 8..15 k-step 1).  Layers 1 and 5 (K = 2, N = 2)
//     stay in FP32 on the vector ALUs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cs_device.h"
#include "cs_internal.h"

namespace cs {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr float kE4M3Max = 448.0f;

__device__ __forceinline__ float silu_f32(float z) { return z / (1.0f + expf(-z)); }

// The reduced-precision paths carry every pre-activation and activation of
// the hidden layers scaled by kSiluScale = -log2(e): with t = kSiluScale z,
// e^-z = 2^t, so SiLU(z) = z / (1 + e^-z) becomes t / (1 + 2^t) / kSiluScale
// and the exponential takes the layer's output directly.  The factor is
// folded into the FP32 parameters the engine keeps in LDS (W1, the biases,
// and 1 / kSiluScale into W5) and into the FP8 input scales; the MFMA weights
// are unchanged.  Its result is rounded to BF16/FP8, so the hardware exp2 and
// reciprocal approximations (about 1 ulp of FP32) replace the correctly
// rounded division.
constexpr float kSiluScale = -1.4426950408889634f;

__device__ __forceinline__ float silu_scaled(float t) {
    return t * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(t));
}

// Input features: f1 = log10 x mapped from the network's x range onto
// [-1, 1] (the hardware log2, about 1 ulp, scaled), f2 = 2u - 1.
__device__ __forceinline__ void features(float x, float u, const NetDomain& d, float& f1, float& f2) {
    f1 = fmaf(__builtin_amdgcn_logf(x), d.f_a, d.f_b);
    f2 = 2.0f * u - 1.0f;
}

__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// The network answers for x in its range (bounds as FP32); the plain sampler
// answers elsewhere.
__device__ __forceinline__ bool in_range(float x, const NetDomain& d) { return x >= d.x_lo && x <= d.x_hi; }

// Input neuron of k-slot e (0..7) of k-step s in lane group g.
__host__ __device__ __forceinline__ int frag_in_neuron(int s, int g, int e) {
    return 16 * (2 * s + e / 4) + 4 * g + (e & 3);
}

__device__ __forceinline__ uint8_t to_e4m3(float v) {
    v = fminf(fmaxf(v, -kE4M3Max), kE4M3Max);  // saturating conversion
    const uint32_t packed = __builtin_amdgcn_cvt_pk_fp8_f32(v, 0.0f, 0u, false);
    return (uint8_t)(packed & 0xFFu);
}

// Compact copy of the FP32 parameters the MFMA engine reads from LDS: W1 and
// the hidden biases times kSiluScale, W5 divided by it, b5 as is.
constexpr int cW1 = 0, cB1 = 128, cB2 = 192, cB3 = 256, cB4 = 320, cW5 = 384, cB5 = 512, kSmall = 514;

// Entry i of the compact copy: where it comes from in the parameter block,
// and its value there scaled as the engine keeps it.
__device__ __forceinline__ int small_param_src(int i) {
    if (i < cB1) return kOffW1 + i;
    if (i < cB2) return kOffB1 + (i - cB1);
    if (i < cB3) return kOffB2 + (i - cB2);
    if (i < cB4) return kOffB3 + (i - cB3);
    if (i < cW5) return kOffB4 + (i - cB4);
    if (i < cB5) return kOffW5 + (i - cW5);
    return kOffB5 + (i - cB5);
}
__device__ __forceinline__ float small_param_value(int i, float v) {
    return i < cW5 ? v * kSiluScale : (i < cB5 ? v / kSiluScale : v);
}

__device__ __forceinline__ void load_small_params(const float* P, float* s) {
    for (int i = threadIdx.x; i < kSmall; i += blockDim.x) s[i] = small_param_value(i, P[small_param_src(i)]);
}

template <int PREC>
struct FragT;
template <>
struct FragT<CS_SAMPLER_MLP_BF16> {
    typedef bf16x8 type;
};
template <>
struct FragT<CS_SAMPLER_MLP_FP8> {
    typedef long type;
};

// Packed reduced-precision operand of 8 layer inputs.
template <int PREC>
__device__ __forceinline__ typename FragT<PREC>::type pack_inputs(const float (&h)[8], float inv) {
    if constexpr (PREC == CS_SAMPLER_MLP_BF16) {
        bf16x8 b;
#pragma unroll
        for (int e = 0; e < 8; ++e) b[e] = (__bf16)h[e];
        return b;
    } else {
        // two values per conversion, value e into byte e of the operand
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = fminf(fmaxf(h[e] * inv, -kE4M3Max), kE4M3Max);  // saturating
        uint32_t lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[0], v[1], 0u, false);
        lo = __builtin_amdgcn_cvt_pk_fp8_f32(v[2], v[3], lo, true);
        uint32_t hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[4], v[5], 0u, false);
        hi = __builtin_amdgcn_cvt_pk_fp8_f32(v[6], v[7], hi, true);
        return (long)(((uint64_t)hi << 32) | lo);
    }
}

// Four consecutive parameters of the compact copy (f a multiple of 4: every
// group below starts on a 16-byte boundary) in one LDS read.
__device__ __forceinline__ float4 ld4(const float* P_lds, int f) { return *(const float4*)(P_lds + f); }

// NTL tiles of 16 samples each on one wave, evaluated side by side (their
// MFMA and SiLU chains are independent, so each hides the others' latency).
// For tile k every lane passes the features of sample (lane % 16) in f1[k],
// f2[k] and receives that sample's outputs in y0[k], y1[k].  frag, W1,
// biases, W5 come from LDS.  Each tile's arithmetic is that of a lone tile.
//
// A hidden layer's outputs are packed into the next layer's B operands as
// they are produced (lane neurons 0..7 -> B0, 8..15 -> B1), so only the
// packed inputs and outputs of a layer are live; the last hidden layer's
// outputs go straight into the output layer's sums, in the order the lane's
// neurons are produced (t ascending, then r).
template <int PREC, int NTL>
__device__ __forceinline__ void mlp_tiles(const typename FragT<PREC>::type* frag, const float* P_lds,
                                          const float* scales, const float (&f1)[NTL], const float (&f2)[NTL],
                                          float (&y0)[NTL], float (&y1)[NTL]) {
    typedef typename FragT<PREC>::type FT;
    const int lane = lane_id();
    const int g = lane >> 4;
    FT B0[NTL], B1[NTL];
    {
        const float inv = PREC == CS_SAMPLER_MLP_FP8 ? 1.0f / (kSiluScale * scales[3]) : 1.0f;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            float h[NTL][8];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                // neurons nb .. nb + 3: their (W1 row, b1) as three 16-byte reads
                const int nb = 16 * (2 * half + q) + 4 * g;
                const float4 wa = ld4(P_lds, cW1 + 2 * nb), wb = ld4(P_lds, cW1 + 2 * nb + 4), b1 = ld4(P_lds, cB1 + nb);
                const float w1a[4] = {wa.x, wa.z, wb.x, wb.z}, w1b[4] = {wa.y, wa.w, wb.y, wb.w};
                const float b1v[4] = {b1.x, b1.y, b1.z, b1.w};
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int k = 0; k < NTL; ++k)
                        h[k][4 * q + e] = silu_scaled(fmaf(w1b[e], f2[k], fmaf(w1a[e], f1[k], b1v[e])));
            }
#pragma unroll
            for (int k = 0; k < NTL; ++k) {
                if (half == 0)
                    B0[k] = pack_inputs<PREC>(h[k], inv);
                else
                    B1[k] = pack_inputs<PREC>(h[k], inv);
            }
        }
    }
    const int offB[3] = {cB2, cB3, cB4};
    float p0[NTL], p1[NTL];
#pragma unroll
    for (int k = 0; k < NTL; ++k) p0[k] = p1[k] = 0.0f;
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        float sc = 1.0f, inv_next = 1.0f;
        if constexpr (PREC == CS_SAMPLER_MLP_FP8) {
            // the FP8 inputs are h / s (kSiluScale divided out), so the
            // accumulator takes the factor with the scales
            sc = kSiluScale * (scales[L] * scales[3 + L]);
            if (L < 2) inv_next = 1.0f / (kSiluScale * scales[4 + L]);
        }
        FT N0[NTL], N1[NTL];
        float half[NTL][4];  // outputs of an even tile t, packed with tile t + 1
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const FT A0 = frag[((L * 4 + t) * 2 + 0) * 64 + lane];
            const FT A1 = frag[((L * 4 + t) * 2 + 1) * 64 + lane];
            const float4 b4 = ld4(P_lds, offB[L] + 16 * t + 4 * g);
            const float bias[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
            for (int k = 0; k < NTL; ++k) {
                floatx4 acc;
                float o[4];
                if constexpr (PREC == CS_SAMPLER_MLP_BF16) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[r] = bias[r];
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A0, B0[k], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1, B1[k], acc, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = silu_scaled(acc[r]);
                } else {
                    acc = {0.0f, 0.0f, 0.0f, 0.0f};
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(A0, B0[k], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(A1, B1[k], acc, 0, 0, 0);
#pragma unroll
                    for (int r = 0; r < 4; ++r) o[r] = silu_scaled(fmaf(acc[r], sc, bias[r]));
                }
                if (L == 2) {
                    // output layer sums, neuron order t ascending then r
                    const float4 v0 = ld4(P_lds, cW5 + 16 * t + 4 * g), v1 = ld4(P_lds, cW5 + kMlpHidden + 16 * t + 4 * g);
                    const float w50[4] = {v0.x, v0.y, v0.z, v0.w}, w51[4] = {v1.x, v1.y, v1.z, v1.w};
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        p0[k] = fmaf(w50[r], o[r], p0[k]);
                        p1[k] = fmaf(w51[r], o[r], p1[k]);
                    }
                } else if ((t & 1) == 0) {
#pragma unroll
                    for (int r = 0; r < 4; ++r) half[k][r] = o[r];
                } else {
                    const float h8[8] = {half[k][0], half[k][1], half[k][2], half[k][3], o[0], o[1], o[2], o[3]};
                    if (t == 1)
                        N0[k] = pack_inputs<PREC>(h8, inv_next);
                    else
                        N1[k] = pack_inputs<PREC>(h8, inv_next);
                }
            }
        }
        if (L < 2) {
#pragma unroll
            for (int k = 0; k < NTL; ++k) {
                B0[k] = N0[k];
                B1[k] = N1[k];
            }
        }
    }
#pragma unroll
    for (int k = 0; k < NTL; ++k) {
        float q0 = p0[k], q1 = p1[k];
        // sum the four lane groups (fixed butterfly order)
        q0 += __shfl_xor(q0, 16, 64);
        q1 += __shfl_xor(q1, 16, 64);
        q0 += __shfl_xor(q0, 32, 64);
        q1 += __shfl_xor(q1, 32, 64);
        y0[k] = q0 + P_lds[cB5];
        y1[k] = q1 + P_lds[cB5 + 1];
    }
}

// One tile of 16 samples on one wave (mlp_tiles with one tile).
template <int PREC>
__device__ __forceinline__ void mlp_tile(const typename FragT<PREC>::type* frag, const float* P_lds,
                                         const float* scales, float f1, float f2, float& y0, float& y1) {
    const float a1[1] = {f1}, a2[1] = {f2};
    float b0[1], b1[1];
    mlp_tiles<PREC, 1>(frag, P_lds, scales, a1, a2, b0, b1);
    y0 = b0[0];
    y1 = b1[0];
}

// One sample per lane in FP32, both outputs.  hb: this wave's [64 neurons]
// [64 lanes] LDS buffer.  The weights are read with wave-uniform addresses
// (scalar loads).  Must be called by the whole wave.
__device__ __forceinline__ float2 mlp_lane_f32(const float* __restrict__ P, float* hb, float f1, float f2) {
    const int lane = lane_id();
#pragma unroll 4
    for (int j = 0; j < kMlpHidden; ++j) {
        const float z = fmaf(P[kOffW1 + 2 * j + 1], f2, fmaf(P[kOffW1 + 2 * j], f1, P[kOffB1 + j]));
        hb[j * 64 + lane] = silu_f32(z);
    }
    const int offW[3] = {kOffW2, kOffW3, kOffW4};
    const int offB[3] = {kOffB2, kOffB3, kOffB4};
    float h[kMlpHidden];
#pragma unroll 1
    for (int L = 0; L < 3; ++L) {
#pragma unroll
        for (int k = 0; k < kMlpHidden; ++k) h[k] = hb[k * 64 + lane];
        const float* W = P + offW[L];
        const float* B = P + offB[L];
#pragma unroll 1
        for (int j = 0; j < kMlpHidden; ++j) {
            float z = B[j];
#pragma unroll
            for (int k = 0; k < kMlpHidden; ++k) z = fmaf(W[j * kMlpHidden + k], h[k], z);
            hb[j * 64 + lane] = silu_f32(z);
        }
    }
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) h[k] = hb[k * 64 + lane];
    float a0 = P[kOffB5], a1 = P[kOffB5 + 1];
#pragma unroll
    for (int k = 0; k < kMlpHidden; ++k) {
        a0 = fmaf(P[kOffW5 + k], h[k], a0);
        a1 = fmaf(P[kOffW5 + kMlpHidden + k], h[k], a1);
    }
    return make_float2(a0, a1);
}

// The sampler's reading of the two outputs (cos theta, eps'/eps) at FP32 x,
// as v = 1 - cos(theta) in FP64.  Both outputs carry the event; each is
// trusted where its error moves the event least.  With absolute errors e of
// either output, cos theta gives v to e and the energy ratio r = 1/(1 + x v)
// gives it to e (1 + x v)^2 / x; the ratio is the better guide iff
// (1 + x v)^2 < x, i.e. iff x > 1 and r > 1/sqrt(x) (r^2 x > 1).  So: v from
// the ratio (clamped to [1/(1 + 2x), 1]) there, else from the cosine
// (clamped to [-1, 1]).  The energy ratio written back is recomputed from v,
// so the step conserves energy and momentum exactly whichever output is read.
__device__ __forceinline__ double net_reading_v(float x, float y0, float y1) {
    const double xd = (double)x;
    if (xd > 1.0) {
        const double r = fmin(fmax((double)y1, recip_approx(fma(2.0, xd, 1.0))), 1.0);
        if (r * r * xd > 1.0) return div_normal(1.0 - r, r * xd);
    }
    return 1.0 - (double)fminf(fmaxf(y0, -1.0f), 1.0f);
}

// LDS of the network inside a step kernel (nothing for the plain sampler).
template <int SAMP>
struct NetLds {
    char unused;
};
template <>
struct NetLds<CS_SAMPLER_MLP_F32> {
    float h[4][kMlpHidden * 64];  // one [64][64] buffer per wave (4 waves)
};
template <>
struct NetLds<CS_SAMPLER_MLP_BF16> {
    bf16x8 frag[kFragCount];
    alignas(16) float P[kSmall];  // read in 16-byte groups
    float sc[6];
};
template <>
struct NetLds<CS_SAMPLER_MLP_FP8> {
    long frag[kFragCount];
    alignas(16) float P[kSmall];  // read in 16-byte groups
    float sc[6];
};

// Fill the network LDS (MFMA precisions); every thread of the block calls it,
// followed by a barrier.
template <int SAMP>
__device__ __forceinline__ void net_load(NetLds<SAMP>& s, const MlpDev& m) {
    if constexpr (SAMP == CS_SAMPLER_MLP_BF16 || SAMP == CS_SAMPLER_MLP_FP8) {
        typedef typename FragT<SAMP>::type FT;
        const FT* src = (const FT*)(SAMP == CS_SAMPLER_MLP_BF16 ? m.frag_bf16 : m.frag_fp8);
        for (int i = threadIdx.x; i < kFragCount; i += blockDim.x) s.frag[i] = src[i];
        load_small_params(m.params, s.P);
        if (threadIdx.x < 6) s.sc[threadIdx.x] = SAMP == CS_SAMPLER_MLP_FP8 ? m.fp8_scales[threadIdx.x] : 1.0f;
    }
}

// The same copy in two phases for a workgroup of NT threads, so that a
// kernel can issue its global reads together with its own and wait once:
// fetch reads this thread's share into registers (every read unconditional,
// clamped into the arrays), store writes it to LDS; a barrier must follow
// before the copy is read.  Nothing to do for the other samplers.
template <int SAMP, int NT, bool MFMA = SAMP == CS_SAMPLER_MLP_BF16 || SAMP == CS_SAMPLER_MLP_FP8>
struct NetFetch {
    __device__ __forceinline__ void fetch(const MlpDev&) {}
    __device__ __forceinline__ void store(NetLds<SAMP>&) const {}
};
template <int SAMP, int NT>
struct NetFetch<SAMP, NT, true> {
    typedef typename FragT<SAMP>::type FT;
    static constexpr int kF = (kFragCount + NT - 1) / NT;
    static constexpr int kP = (kSmall + NT - 1) / NT;
    FT f[kF];
    float p[kP];
    float sc;
    __device__ __forceinline__ void fetch(const MlpDev& m) {
        const FT* src = (const FT*)(SAMP == CS_SAMPLER_MLP_BF16 ? m.frag_bf16 : m.frag_fp8);
#pragma unroll
        for (int q = 0; q < kF; ++q) {
            const int i = (int)threadIdx.x + q * NT;
            f[q] = src[i < kFragCount ? i : kFragCount - 1];
        }
#pragma unroll
        for (int q = 0; q < kP; ++q) {
            const int i = (int)threadIdx.x + q * NT;
            p[q] = m.params[small_param_src(i < kSmall ? i : kSmall - 1)];
        }
        sc = SAMP == CS_SAMPLER_MLP_FP8 ? m.fp8_scales[threadIdx.x < 6 ? threadIdx.x : 0] : 1.0f;
    }
    __device__ __forceinline__ void store(NetLds<SAMP>& s) const {
#pragma unroll
        for (int q = 0; q < kF; ++q) {
            const int i = (int)threadIdx.x + q * NT;
            if (i < kFragCount) s.frag[i] = f[q];
        }
#pragma unroll
        for (int q = 0; q < kP; ++q) {
            const int i = (int)threadIdx.x + q * NT;
            if (i < kSmall) s.P[i] = small_param_value(i, p[q]);
        }
        if (threadIdx.x < 6) s.sc[threadIdx.x] = sc;
    }
};

// The network's two outputs for every lane of the wave with need == true
// (features f1, f2 of the lane's own sample); other lanes get 0.  Must be
// called by the whole wave (converged).
template <int SAMP>
__device__ __forceinline__ float2 net_outputs(NetLds<SAMP>& s, const MlpDev& m, bool need, float f1, float f2) {
    float2 out = make_float2(0.0f, 0.0f);
    if constexpr (SAMP == CS_SAMPLER_MLP_F32) {
        if (__any(need)) out = mlp_lane_f32(m.params, s.h[wave_uniform((int)threadIdx.x >> 6)], f1, f2);
    } else if constexpr (SAMP == CS_SAMPLER_MLP_BF16 || SAMP == CS_SAMPLER_MLP_FP8) {
        // the wave's four tiles two at a time, side by side; a pair of tiles
        // none of whose samples is needed is skipped
        const int lane = lane_id();
#pragma unroll 1
        for (int tile = 0; tile < 4; tile += 2) {
            if (!__any(need && (lane >> 5) == (tile >> 1))) continue;
            float g1[2], g2[2], y0[2], y1[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int src = 16 * (tile + k) + (lane & 15);
                g1[k] = __shfl(f1, src, 64);
                g2[k] = __shfl(f2, src, 64);
            }
            mlp_tiles<SAMP, 2>(s.frag, s.P, s.sc, g1, g2, y0, y1);
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if ((lane >> 4) == tile + k) out = make_float2(y0[k], y1[k]);
        }
    }
    return need ? out : make_float2(0.0f, 0.0f);
}

}  // namespace cs
