// cs_pnet.hip -- the paper's own learned component (Sec. 3.2): a small dense
// network that predicts, for a candidate lepton-photon pair, the probability
// of interaction against the cell's majorant, y' = P / P_max, in place of the
// analytic Klein-Nishina evaluation.
//
// Nine inputs per pair (FP32 rows): photon momentum k (3), lepton momentum p
// (3), P_max, w_e, w_g.  Widths 9 -> 9 -> 12 -> 9 -> 1, ReLU hidden layers
// (ReLU'(0) = 0), sigmoid output.  Parameters: per layer W[n_out][n_in]
// row-major, then b[n_out] (337 floats).  FP32 arithmetic, one pair per lane
// (the layers are far too narrow for matrix-core tiles).
//
//   k_pnet_target     y = P / P_max = s(x) (1 - beta . k_hat) / 2 in FP64
//                     (the training target and the analytic reference)
//   k_pnet_fwd        y' per pair
//   k_pnet_grad_block forward and backward per pair; each parameter's
//                     contributions summed over the wave (fixed butterfly),
//                     then over the workgroup's waves, into per-workgroup
//                     partials
//   k_pnet_reduce     fixed-order sum of the partials over the workgroups,
//                     divided by n (gradient of the mean loss) and the loss
//   k_pnet_adam       one Adam step (Kingma & Ba; bias corrections from the
//                     host)
#include <hip/hip_runtime.h>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"

namespace cs {

constexpr int kPnetThreads = 256;
// parameter offsets of the four layers
constexpr int kW1 = 0, kB1 = 81, kW2 = 90, kB2 = 198, kW3 = 210, kB3 = 318, kW4 = 327, kB4 = 336;
constexpr int kPnetParams = 337;
constexpr int kPnetPart = kPnetParams + 1;  // per-workgroup partials: the gradient, then the loss

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(kPnetThreads) void k_pnet_target(const float* in, int64_t n, float* y) {
    const int64_t i = (int64_t)blockIdx.x * kPnetThreads + threadIdx.x;
    if (i >= n) return;
    const float* r = in + 9 * i;
    const d3 k = {(double)r[0], (double)r[1], (double)r[2]};
    const d3 p = {(double)r[3], (double)r[4], (double)r[5]};
    const XFlux xf = x_flux(p, k, dot(p, p), dot(k, k));
    y[i] = xf.x > 0.0 ? (float)(0.5 * sigma_ratio(xf.x) * xf.flux) : 0.0f;
}

// The forward pass of one pair from LDS parameters P: pre-activations and
// activations kept for the backward pass.
struct PnetActs {
    float a0[9], z1[9], a1[9], z2[12], a2[12], z3[9], a3[9];
    float y;
};

__device__ __forceinline__ void pnet_forward(const float* P, const float* x, PnetActs& s) {
#pragma unroll
    for (int q = 0; q < 9; ++q) s.a0[q] = x[q];
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        float z = P[kB1 + m];
#pragma unroll
        for (int q = 0; q < 9; ++q) z = fmaf(P[kW1 + 9 * m + q], s.a0[q], z);
        s.z1[m] = z;
        s.a1[m] = fmaxf(z, 0.0f);
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) {
        float z = P[kB2 + i];
#pragma unroll
        for (int m = 0; m < 9; ++m) z = fmaf(P[kW2 + 9 * i + m], s.a1[m], z);
        s.z2[i] = z;
        s.a2[i] = fmaxf(z, 0.0f);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        float z = P[kB3 + j];
#pragma unroll
        for (int i = 0; i < 12; ++i) z = fmaf(P[kW3 + 12 * j + i], s.a2[i], z);
        s.z3[j] = z;
        s.a3[j] = fmaxf(z, 0.0f);
    }
    float z = P[kB4];
#pragma unroll
    for (int j = 0; j < 9; ++j) z = fmaf(P[kW4 + j], s.a3[j], z);
    s.y = 1.0f / (1.0f + expf(-z));
}

__device__ __forceinline__ void load_pnet_params(const float* params, float* s_p) {
    for (int q = threadIdx.x; q < kPnetParams; q += blockDim.x) s_p[q] = params[q];
    __syncthreads();
}

__global__ __launch_bounds__(kPnetThreads) void k_pnet_fwd(const float* params, const float* in, int64_t n,
                                                         float* y) {
    __shared__ float s_p[kPnetParams];
    load_pnet_params(params, s_p);
    const int64_t i = (int64_t)blockIdx.x * kPnetThreads + threadIdx.x;
    if (i >= n) return;
    float x[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) x[q] = in[9 * i + q];
    PnetActs s;
    pnet_forward(s_p, x, s);
    y[i] = s.y;
}

__global__ __launch_bounds__(kPnetThreads) void k_pnet_grad_block(const float* params, const float* in,
                                                                const float* target, int64_t n, int mae,
                                                                float* partials) {
    __shared__ float s_p[kPnetParams];
    __shared__ float s_part[kPnetThreads / 64][kPnetPart];
    load_pnet_params(params, s_p);
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int64_t i = (int64_t)blockIdx.x * kPnetThreads + tid;
    const bool act = i < n;
    float x[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) x[q] = act ? in[9 * i + q] : 0.0f;
    PnetActs s;
    pnet_forward(s_p, x, s);
    const float e = act ? s.y - target[i] : 0.0f;
    const float dy = mae ? (e > 0.0f ? 1.0f : (e < 0.0f ? -1.0f : 0.0f)) : e;
    const float lossv = mae ? fabsf(e) : 0.5f * e * e;
    // backward (per pair; the 1/n of the mean is applied by k_pnet_reduce)
    const float d4 = dy * s.y * (1.0f - s.y);
    float d3[9], d2[12], d1[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) d3[j] = s.z3[j] > 0.0f ? d4 * s_p[kW4 + j] : 0.0f;
#pragma unroll
    for (int i2 = 0; i2 < 12; ++i2) {
        float t = 0.0f;
#pragma unroll
        for (int j = 0; j < 9; ++j) t = fmaf(s_p[kW3 + 12 * j + i2], d3[j], t);
        d2[i2] = s.z2[i2] > 0.0f ? t : 0.0f;
    }
#pragma unroll
    for (int m = 0; m < 9; ++m) {
        float t = 0.0f;
#pragma unroll
        for (int i2 = 0; i2 < 12; ++i2) t = fmaf(s_p[kW2 + 9 * i2 + m], d2[i2], t);
        d1[m] = s.z1[m] > 0.0f ? t : 0.0f;
    }
    // each parameter's contribution, summed over the wave; lane 0 keeps it
    auto put = [&](int q, float g) {
        const float w = wave_sum_f(g);
        if (lane == 0) s_part[wave][q] = w;
    };
#pragma unroll
    for (int m = 0; m < 9; ++m) {
#pragma unroll
        for (int q = 0; q < 9; ++q) put(kW1 + 9 * m + q, d1[m] * s.a0[q]);
        put(kB1 + m, d1[m]);
    }
#pragma unroll
    for (int i2 = 0; i2 < 12; ++i2) {
#pragma unroll
        for (int m = 0; m < 9; ++m) put(kW2 + 9 * i2 + m, d2[i2] * s.a1[m]);
        put(kB2 + i2, d2[i2]);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) {
#pragma unroll
        for (int i2 = 0; i2 < 12; ++i2) put(kW3 + 12 * j + i2, d3[j] * s.a2[i2]);
        put(kB3 + j, d3[j]);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) put(kW4 + j, d4 * s.a3[j]);
    put(kB4, d4);
    put(kPnetParams, lossv);
    __syncthreads();
    for (int q = tid; q < kPnetPart; q += kPnetThreads) {
        float t = 0.0f;
#pragma unroll
        for (int w = 0; w < kPnetThreads / 64; ++w) t += s_part[w][q];
        partials[(int64_t)blockIdx.x * kPnetPart + q] = t;
    }
}

__global__ __launch_bounds__(kPnetThreads) void k_pnet_reduce(const float* partials, int64_t n_blocks, int64_t n,
                                                            float* grad, float* loss) {
    const int q = blockIdx.x * kPnetThreads + threadIdx.x;
    if (q >= kPnetPart) return;
    float t = 0.0f;
    for (int64_t b = 0; b < n_blocks; ++b) t += partials[b * kPnetPart + q];
    const float v = n > 0 ? t / (float)n : 0.0f;
    if (q < kPnetParams)
        grad[q] = v;
    else if (loss)
        *loss = v;
}

__global__ __launch_bounds__(kPnetThreads) void k_pnet_adam(float* params, const float* grad, float* m_, float* v_,
                                                          float lr, float bc1, float bc2) {
    const int q = blockIdx.x * kPnetThreads + threadIdx.x;
    if (q >= kPnetParams) return;
    const float g = grad[q];
    const float m = 0.9f * m_[q] + 0.1f * g;
    const float v = 0.999f * v_[q] + 0.001f * g * g;
    m_[q] = m;
    v_[q] = v;
    params[q] -= lr * (m / bc1) / (sqrtf(v / bc2) + 1e-8f);
}

size_t pnet_workspace_bytes(int64_t n) {
    const int64_t nb = n > 0 ? (n + kPnetThreads - 1) / kPnetThreads : 1;
    return sizeof(float) * (size_t)nb * kPnetPart;
}

hipError_t launch_pnet_target(const float* in, int64_t n, float* y, hipStream_t st) {
    if (n > 0) k_pnet_target<<<(unsigned)((n + kPnetThreads - 1) / kPnetThreads), kPnetThreads, 0, st>>>(in, n, y);
    return hipGetLastError();
}

hipError_t launch_pnet_forward(const float* params, const float* in, int64_t n, float* y, hipStream_t st) {
    if (n > 0)
        k_pnet_fwd<<<(unsigned)((n + kPnetThreads - 1) / kPnetThreads), kPnetThreads, 0, st>>>(params, in, n, y);
    return hipGetLastError();
}

hipError_t launch_pnet_grad(const float* params, const float* in, const float* target, int64_t n, int mae,
                            float* grad, float* loss, void* ws, hipStream_t st) {
    const int64_t nb = n > 0 ? (n + kPnetThreads - 1) / kPnetThreads : 0;
    float* part = (float*)ws;
    if (nb > 0) k_pnet_grad_block<<<(unsigned)nb, kPnetThreads, 0, st>>>(params, in, target, n, mae, part);
    k_pnet_reduce<<<(kPnetPart + kPnetThreads - 1) / kPnetThreads, kPnetThreads, 0, st>>>(part, nb, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_pnet_adam(float* params, const float* grad, float* m, float* v, float lr, float bc1, float bc2,
                            hipStream_t st) {
    k_pnet_adam<<<(kPnetParams + kPnetThreads - 1) / kPnetThreads, kPnetThreads, 0, st>>>(params, grad, m, v, lr,
                                                                                        bc1, bc2);
    return hipGetLastError();
}

}  // namespace cs
