// cs_mlp.hip -- kernels of the sampler network (2 -> 64 x4 (SiLU) -> 2).
//
// Every engine runs the hidden layers on MFMA:
//   * BF16 / FP8 inference: the tile evaluator of cs_net.h, 64-sample groups
//     per wave, the fragments and small parameters in LDS; preparation
//     kernels build the fragments (BF16 rounding, or per-layer FP8 scales
//     from the weight amax and a calibration pass of the FP32 engine);
//   * FP32 inference and calibration: the same walk with FP32 MFMA
//     (v_mfma_f32_16x16x4_f32) and the correctly rounded FP32 SiLU;
//   * training: forward and backward of 16-sample tiles on FP32 MFMA, one
//     partial gradient per workgroup, then a fixed-order sum of the partials
//     and Adam (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <cmath>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_net.h"

namespace cs {

constexpr int kMlpThreads = 256;

// SiLU and its derivative from one exponential and one division (training).
__device__ __forceinline__ void silu_and_grad(float z, float& h, float& g) {
    const float sg = 1.0f / (1.0f + expf(-z));
    h = z * sg;
    g = sg * (1.0f + z * (1.0f - sg));
}

__device__ __forceinline__ float silu_grad_f32(float z) {
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

struct FwdArgs {
    const float* P;
    NetDomain dom;
    const float *x, *u;
    int64_t n;
    float* y;      // nullable, 2n
    float* mu;     // nullable
    float* ratio;  // nullable
    uint8_t* mask; // nullable
    uint32_t* amax;  // nullable: calibration
};


// Sampler reading of the outputs (shared by every precision and by the step):
// inside the network's x range v = 1 - cos(theta) from net_reading_v, and the
// energy ratio follows from it by the Compton relation (both evaluated in
// FP64, stored as FP32); outside it the plain sampler answers.
__device__ __forceinline__ void net_out(const FwdArgs& a, int64_t i, float x, float y0, float y1) {
    const double v = net_reading_v(x, y0, y1);
    if (a.mu) a.mu[i] = (float)(1.0 - v);
    if (a.ratio) a.ratio[i] = (float)recip_approx(fma((double)x, v, 1.0));
    if (a.mask) a.mask[i] = 0;
}
__device__ __forceinline__ void fallback_out(const FwdArgs& a, int64_t i, float x, float u) {
    const double v = angle_icdf_v((double)u, (double)x);
    if (a.mu) a.mu[i] = (float)(1.0 - v);
    if (a.ratio) a.ratio[i] = (float)(1.0 / (1.0 + (double)x * v));
    if (a.mask) a.mask[i] = 1;
}
__device__ __forceinline__ void sampler_out(const FwdArgs& a, int64_t i, float x, float u, float y0, float y1) {
    if (in_range(x, a.dom))
        net_out(a, i, x, y0, y1);
    else
        fallback_out(a, i, x, u);
}

// ---------------------------------------------------------------------------
// training: forward + backward per workgroup, partial gradients
// ---------------------------------------------------------------------------
struct GradArgs {
    const float* P;
    NetDomain dom;
    const float *x, *u, *mu_t, *r_t;
    int64_t n;
    int loss;         // 0 MSE, 1 MAE
    float* partials;  // [blocks][kMlpParams]
    float* loss_partials;  // [blocks]
};

// Training on FP32 MFMA (v_mfma_f32_16x16x4_f32: lane l supplies A[l%16][l/16]
// and B[l/16][l%16]; lane l receives D[4(l/16) + r][l%16], r = 0..3).
//
// A workgroup takes tiles of 16 samples (a batch of 4096 spreads over 256
// workgroups, one per compute unit) and walks the tiles blockIdx.x,
// blockIdx.x + gridDim.x, ...  Wave w owns neurons 16w .. 16w + 15 of every
// layer: in the forward pass Z[16w.., :] = W[16w.., :] H (16 MFMAs over
// K = 64), in the backward pass the delta rows (W^T delta)[16w.., :] * SiLU'
// -- the lane that produced z keeps SiLU'(z) in registers for that --, and
// the weight gradients dW[16w.., :] = delta[16w.., :] H^T (four 16x16 tiles,
// K = 16 samples), which stay in MFMA accumulators over the workgroup's tiles
// and are written once: on the workgroup's last tile, right after the layer's
// backward pass (the stores then drain while the layers below run), and
// non-temporal (they are read once, by the reduction kernel, so they skip the
// cache rather than wait in it for the end-of-kernel write-back; with a
// 4096-sample batch, 13 MB of partials).  The workgroup first issues the loads of its first
// tile's inputs and targets (vector-memory loads complete in issue order,
// so a wait for them must not sit behind the parameter loads), then copies
// the parameters into LDS with coalesced 16-byte loads, and each lane takes
// the parameters it uses from there into registers, once for all its tiles
// (its 96 MFMA weight operands among them); each tile issues the next
// tile's input loads as soon as it has consumed its own.  Activations and
// deltas are
// written to LDS in two layouts, [feature][sample] for the operands whose
// K index is a feature and [sample][feature] (rows of kYRow) for those whose
// K index is a sample, so that every operand read is conflict-free.  Each
// gradient entry has one owner and a fixed summation order (no atomics;
// bitwise reproducible); the reduction kernel adds the workgroups' partials
// in a fixed order.
constexpr int kTrainTile = 16;
constexpr int kYRow = 80;  // [sample][feature] rows: 64 + 16 floats
// The parameters in LDS: the three 64x64 hidden matrices with rows of 68
// floats (so that the operand reads, 16 rows by 4 columns, spread over the
// banks), then the other 514 parameters packed: W1, b1, b2, b3, b4, W5, b5.
constexpr int kParRow = 68;
constexpr int kParMat = kMlpHidden * kParRow;
constexpr int kParSmall = 3 * kParMat;
constexpr int kParSW1 = 0, kParSB1 = 128, kParSB2 = 192, kParSW5 = 384, kParSB5 = 512;
constexpr int kParFloats = kParSmall + 516;

// LDS position of the 4-aligned parameter index f (below kOffB5).  Written
// with selects only: with branches, the compiler moves each of the copy's
// global loads down to its LDS store and waits for it there, fourteen memory
// round trips in a row instead of one.
__device__ __forceinline__ int par_slot(int f) {
    const int m = (f >= kOffW3) + (f >= kOffW4);       // hidden matrix W_{m+2} and its bias b_{m+2}
    const int rel = f - (kOffW2 + m * (kOffW3 - kOffW2));  // offset from the start of W_{m+2}
    const bool hidden = f >= kOffW2 && f < kOffW5;
    const int mat = m * kParMat + (rel >> 6) * kParRow + (rel & 63);
    const int bias = kParSmall + kParSB2 + kMlpHidden * m + (rel - kMlpHidden * kMlpHidden);
    const int small = f < kOffW2 ? kParSmall + f : kParSmall + kParSW5 + (f - kOffW5);  // W1, b1 | W5
    return hidden ? (rel < kMlpHidden * kMlpHidden ? mat : bias) : small;
}

typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4_t mfma_f32(float a, float b, floatx4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kMlpThreads) void k_mlp_grad_block(const GradArgs a) {
    __shared__ float4 s_par4[kParFloats / 4];             // the parameters (layout: par_slot)
    __shared__ float HX[4][kMlpHidden * kTrainTile];      // h1..h4, [feature][sample]
    __shared__ float HY[4][kTrainTile * kYRow];           // h1..h4, [sample][feature]
    __shared__ float DX[kMlpHidden * kTrainTile];         // delta of the current layer, [feature][sample]
    __shared__ float DY_[2][kTrainTile * kYRow];          // deltas, [sample][feature], ping-pong
    __shared__ float F[kTrainTile][2];                    // features
    __shared__ float dOut[kTrainTile][2];                 // output deltas
    __shared__ float s_loss[2][kTrainTile];
    __shared__ float yPart[4][2][kTrainTile];             // output-layer sums of each wave's neurons
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = wave_uniform(tid >> 6);
    const int li = lane & 15, lg = lane >> 4;  // MFMA operand row / k index of this lane
    const int64_t n_tiles = (a.n + kTrainTile - 1) / kTrainTile;
    // this thread's inputs of the first tile: features (tid < kTrainTile),
    // target (tid < 2 kTrainTile: sample tid / 2, output tid % 2)
    float in_x = 0.0f, in_u = 0.0f, in_t = 0.0f;
    auto load_inputs = [&](int64_t tile) {
        const int64_t i = tile * kTrainTile + tid;
        if (tid < kTrainTile && i < a.n) {
            in_x = a.x[i];
            in_u = a.u[i];
        }
        const int64_t it = tile * kTrainTile + (tid >> 1);
        if (tid < 2 * kTrainTile && it < a.n) in_t = (tid & 1) == 0 ? a.mu_t[it] : a.r_t[it];
    };
    if ((int64_t)blockIdx.x < n_tiles) load_inputs(blockIdx.x);
    // the parameters into LDS (12802 floats: 3200 16-byte loads and two floats)
    {
        constexpr int kN4 = kMlpParams / 4;              // 3200 16-byte pieces
        constexpr int kFull = kN4 / kMlpThreads;         // 12 rounds for every thread
        constexpr int kRest = kN4 - kFull * kMlpThreads;  // then 128 threads once more
        const float4* P4 = (const float4*)a.P;
        float4 v[kFull + 1];
        // all issued before the first store; in the last round the threads
        // past kRest repeat the piece of thread 0, and every thread stores
        // one of the two tail floats (same value, same place)
        const int last = kFull * kMlpThreads + (tid < kRest ? tid : 0);
#pragma unroll
        for (int q = 0; q < kFull; ++q) v[q] = P4[tid + q * kMlpThreads];
        v[kFull] = P4[last];
        const float tail = a.P[kN4 * 4 + (tid & 1)];
#pragma unroll
        for (int q = 0; q < kFull; ++q) s_par4[par_slot(4 * (tid + q * kMlpThreads)) / 4] = v[q];
        s_par4[par_slot(4 * last) / 4] = v[kFull];
        static_assert(kMlpParams % 4 == 2, "two tail floats");
        ((float*)s_par4)[kParSmall + kParSB5 + (tid & 1)] = tail;
        // scheduling: the fifteen global loads first, then the LDS stores
        __builtin_amdgcn_sched_group_barrier(0x0020, kFull + 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x0200, kFull + 2, 0);
    }
    __syncthreads();
    const float* P = (const float*)s_par4;
    // every parameter this lane uses, taken once for all its tiles: the
    // hidden layers' MFMA operands A = W[16w + li][4ks + lg] (forward) and
    // W^T[16w + li][4ks + lg] (backward), and for its neurons
    // n(r) = 16w + 4 lg + r the first layer, the biases and the output weights
    const int offW[3] = {kOffW2, kOffW3, kOffW4};
    float wf[3][16], wt[3][16];
#pragma unroll
    for (int L = 0; L < 3; ++L)
#pragma unroll
        for (int ks = 0; ks < 16; ++ks) {
            wf[L][ks] = P[L * kParMat + (16 * w + li) * kParRow + 4 * ks + lg];
            wt[L][ks] = P[L * kParMat + (4 * ks + lg) * kParRow + 16 * w + li];
        }
    const float* Ps = P + kParSmall;
    float w1a[4], w1b[4], bias[4][4], w50[4], w51[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int n = 16 * w + 4 * lg + r;
        w1a[r] = Ps[kParSW1 + 2 * n];
        w1b[r] = Ps[kParSW1 + 2 * n + 1];
        bias[0][r] = Ps[kParSB1 + n];
#pragma unroll
        for (int L = 0; L < 3; ++L) bias[L + 1][r] = Ps[kParSB2 + 64 * L + n];
        w50[r] = Ps[kParSW5 + n];
        w51[r] = Ps[kParSW5 + kMlpHidden + n];
    }
    // this lane's neurons of every layer: n(r) = 16w + 4 lg + r, sample li
    floatx4_t gW[3][4];  // dW_{2,3,4}[16w + 4lg + r][16tk + li], accumulated over the tiles
#pragma unroll
    for (int L = 0; L < 3; ++L)
#pragma unroll
        for (int tk = 0; tk < 4; ++tk) gW[L][tk] = {0.0f, 0.0f, 0.0f, 0.0f};
    float gB[4] = {0.0f, 0.0f, 0.0f, 0.0f};  // w == 0: db_{1..4}[lane]
    float gW1a = 0.0f, gW1b = 0.0f;          // w == 0: dW1[lane][0], dW1[lane][1]
    float gW5 = 0.0f;                        // tid < 128: dW5[tid / 64][tid % 64]
    float gB5 = 0.0f, g_loss = 0.0f;         // tid < 2: db5[tid]; tid == 2: the loss
    const float inv_n = 1.0f / (float)a.n;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        __syncthreads();  // the previous tile's LDS reads are done
        if (tid < kTrainTile) {
            const int64_t i = tile * kTrainTile + tid;
            float f1 = 0.0f, f2 = 0.0f;
            if (i < a.n) features(in_x, in_u, a.dom, f1, f2);
            F[tid][0] = f1;
            F[tid][1] = f2;
        }
        const float target = in_t;
        if (tile + gridDim.x < n_tiles) load_inputs(tile + gridDim.x);
        __syncthreads();
        float gp[4][4];  // SiLU'(z) of layers 1..4 at this lane's (neuron, sample)
        // layer 1 (2 -> 64) on the vector ALUs, in the MFMA output layout
        {
            const float f1 = F[li][0], f2 = F[li][1];
            float h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * w + 4 * lg + r;
                const float z = fmaf(w1b[r], f2, fmaf(w1a[r], f1, bias[0][r]));
                silu_and_grad(z, h[r], gp[0][r]);
                HX[0][n * kTrainTile + li] = h[r];
            }
            *(float4*)(&HY[0][li * kYRow + 16 * w + 4 * lg]) = make_float4(h[0], h[1], h[2], h[3]);
        }
        __syncthreads();
        // hidden layers 2..4: Z = W H + b on MFMA
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            floatx4_t acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = bias[L + 1][r];
            const float* hx = &HX[L][lg * kTrainTile + li];
#pragma unroll
            for (int ks = 0; ks < 16; ++ks) acc = mfma_f32(wf[L][ks], hx[4 * ks * kTrainTile], acc);
            float h[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * w + 4 * lg + r;
                silu_and_grad(acc[r], h[r], gp[L + 1][r]);
                HX[L + 1][n * kTrainTile + li] = h[r];
            }
            *(float4*)(&HY[L + 1][li * kYRow + 16 * w + 4 * lg]) = make_float4(h[0], h[1], h[2], h[3]);
            if (L == 2) {
                // output layer: this lane's four neurons of h4, then the lane
                // groups (fixed butterfly), then the waves in order below
                float q0 = 0.0f, q1 = 0.0f;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    q0 = fmaf(w50[r], h[r], q0);
                    q1 = fmaf(w51[r], h[r], q1);
                }
                q0 += __shfl_xor(q0, 16, 64);
                q1 += __shfl_xor(q1, 16, 64);
                q0 += __shfl_xor(q0, 32, 64);
                q1 += __shfl_xor(q1, 32, 64);
                if (lg == 0) {
                    yPart[w][0][li] = q0;
                    yPart[w][1][li] = q1;
                }
            }
            __syncthreads();
        }
        // output layer and loss gradient: one thread per (sample, output)
        if (tid < 2 * kTrainTile) {
            const int sm = tid >> 1, o = tid & 1;
            const int64_t i = tile * kTrainTile + sm;
            const float y = (((Ps[kParSB5 + o] + yPart[0][o][sm]) + yPart[1][o][sm]) + yPart[2][o][sm]) + yPart[3][o][sm];
            float d = 0.0f, l = 0.0f;
            if (i < a.n) {
                const float e = y - target;
                if (a.loss == 0) {
                    d = e * inv_n;
                    l = 0.5f * e * e * inv_n;
                } else {
                    d = (e > 0.0f ? 0.5f : (e < 0.0f ? -0.5f : 0.0f)) * inv_n;
                    l = 0.5f * fabsf(e) * inv_n;
                }
            }
            dOut[sm][o] = d;
            s_loss[o][sm] = l;
        }
        __syncthreads();
        if (tid == 2) {
            float acc = 0.0f;
            for (int sm = 0; sm < kTrainTile; ++sm) acc += s_loss[0][sm] + s_loss[1][sm];
            g_loss += acc;
        }
        // layer 5 gradients
        if (tid < 128) {
            const int o = tid >> 6, k = tid & 63;
            float acc = 0.0f;
            for (int sm = 0; sm < kTrainTile; ++sm) acc = fmaf(dOut[sm][o], HY[3][sm * kYRow + k], acc);
            gW5 += acc;
        } else if (tid < 130) {
            const int o = tid - 128;
            float acc = 0.0f;
            for (int sm = 0; sm < kTrainTile; ++sm) acc += dOut[sm][o];
            gB5 += acc;
        }
        // delta of layer 4: (W5^T dy) * SiLU'(z4), in this lane's layout
        float dl[4];
        {
            const float d0 = dOut[li][0], d1 = dOut[li][1];
#pragma unroll
            for (int r = 0; r < 4; ++r) dl[r] = fmaf(w50[r], d0, w51[r] * d1) * gp[3][r];
        }
        // hidden layers 4, 3, 2 (staged matrix L = 2, 1, 0): store the delta,
        // weight gradient delta H^T, delta of the layer below W^T delta
        int cur = 0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const int L = 2 - m;
            float* dy = DY_[cur];
#pragma unroll
            for (int r = 0; r < 4; ++r) DX[(16 * w + 4 * lg + r) * kTrainTile + li] = dl[r];
            *(float4*)(&dy[li * kYRow + 16 * w + 4 * lg]) = make_float4(dl[0], dl[1], dl[2], dl[3]);
            __syncthreads();
            // dW[16w + 4lg + r][16tk + li] += sum_s delta[16w + 4lg + r][s] h[16tk + li][s]
            {
                const float* hy = HY[L];  // input of this layer: h_{L+1} in 1-based terms
#pragma unroll
                for (int ks = 0; ks < 4; ++ks) {
                    const int sm = 4 * ks + lg;
                    const float aop = dy[sm * kYRow + 16 * w + li];
#pragma unroll
                    for (int tk = 0; tk < 4; ++tk) gW[L][tk] = mfma_f32(aop, hy[sm * kYRow + 16 * tk + li], gW[L][tk]);
                }
            }
            if (tile + gridDim.x >= n_tiles) {
                // the workgroup's last tile: this layer's partial is final
                float* out = a.partials + (int64_t)blockIdx.x * kMlpParams;
#pragma unroll
                for (int tk = 0; tk < 4; ++tk)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        __builtin_nontemporal_store(gW[L][tk][r],
                                                    &out[offW[L] + (16 * w + 4 * lg + r) * kMlpHidden + 16 * tk + li]);
            }
            if (w == 0) {
                float db = 0.0f;
                for (int sm = 0; sm < kTrainTile; ++sm) db += dy[sm * kYRow + lane];
                gB[L + 1] += db;
            }
            // delta below: (W^T delta)[16w + 4lg + r][li] * SiLU'(z_L)
            {
                floatx4_t acc = {0.0f, 0.0f, 0.0f, 0.0f};
                const float* dx = &DX[lg * kTrainTile + li];
#pragma unroll
                for (int ks = 0; ks < 16; ++ks) acc = mfma_f32(wt[L][ks], dx[4 * ks * kTrainTile], acc);
#pragma unroll
                for (int r = 0; r < 4; ++r) dl[r] = acc[r] * gp[L][r];
            }
            __syncthreads();  // DX and this layer's delta rows are read
            cur ^= 1;
        }
        // layer 1: dW1[j][i] = sum_s delta1[j][s] F[s][i], db1[j] = sum_s delta1[j][s]
        {
            float* dy = DY_[cur];
            *(float4*)(&dy[li * kYRow + 16 * w + 4 * lg]) = make_float4(dl[0], dl[1], dl[2], dl[3]);
            __syncthreads();
            if (w == 0) {
                float a0 = 0.0f, a1 = 0.0f, db = 0.0f;
                for (int sm = 0; sm < kTrainTile; ++sm) {
                    const float d = dy[sm * kYRow + lane];
                    a0 = fmaf(d, F[sm][0], a0);
                    a1 = fmaf(d, F[sm][1], a1);
                    db += d;
                }
                gW1a += a0;
                gW1b += a1;
                gB[0] += db;
            }
        }
    }
    // the rest of this workgroup's partial gradient (every entry by its
    // owner; the hidden matrices were written with the last tile, or here
    // as zeros by a workgroup that had no tile)
    float* out = a.partials + (int64_t)blockIdx.x * kMlpParams;
    if ((int64_t)blockIdx.x >= n_tiles) {
#pragma unroll
        for (int L = 0; L < 3; ++L)
#pragma unroll
            for (int tk = 0; tk < 4; ++tk)
#pragma unroll
                for (int r = 0; r < 4; ++r) out[offW[L] + (16 * w + 4 * lg + r) * kMlpHidden + 16 * tk + li] = gW[L][tk][r];
    }
    if (w == 0) {
        out[kOffW1 + 2 * lane] = gW1a;
        out[kOffW1 + 2 * lane + 1] = gW1b;
        out[kOffB1 + lane] = gB[0];
        out[kOffB2 + lane] = gB[1];
        out[kOffB3 + lane] = gB[2];
        out[kOffB4 + lane] = gB[3];
    }
    if (tid < 128) out[kOffW5 + tid] = gW5;
    else if (tid < 130) out[kOffB5 + tid - 128] = gB5;
    if (tid == 2) a.loss_partials[blockIdx.x] = g_loss;
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

// One workgroup of 16 waves per 64 parameters: wave w sums the partials of
// workgroups b = 16c + w (c ascending; 16 loads in flight per lane), then
// wave 0 adds the 16 wave sums in order -- a fixed summation order.  The
// loss partials the same way (lane j of wave w holds entry w + 16j, lane 0
// adds them in order).  Every global read is issued before the first sum
// that needs it, so that each costs one memory round trip.
constexpr int kReduceWaves = 16;

__global__ __launch_bounds__(64 * kReduceWaves) void k_mlp_reduce(const ReduceArgs a) {
    __shared__ float s_q[kReduceWaves][64];
    __shared__ float s_lq[kReduceWaves];
    const int lane = threadIdx.x & 63;
    const int w = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + lane;
    // this wave's loss partials, one per lane (blockIdx.x == 0)
    const int64_t lb = w + (int64_t)kReduceWaves * lane;
    const float lv = blockIdx.x == 0 && lb < a.blocks ? a.loss_partials[lb] : 0.0f;
    float g = 0.0f;
    if (p < kMlpParams) {
        int64_t b = w;
        for (; b + 15 * kReduceWaves < a.blocks; b += 16 * kReduceWaves) {
            float v[16];
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = a.partials[(b + kReduceWaves * k) * kMlpParams + p];
            __builtin_amdgcn_sched_group_barrier(0x0020, 16, 0);  // the sixteen loads first
#pragma unroll
            for (int k = 0; k < 16; ++k) g += v[k];
        }
        for (; b < a.blocks; b += kReduceWaves) g += a.partials[b * kMlpParams + p];
    }
    s_q[w][lane] = g;
    if (blockIdx.x == 0) {
        float l = 0.0f;
        for (int j = 0; w + (int64_t)kReduceWaves * j < a.blocks; ++j) l += __shfl(lv, j, 64);
        if (lane == 0) s_lq[w] = l;
    }
    __syncthreads();
    if (w != 0) return;
    if (p < kMlpParams) {
        g = s_q[0][lane];
#pragma unroll
        for (int k = 1; k < kReduceWaves; ++k) g += s_q[k][lane];
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
    if (blockIdx.x == 0 && lane == 0 && a.loss_out) {
        float l = s_lq[0];
        for (int k = 1; k < kReduceWaves; ++k) l += s_lq[k];
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
        features(x, u, m.dom, f1, f2);
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
        if (sampling && active && in_range(x, m.dom)) net_out(a, i, x, o0, o1);
    }
    if (!sampling) return;
    int64_t* fb = s_fb[wave];
    int nfb = 0;  // wave-uniform
    for (int64_t grp = first; grp < n_groups; grp += stride) {
        const int64_t i = grp * 64 + lane;
        const bool defer = i < a.n && !in_range(a.x[i], m.dom);
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
// FP32 inference on MFMA (v_mfma_f32_16x16x4_f32)
// ---------------------------------------------------------------------------
// The layout of the reduced-precision engine (lane l owns sample l % 16 and
// neurons 16t + 4g + r of a 16-sample tile, g = l / 16), with the K index of
// each layer's contraction permuted so that every lane's B operand is one of
// its own outputs of the previous layer: k-step (t, r) pairs lane group g
// with input neuron 16t + 4g + r, so the A operand of lane l at (output tile
// T, k-step (t, r)) is W[16T + l % 16][16t + 4 (l / 16) + r].  These
// fragments (3 layers x 4 x 16 x 64 floats, 48 KB) are built in LDS by each
// workgroup.  SiLU is the correctly rounded FP32 one; the first and last
// layers run on the vector ALUs as in the other engine.
constexpr int kF32Frag = 3 * 4 * 16 * 64;

struct F32Lds {
    float frag[kF32Frag];
    float P[kSmall];  // W1, b1..b4, W5, b5 (unscaled)
};

__device__ __forceinline__ void f32_lds_load(F32Lds& s, const float* P) {
    const int offW[3] = {kOffW2, kOffW3, kOffW4};
    for (int i = threadIdx.x; i < kF32Frag; i += blockDim.x) {
        const int l = i & 63, rr = (i >> 6) & 3, t = (i >> 8) & 3, T = (i >> 10) & 3, L = i >> 12;
        s.frag[i] = P[offW[L] + (16 * T + (l & 15)) * kMlpHidden + 16 * t + 4 * (l >> 4) + rr];
    }
    for (int i = threadIdx.x; i < kSmall; i += blockDim.x) {
        int src;
        if (i < cB1)
            src = kOffW1 + i;
        else if (i < cB2)
            src = kOffB1 + (i - cB1);
        else if (i < cB3)
            src = kOffB2 + (i - cB2);
        else if (i < cB4)
            src = kOffB3 + (i - cB3);
        else if (i < cW5)
            src = kOffB4 + (i - cB4);
        else if (i < cB5)
            src = kOffW5 + (i - cW5);
        else
            src = kOffB5 + (i - cB5);
        s.P[i] = P[src];
    }
}

// NTL tiles side by side; amax (nullable): this lane's running max |h| of the
// inputs of hidden layers 2..4, over the tiles k whose sample is real[k].
template <int NTL>
__device__ __forceinline__ void mlp_tiles_f32(const float* frag, const float* Ps, const float (&f1)[NTL],
                                              const float (&f2)[NTL], float (&y0)[NTL], float (&y1)[NTL],
                                              float* amax, const bool (&real)[NTL]) {
    const int lane = lane_id();
    const int g = lane >> 4;
    float h[NTL][16];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = 16 * t + 4 * g + r;
            const float w1a = Ps[cW1 + 2 * n], w1b = Ps[cW1 + 2 * n + 1], b1 = Ps[cB1 + n];
#pragma unroll
            for (int k = 0; k < NTL; ++k) {
                h[k][4 * t + r] = silu_f32(fmaf(w1b, f2[k], fmaf(w1a, f1[k], b1)));
                if (amax && real[k]) amax[0] = fmaxf(amax[0], fabsf(h[k][4 * t + r]));
            }
        }
    const int offB[3] = {cB2, cB3, cB4};
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        float o[NTL][16];
#pragma unroll
        for (int T = 0; T < 4; ++T) {
            floatx4 acc[NTL];
#pragma unroll
            for (int k = 0; k < NTL; ++k)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[k][r] = Ps[offB[L] + 16 * T + 4 * g + r];
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                const float A = frag[((L * 4 + T) * 16 + q) * 64 + lane];
#pragma unroll
                for (int k = 0; k < NTL; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x4f32(A, h[k][q], acc[k], 0, 0, 0);
            }
#pragma unroll
            for (int k = 0; k < NTL; ++k)
#pragma unroll
                for (int r = 0; r < 4; ++r) o[k][4 * T + r] = silu_f32(acc[k][r]);
        }
#pragma unroll
        for (int k = 0; k < NTL; ++k)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                h[k][j] = o[k][j];
                if (amax && L < 2 && real[k]) amax[L + 1] = fmaxf(amax[L + 1], fabsf(o[k][j]));
            }
    }
#pragma unroll
    for (int k = 0; k < NTL; ++k) {
        float p0 = 0.0f, p1 = 0.0f;
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int n = 16 * t + 4 * g + r;
                p0 = fmaf(Ps[cW5 + n], h[k][4 * t + r], p0);
                p1 = fmaf(Ps[cW5 + kMlpHidden + n], h[k][4 * t + r], p1);
            }
        p0 += __shfl_xor(p0, 16, 64);
        p1 += __shfl_xor(p1, 16, 64);
        p0 += __shfl_xor(p0, 32, 64);
        p1 += __shfl_xor(p1, 32, 64);
        y0[k] = p0 + Ps[cB5];
        y1[k] = p1 + Ps[cB5 + 1];
    }
}

// FP32 forward / sampler / calibration: the walk of k_mlp_mfma (64-sample
// groups per wave, the out-of-domain samples in a second walk), two tiles
// side by side.
__global__ __launch_bounds__(kMfmaThreads, 2) void k_mlp_f32(const FwdArgs a) {
    __shared__ F32Lds s_net;
    __shared__ int64_t s_fb[kMfmaThreads / 64][kFbCap];
    f32_lds_load(s_net, a.P);
    __syncthreads();
    const int lane = lane_id();
    const int wave = wave_uniform((int)threadIdx.x >> 6);
    const bool sampling = a.mu || a.ratio || a.mask;
    const int64_t n_groups = (a.n + 63) / 64;
    const int64_t first = (int64_t)blockIdx.x * (kMfmaThreads / 64) + wave;
    const int64_t stride = (int64_t)gridDim.x * (kMfmaThreads / 64);
    float amax[3] = {0.0f, 0.0f, 0.0f};
    for (int64_t grp = first; grp < n_groups; grp += stride) {
        const int64_t i = grp * 64 + lane;
        const bool active = i < a.n;
        const float x = active ? a.x[i] : 1.0f, u = active ? a.u[i] : 0.5f;
        float f1, f2;
        features(x, u, a.dom, f1, f2);
        int opaque = 0;
        asm volatile("" : "+s"(opaque));
        const float* frag = s_net.frag + opaque;
        const float* Ps = s_net.P + opaque;
        float o0 = 0.0f, o1 = 0.0f;
#pragma unroll
        for (int t0 = 0; t0 < 4; t0 += 2) {
            float g1[2], g2[2], y0[2], y1[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int src = 16 * (t0 + k) + (lane & 15);
                g1[k] = __shfl(f1, src, 64);
                g2[k] = __shfl(f2, src, 64);
            }
            // calibration counts only the group's real samples: lane (g, li)
            // of tile t0 + k evaluates sample 16 (t0 + k) + li of the group
            const bool real[2] = {grp * 64 + 16 * t0 + (lane & 15) < a.n,
                                  grp * 64 + 16 * (t0 + 1) + (lane & 15) < a.n};
            mlp_tiles_f32<2>(frag, Ps, g1, g2, y0, y1, a.amax ? amax : nullptr, real);
#pragma unroll
            for (int k = 0; k < 2; ++k)
                if ((lane >> 4) == t0 + k) {
                    o0 = y0[k];
                    o1 = y1[k];
                }
        }
        if (active && a.y) *(float2*)(a.y + 2 * i) = make_float2(o0, o1);
        if (sampling && active && in_range(x, a.dom)) net_out(a, i, x, o0, o1);
    }
    if (a.amax) {
        // non-negative floats order as their bits
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            float wm = amax[L];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) wm = fmaxf(wm, __shfl_xor(wm, off, 64));
            if (lane == 0) atomicMax(&a.amax[L], __float_as_uint(wm));
        }
    }
    if (!sampling) return;
    int64_t* fb = s_fb[wave];
    int nfb = 0;
    for (int64_t grp = first; grp < n_groups; grp += stride) {
        const int64_t i = grp * 64 + lane;
        const bool defer = i < a.n && !in_range(a.x[i], a.dom);
        const uint64_t msk = __ballot(defer);
        if (msk == 0) continue;
        if (defer) fb[nfb + __popcll(msk & ((1ull << lane) - 1ull))] = i;
        nfb += __popcll(msk);
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
// Feature constants of a network's x range (see NetDomain).
NetDomain net_domain(double x_min, double x_max) {
    const double lo = std::log10(x_min), hi = std::log10(x_max);
    const double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo);
    NetDomain d;
    d.f_a = (float)(std::log10(2.0) / h);
    d.f_b = (float)(-c / h);
    d.x_lo = (float)x_min;
    d.x_hi = (float)x_max;
    return d;
}

constexpr int64_t kMaxGradBlocks = 512;
static_assert(kMaxGradBlocks <= 64 * kReduceWaves, "k_mlp_reduce holds one loss partial per lane");

int64_t mlp_grad_blocks(int64_t n) {
    const int64_t t = (n + kTrainTile - 1) / kTrainTile;
    return t < kMaxGradBlocks ? t : kMaxGradBlocks;
}

hipError_t launch_mlp_forward(const MlpDev& m, cs_sampler prec, const float* x, const float* u, int64_t n, float* y,
                              float* mu, float* ratio, uint8_t* mask, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    FwdArgs a = {m.params, m.dom, x, u, n, y, mu, ratio, mask, nullptr};
    if (prec == CS_SAMPLER_MLP_F32) {
        const int64_t groups = (n + 63) / 64;
        int64_t blocks = (groups + kMfmaThreads / 64 - 1) / (kMfmaThreads / 64);
        if (blocks > 1024) blocks = 1024;
        k_mlp_f32<<<(unsigned)blocks, kMfmaThreads, 0, st>>>(a);
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
    GradArgs g = {m.params, m.dom, x, u, mu_t, r_t, n, loss, partials, loss_partials};
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
    k_mlp_reduce<<<(kMlpParams + 63) / 64, 64 * kReduceWaves, 0, st>>>(r);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* params, float* m, float* v, const float* grad, float lr, int64_t t, hipStream_t st) {
    const float bc1 = (float)(1.0 - std::pow(0.9, (double)t));
    const float bc2 = (float)(1.0 - std::pow(0.999, (double)t));
    k_mlp_adam_only<<<(kMlpParams + 255) / 256, 256, 0, st>>>(params, m, v, grad, lr, bc1, bc2);
    return hipGetLastError();
}

hipError_t launch_mlp_quantize(float* params, const NetDomain& dom, void* frag_bf16, void* frag_fp8, float* scales,
                               cs_sampler prec, const float* cx, const float* cu, int64_t n, hipStream_t st) {
    const unsigned nb = (kFragCount * 8 + 255) / 256;
    if (prec == CS_SAMPLER_MLP_BF16) {
        k_mlp_build_frag<<<nb, 256, 0, st>>>(params, scales, CS_SAMPLER_MLP_BF16, (__bf16*)frag_bf16, nullptr);
    } else {
        k_mlp_zero_amax<<<1, 64, 0, st>>>((uint32_t*)scales + 6);
        FwdArgs a = {params, dom, cx, cu, n, nullptr, nullptr, nullptr, nullptr, (uint32_t*)scales + 6};
        const int64_t groups = (n + 63) / 64;
        int64_t blocks = (groups + kMfmaThreads / 64 - 1) / (kMfmaThreads / 64);
        if (blocks > 1024) blocks = 1024;
        k_mlp_f32<<<(unsigned)blocks, kMfmaThreads, 0, st>>>(a);
        k_mlp_act_scale<<<1, 64, 0, st>>>(scales);
        k_mlp_weight_scale<<<3, 256, 0, st>>>(params, scales);
        k_mlp_build_frag<<<nb, 256, 0, st>>>(params, scales, CS_SAMPLER_MLP_FP8, nullptr, (uint8_t*)frag_fp8);
    }
    return hipGetLastError();
}

}  // namespace cs
