// cs_block.h -- wavefront (64-lane) and workgroup primitives for gfx950:
// scans, fixed-order reductions.  Every reduction here has an order fixed by
// the lane and wave indices, so results are bitwise reproducible.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cs {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ int wave_inclusive_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(v, off, 64);
        if (lane >= off) v += t;
    }
    return v;
}

// Exclusive scan across the block; `lds` holds >= blockDim/64 ints.
__device__ __forceinline__ int block_exclusive_scan(int v, int* lds, int* total) {
    const int lane = lane_id();
    const int wave = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    const int inc = wave_inclusive_scan(v);
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        int w = lane < nw ? lds[lane] : 0;
        const int ws = wave_inclusive_scan(w);
        if (lane < nw) lds[lane] = ws - w;  // exclusive wave offsets
        if (lane == nw - 1) lds[nw] = ws;
    }
    __syncthreads();
    const int res = lds[wave] + inc - v;
    if (total) *total = lds[nw];
    __syncthreads();
    return res;
}

// Fixed-order tree sum of one double per thread (blockDim a power of two).
__device__ __forceinline__ double block_sum(double v, double* lds) {
    const int tid = threadIdx.x;
    lds[tid] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (tid < s) lds[tid] += lds[tid + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

__device__ __forceinline__ long long block_sum_i(long long v, long long* lds) {
    const int tid = threadIdx.x;
    lds[tid] = v;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
        if (tid < s) lds[tid] += lds[tid + s];
        __syncthreads();
    }
    const long long r = lds[0];
    __syncthreads();
    return r;
}

// Fixed-order butterfly sum over the 64 lanes of a wave (every lane gets it).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ long long wave_sum_i(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace cs
