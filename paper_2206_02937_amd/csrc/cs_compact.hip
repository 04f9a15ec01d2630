// cs_compact.hip -- the step as four kernels (default strategy):
//
//   k_prep_scan       (cs_fused.hip) cells -> pair offsets, keys, chunk map
//   k_pair_compact    one lane per pair, one workgroup per 256-pair chunk:
//                     pairing, x, s(x), P, accept; the accepted pairs of the
//                     chunk get their global position by decoupled look-back
//                     over the chunks, so the list of accepted pairs is dense
//                     and in pair order with no atomics.  Lean (no sampler),
//                     so it runs at full occupancy.
//   k_collide_dense   workgroups stride over the dense list: sample the
//                     angle, scatter, write back (one wave per workgroup with
//                     the plain sampler; four waves sharing the network's LDS
//                     copy with a network sampler).
//   k_finalize_step   (cs_fused.hip) fixed-order reduction of the partial sums.
#include <hip/hip_runtime.h>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_lookback.h"
#include "cs_pair.h"

namespace cs {

constexpr int kDenseThreads = 64;      // plain sampler
constexpr int kDenseNetThreads = 256;  // network samplers

template <typename T>
struct CompactArgs {
    Particles<T> pt;
    const int64_t *off_e, *off_g;
    int64_t n_cells, n_chunks;
    const int32_t* pair_off;
    const uint32_t* keys;
    const int32_t* chunk_cell;
    double dt, density_norm;
    uint64_t seed;
    StepControl* ctrl;
    uint64_t* status;  // one word per chunk
    int2* list;
    double* chunk_prob;
    int64_t* chunk_clip;
    int64_t* chunk_inv;
    double* coll_eb;
    double* coll_ea;
    int64_t* coll_fb;
    cs_stats* stats;
    MlpDev mlp;
};

// One workgroup takes PPL consecutive 256-pair chunks, one pair of each per
// lane.  The phases run for all PPL pairs before the next phase starts --
// find the cell, read its offsets and key; pair; read the particles; the
// physics -- so that each lane has PPL independent memory accesses in flight
// instead of one.  The accepted pairs of the PPL chunks (in pair order) take
// their place in the global list with one look-back per workgroup.
template <typename T, int PPL>
__global__ __launch_bounds__(kChunk) void k_pair_compact(const CompactArgs<T> a) {
    __shared__ int s_wcnt[PPL][kChunk / 64];
    __shared__ int s_prefix;
    __shared__ double s_rd[kChunk / 64];
    __shared__ long long s_ri[2 * (kChunk / 64)];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int64_t blk = blockIdx.x;
    StepControl* ctrl = a.ctrl;
    const uint32_t E = ctrl->epoch;
    const uint64_t step = ctrl->step;
    const bool layout_ok = ctrl->layout_epoch != E && ctrl->scan_fault_epoch != E;
    const int32_t T_total = layout_ok ? a.pair_off[a.n_cells] : 0;
    // phase 1: cell of each pair (binary search over the chunk's cells),
    // then the cell's particle ranges and pairing key
    int32_t t[PPL];
    int c[PPL];
    bool act[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const int64_t j = blk * PPL + q;
        t[q] = (int32_t)(j * kChunk) + tid;
        act[q] = j < a.n_chunks && t[q] < T_total;
        c[q] = 0;
        if (act[q]) {
            int lo = a.chunk_cell[j], hi = a.chunk_cell[j + 1];
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (a.pair_off[mid] <= t[q])
                    lo = mid;
                else
                    hi = mid - 1;
            }
            c[q] = lo;
        }
    }
    int64_t e0[PPL], e1[PPL], g0[PPL], g1[PPL];
    uint4 key[PPL];
    int32_t po[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        e0[q] = e1[q] = g0[q] = g1[q] = 0;
        key[q] = make_uint4(0, 0, 0, 0);
        po[q] = 0;
        if (act[q]) {
            e0[q] = a.off_e[c[q]];
            e1[q] = a.off_e[c[q] + 1];
            g0[q] = a.off_g[c[q]];
            g1[q] = a.off_g[c[q] + 1];
            key[q] = *(const uint4*)(a.keys + 4 * c[q]);
            po[q] = a.pair_off[c[q]];
        }
    }
    // phase 2: pairing and the particle reads
    PairSlot sl[PPL];
    PairRaw<T> raw[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q)
        sl[q] = pair_index(act[q], e0[q], e1[q], g0[q], g1[q], key[q].x, key[q].y, key[q].z, key[q].w,
                           (uint32_t)(t[q] - po[q]));
#pragma unroll
    for (int q = 0; q < PPL; ++q) raw[q] = pair_load<T>(a.pt, sl[q]);
    // phase 3: physics, per-chunk ballots
    double sum_p = 0.0;
    long long n_clip = 0, n_inv = 0;
    bool acc[PPL];
    int before[PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const PairOutcome o = pair_physics<T>(sl[q], raw[q], a.dt, a.density_norm, a.seed, step);
        sum_p += o.P;
        n_clip += o.clipped ? 1 : 0;
        n_inv += o.invalid ? 1 : 0;
        acc[q] = o.accept;
        const uint64_t mask = __ballot(o.accept);
        before[q] = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) s_wcnt[q][wave] = __popcll(mask);
    }
    const double wp = wave_sum(sum_p);
    const long long wc = wave_sum_i(n_clip), wi = wave_sum_i(n_inv);
    if (lane == 0) {
        s_rd[wave] = wp;
        s_ri[2 * wave] = wc;
        s_ri[2 * wave + 1] = wi;
    }
    __syncthreads();
    // position of this lane's accepted pairs within the workgroup's list:
    // chunk-major, then wave, then lane (pair order)
    int base[PPL];
    int total = 0;
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        int wb = 0, tq = 0;
#pragma unroll
        for (int w = 0; w < kChunk / 64; ++w) {
            wb += w < wave ? s_wcnt[q][w] : 0;
            tq += s_wcnt[q][w];
        }
        base[q] = total + wb + before[q];
        total += tq;
    }
    if (tid < 64) {
        const uint32_t ex = lookback_exclusive_wave(a.status, blk, E, (uint32_t)total, &ctrl->scan_fault_epoch);
        if (tid == 0) s_prefix = (int)ex;
    }
    if (tid == 0) {
        double p = 0.0;
        long long cl = 0, in = 0;
        for (int w = 0; w < kChunk / 64; ++w) {
            p += s_rd[w];
            cl += s_ri[2 * w];
            in += s_ri[2 * w + 1];
        }
        a.chunk_prob[blk] = p;
        a.chunk_clip[blk] = cl;
        a.chunk_inv[blk] = in;
    }
    __syncthreads();
    const int prefix = s_prefix;
#pragma unroll
    for (int q = 0; q < PPL; ++q)
        if (acc[q]) a.list[prefix + base[q]] = make_int2(sl[q].ie, sl[q].ig);
    if (tid == 0 && blk == (int64_t)gridDim.x - 1) ctrl->n_accepted = (uint32_t)(prefix + total);
}

// Network samplers defer the pairs outside the network's domain: their list
// positions are compacted in order into s_fb and resolved with the plain
// sampler in dense passes once a full workgroup's worth has gathered (and at
// the end), so that the Newton iteration never runs on a mostly idle wave.
template <typename T, int SAMP>
__global__ __launch_bounds__(SAMP == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads) void k_collide_dense(
    const CompactArgs<T> a) {
    constexpr int NT = SAMP == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads;
    constexpr bool NET = SAMP != CS_SAMPLER_PLAIN;
    __shared__ NetLds<SAMP> s_net;
    __shared__ double s_d[2 * (NT / 64)];
    __shared__ long long s_fbc[NT / 64];
    __shared__ int s_fb[NET ? 2 * NT : 1];
    __shared__ int s_wcnt[NT / 64];
    __shared__ int s_fbn;
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    net_load<SAMP>(s_net, a.mlp);
    if constexpr (NET) {
        if (tid == 0) s_fbn = 0;
        __syncthreads();
    }
    StepControl* ctrl = a.ctrl;
    const uint32_t E = ctrl->epoch;
    const uint64_t step = ctrl->step;
    const bool layout_ok = ctrl->layout_epoch != E && ctrl->scan_fault_epoch != E;
    const int64_t A = layout_ok ? (int64_t)ctrl->n_accepted : 0;
    const int64_t stride = (int64_t)gridDim.x * NT;
    const int64_t n_iter = (A + stride - 1) / stride;  // uniform over the grid
    CollideSums sums;
    // dense plain-sampler passes over the deferred list positions
    auto flush = [&](int n) {
        for (int base = 0; base < n; base += NT) {
            const int q2 = base + tid;
            if (__any(q2 < n)) {
                const bool act = q2 < n;
                const int2 pr = act ? a.list[s_fb[q2]] : make_int2(0, 0);
                collide_plain<T>(a.pt, act, pr.x, pr.y, a.seed, step, sums);
                sums.n_fallback += act ? 1 : 0;
            }
        }
    };
    for (int64_t it = 0; it < n_iter; ++it) {
        const int64_t q = it * stride + (int64_t)blockIdx.x * NT + tid;
        const bool active = q < A;
        if constexpr (!NET) {
            if (!__any(active)) break;
            const int2 pr = active ? a.list[q] : make_int2(0, 0);
            collide_plain<T>(a.pt, active, pr.x, pr.y, a.seed, step, sums);
        } else {
            // every wave takes part in every iteration (barriers below)
            const int2 pr = active ? a.list[q] : make_int2(0, 0);
            const bool defer =
                collide_net<T, SAMP, true>(a.pt, active, FromArrays<T>{pr.x, pr.y}, s_net, a.mlp, a.seed, step, sums);
            const uint64_t m = __ballot(defer);
            if (lane == 0) s_wcnt[wave] = __popcll(m);
            __syncthreads();
            int wbase = 0, total = 0;
#pragma unroll
            for (int w = 0; w < NT / 64; ++w) {
                wbase += w < wave ? s_wcnt[w] : 0;
                total += s_wcnt[w];
            }
            const int nf = s_fbn;  // < NT here, so nf + total < 2 NT
            if (defer) s_fb[nf + wbase + __popcll(m & ((1ull << lane) - 1ull))] = (int)q;
            __syncthreads();
            if (nf + total >= NT) {
                flush(nf + total);
                __syncthreads();
                if (tid == 0) s_fbn = 0;
            } else if (tid == 0) {
                s_fbn = nf + total;
            }
            __syncthreads();
        }
    }
    if constexpr (NET) flush(s_fbn);
    const double eb = wave_sum(sums.e_before), ea = wave_sum(sums.e_after);
    const long long fb = wave_sum_i(sums.n_fallback);
    if (lane == 0) {
        s_d[2 * wave] = eb;
        s_d[2 * wave + 1] = ea;
        s_fbc[wave] = fb;
    }
    __syncthreads();
    if (tid == 0) {
        double teb = 0.0, tea = 0.0;
        long long tfb = 0;
        for (int w = 0; w < NT / 64; ++w) {
            teb += s_d[2 * w];
            tea += s_d[2 * w + 1];
            tfb += s_fbc[w];
        }
        a.coll_eb[blockIdx.x] = teb;
        a.coll_ea[blockIdx.x] = tea;
        a.coll_fb[blockIdx.x] = tfb;
    }
}

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

int64_t compact_pair_blocks(const StepShape& s) {
    const int64_t ppl = s.pairs_per_lane;
    return s.n_chunks > 0 ? (s.n_chunks + ppl - 1) / ppl : 0;
}

size_t compact_workspace_bytes(const StepShape& s) {
    size_t b = 0;
    b += al(sizeof(int32_t) * (s.n_cells + 1));
    b += al(sizeof(uint32_t) * 4 * (s.n_cells > 0 ? s.n_cells : 1));
    b += al(sizeof(int32_t) * (s.n_chunks + 1));
    b += al(sizeof(int2) * s.n_chunks * kChunk + 8);
    b += 3 * al(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b += 3 * al(8 * s.n_collide_blocks);
    return b;
}

void carve_compact_buffers(const Workspace& w, const StepShape& s, CompactBuffers* b) {
    b->ctrl = ws_control(w);
    b->status = ws_status(w);
    char* p = (char*)ws_step_area(w);
    auto take = [&](size_t n) {
        char* r = p;
        p += al(n);
        return (void*)r;
    };
    b->pair_off = (int32_t*)take(sizeof(int32_t) * (s.n_cells + 1));
    b->cell_keys = (uint32_t*)take(sizeof(uint32_t) * 4 * (s.n_cells > 0 ? s.n_cells : 1));
    b->chunk_cell = (int32_t*)take(sizeof(int32_t) * (s.n_chunks + 1));
    b->list = (int2*)take(sizeof(int2) * s.n_chunks * kChunk + 8);
    b->chunk_prob = (double*)take(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b->chunk_clip = (int64_t*)take(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b->chunk_inv = (int64_t*)take(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b->coll_eb = (double*)take(8 * s.n_collide_blocks);
    b->coll_ea = (double*)take(8 * s.n_collide_blocks);
    b->coll_fb = (int64_t*)take(8 * s.n_collide_blocks);
}

template <typename T, int SAMP>
static hipError_t launch_compact_t(const StepShape& sh, const CompactBuffers& b, const StepParams& p, hipStream_t st) {
    auto mark = [&](int i) {
        if (p.events) (void)hipEventRecord(p.events[i], st);
    };
    mark(0);
    // prep status words first, then one per chunk
    hipError_t e = launch_prep(sh, b.ctrl, b.status, b.pair_off, b.cell_keys, b.chunk_cell, p, st);
    if (e != hipSuccess) return e;
    mark(1);
    CompactArgs<T> a;
    a.pt = {(T*)p.e.x, (T*)p.e.y, (T*)p.e.z, (T*)p.e.w, (T*)p.g.x, (T*)p.g.y, (T*)p.g.z, (T*)p.g.w};
    a.off_e = p.off_e;
    a.off_g = p.off_g;
    a.n_cells = sh.n_cells;
    a.n_chunks = sh.n_chunks;
    a.pair_off = b.pair_off;
    a.keys = b.cell_keys;
    a.chunk_cell = b.chunk_cell;
    a.dt = p.dt;
    a.density_norm = p.density_norm;
    a.seed = p.seed;
    a.ctrl = b.ctrl;
    a.status = b.status + sh.n_prep_blocks;
    a.list = b.list;
    a.chunk_prob = b.chunk_prob;
    a.chunk_clip = b.chunk_clip;
    a.chunk_inv = b.chunk_inv;
    a.coll_eb = b.coll_eb;
    a.coll_ea = b.coll_ea;
    a.coll_fb = b.coll_fb;
    a.stats = p.stats;
    a.mlp = p.net;
    const int64_t n_pair_blocks = compact_pair_blocks(sh);
    if (sh.n_chunks > 0) {
        if (sh.pairs_per_lane == 1)
            k_pair_compact<T, 1><<<(unsigned)n_pair_blocks, kChunk, 0, st>>>(a);
        else if (sh.pairs_per_lane == 2)
            k_pair_compact<T, 2><<<(unsigned)n_pair_blocks, kChunk, 0, st>>>(a);
        else
            k_pair_compact<T, 4><<<(unsigned)n_pair_blocks, kChunk, 0, st>>>(a);
    }
    mark(2);
    mark(3);
    k_collide_dense<T, SAMP><<<(unsigned)sh.n_collide_blocks,
                               SAMP == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads, 0, st>>>(a);
    mark(4);
    FinalArgs f = {};
    f.ctrl = b.ctrl;
    f.pair_off = b.pair_off;
    f.n_cells = sh.n_cells;
    f.a_prob = b.chunk_prob;
    f.a_clip = b.chunk_clip;
    f.a_inv = b.chunk_inv;
    f.a_coll = nullptr;
    f.n_a = n_pair_blocks;
    f.b_eb = b.coll_eb;
    f.b_ea = b.coll_ea;
    f.b_fb = b.coll_fb;
    f.n_b = sh.n_collide_blocks;
    f.stats = p.stats;
    e = launch_finalize(f, st);
    mark(5);
    return e == hipSuccess ? hipGetLastError() : e;
}

template <typename T>
static hipError_t launch_compact_s(const StepShape& sh, const CompactBuffers& b, const StepParams& p,
                                   hipStream_t st) {
    switch (p.sampler) {
        case CS_SAMPLER_MLP_F32:
            return launch_compact_t<T, CS_SAMPLER_MLP_F32>(sh, b, p, st);
        case CS_SAMPLER_MLP_BF16:
            return launch_compact_t<T, CS_SAMPLER_MLP_BF16>(sh, b, p, st);
        case CS_SAMPLER_MLP_FP8:
            return launch_compact_t<T, CS_SAMPLER_MLP_FP8>(sh, b, p, st);
        default:
            return launch_compact_t<T, CS_SAMPLER_PLAIN>(sh, b, p, st);
    }
}

int64_t compact_collide_threads(cs_sampler s) { return s == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads; }

hipError_t launch_compact(const StepShape& sh, const CompactBuffers& b, const StepParams& p, hipStream_t st) {
    if (p.dtype == CS_F64) return launch_compact_s<double>(sh, b, p, st);
    return launch_compact_s<float>(sh, b, p, st);
}

}  // namespace cs
