// cs_compact.hip -- the step as four kernels (default strategy):
//
//   k_prep_scan       (cs_fused.hip) cells -> pair offsets, keys, chunk map
//   k_pair_compact    one lane per pair, each workgroup loops over G
//                     consecutive 256-pair chunks: pairing, x, s(x), P,
//                     accept; each wave writes its accepted pairs with their
//                     values to its stash region and the workgroup lists
//                     their slots in order: in a segment of its own (up to
//                     kSegMax workgroups), or, for more workgroups, at its
//                     place in a dense list found by decoupled look-back.
//                     Either way the order is fixed and no atomics are used.
//                     Lean (no sampler), so it runs at high occupancy.
//   k_collide_dense   workgroups stride over the accepted pairs in that
//                     order (segments: each collide workgroup first forms the
//                     prefix sums of the segment lengths): sample the angle,
//                     scatter, write back (four waves per workgroup; with a
//                     network sampler they share the network's LDS copy).
//   k_finalize_step   (cs_fused.hip) fixed-order reduction of the partial sums.
#include <hip/hip_runtime.h>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_lookback.h"
#include "cs_pair.h"

namespace cs {

constexpr int kDenseThreads = 256;     // plain sampler
constexpr int kDenseNetThreads = 256;  // network samplers

template <typename T>
struct CompactArgs {
    Particles<T> pt;
    const int64_t *off_e, *off_g;
    int64_t n_cells, n_chunks;
    int32_t chunks_per_block;  // pair kernel: consecutive chunks per workgroup
    int32_t balance;           // pair kernel: pace the waves (the grid is one round of resident workgroups)
    const int32_t* pair_off;
    const uint32_t* keys;
    const int32_t* chunk_cell;
    double dt, density_norm;
    uint64_t seed;
    StepControl* ctrl;
    uint64_t* status;  // pair kernel: one word per workgroup, kPairStatusStride apart
    int32_t* list;          // accepted pairs' stash slots: dense, or one segment per pair workgroup
    int32_t* seg_count;     // segmented: accepted pairs of each pair workgroup
    int32_t n_seg;          // pair workgroups when segmented, else 0 (look-back)
    StashPair<T>* stash;    // accepted pairs with their values, per-wave regions
    double* chunk_prob;
    int64_t* chunk_clip;
    int64_t* chunk_inv;
    double* coll_eb;
    double* coll_ea;
    int64_t* coll_fb;
    cs_stats* stats;
    MlpDev mlp;
};

// s_waitcnt immediate that waits for vmcnt 0 only (gfx9 encoding: vmcnt in
// bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 at their maxima).
constexpr int kWaitVmcnt0 = 0x0F70;

// Read-only data at a wave-uniform index through the constant address space,
// so that the read is one scalar load (the data do not change while the
// kernel runs).
template <typename X>
__device__ __forceinline__ X ld_uniform(const X* p, int64_t i) {
    return ((const __attribute__((address_space(4))) X*)p)[i];
}

// Phases 1 and 2 of one step of the pair kernel for one lane: the pairs of
// chunks j0 .. j0 + PPL - 1 (one pair of each), their cells, particle ranges
// and pairing keys, the pairing, and the particle reads -- issued, to be
// consumed a step later.  The chunk's first cell is the same for the whole
// wave: its metadata come by scalar loads.  If some lane's pair lies in a
// later cell, the wave reads the metadata of the chunk's cells (up to 64, one
// per lane) in one coalesced round trip and each lane finds its own cell
// among them by a binary search over lane shuffles (chunks of more than 64
// cells: a binary search per lane in global memory).  `cc`
// holds chunk_cell[blk G + lane]; c0 is the step's first chunk relative to
// blk G.  valid == false (uniform) yields inactive slots.
template <typename T, int PPL, bool O32>
__device__ __forceinline__ void pair_fetch(const CompactArgs<T>& a, bool valid, int64_t j0, int c0, int cc,
                                           int32_t T_total, int tid, PairSlot (&sl)[PPL],
                                           PairRaw<T> (&raw)[PPL]) {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
        const int64_t j = j0 + q;
        const int32_t t = (int32_t)(j * kChunk) + tid;
        const bool jv = valid && j < a.n_chunks && j * kChunk < (int64_t)T_total;  // uniform
        const bool act = jv && t < T_total;
        int64_t e0 = 0, e1 = 0, g0 = 0, g1 = 0;
        uint4 key = make_uint4(0, 0, 0, 0);
        int32_t po = 0, po_next = 0;
        if (jv) {
            const int cs0 = __builtin_amdgcn_readlane(cc, c0 + q);
            e0 = ld_uniform(a.off_e, cs0);
            e1 = ld_uniform(a.off_e, cs0 + 1);
            g0 = ld_uniform(a.off_g, cs0);
            g1 = ld_uniform(a.off_g, cs0 + 1);
            key = make_uint4(ld_uniform(a.keys, 4 * cs0), ld_uniform(a.keys, 4 * cs0 + 1),
                             ld_uniform(a.keys, 4 * cs0 + 2), ld_uniform(a.keys, 4 * cs0 + 3));
            po = ld_uniform(a.pair_off, cs0);
            po_next = ld_uniform(a.pair_off, cs0 + 1);
            const int ch = __builtin_amdgcn_readlane(cc, c0 + q + 1);
            const int nc = ch - cs0 + 1;  // cells cs0 .. ch hold the chunk's pairs
            if (__any(act && t >= po_next)) {
                if (nc <= 64) {
                    // lane l reads cell cs0 + l's metadata (one coalesced
                    // round trip); each lane finds its cell among them by
                    // a binary search over the wave's pair offsets and takes
                    // that cell's values by lane shuffles
                    const int cl = cs0 + (lane_id() < nc ? lane_id() : nc - 1);
                    const int32_t po_l = a.pair_off[cl];
                    const int64_t e0_l = a.off_e[cl], g0_l = a.off_g[cl];
                    const int32_t ne_l = (int32_t)(a.off_e[cl + 1] - e0_l), ng_l = (int32_t)(a.off_g[cl + 1] - g0_l);
                    const uint4 key_l = *(const uint4*)(a.keys + 4 * cl);
                    int lo = 0, hi = nc - 1;
#pragma unroll
                    for (int it = 0; it < 6; ++it) {  // nc <= 64 = 2^6
                        const int mid = (lo + hi + 1) >> 1;
                        if (__shfl(po_l, mid, 64) <= t)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    // (shuffles by the whole wave, then the selection)
                    const int64_t e0c = (int64_t)__shfl((unsigned long long)e0_l, lo, 64);
                    const int64_t g0c = (int64_t)__shfl((unsigned long long)g0_l, lo, 64);
                    const int32_t nec = __shfl(ne_l, lo, 64), ngc = __shfl(ng_l, lo, 64);
                    const uint4 keyc = make_uint4(__shfl(key_l.x, lo, 64), __shfl(key_l.y, lo, 64),
                                                  __shfl(key_l.z, lo, 64), __shfl(key_l.w, lo, 64));
                    const int32_t poc = __shfl(po_l, lo, 64);
                    if (act && t >= po_next) {
                        e0 = e0c;
                        g0 = g0c;
                        e1 = e0c + nec;
                        g1 = g0c + ngc;
                        key = keyc;
                        po = poc;
                    }
                } else if (act && t >= po_next) {
                    // more than 64 cells in the chunk: per-lane binary search
                    int lo = cs0 + 1, hi = ch;
                    while (lo < hi) {
                        const int mid = (lo + hi + 1) >> 1;
                        if (a.pair_off[mid] <= t)
                            lo = mid;
                        else
                            hi = mid - 1;
                    }
                    e0 = a.off_e[lo];
                    e1 = a.off_e[lo + 1];
                    g0 = a.off_g[lo];
                    g1 = a.off_g[lo + 1];
                    key = *(const uint4*)(a.keys + 4 * lo);
                    po = a.pair_off[lo];
                }
                // complete these reads inside the branch, so that no read of
                // it is still counted as possibly in flight after it (which
                // would make later waits include the particle reads)
                __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
            }
        }
        sl[q] = pair_index(act, e0, e1, g0, g1, key.x, key.y, key.z, key.w, (uint32_t)(t - po));
        raw[q] = pair_load_all<T, O32>(a.pt, sl[q]);
    }
}

// A SIMD's arbiter issues from the oldest of its waves first, so waves of
// equal work (one per workgroup on the SIMD) drift apart and finish one after
// another, the last ones alone with their latency exposed.  Before each step
// a wave takes the priority (rem - 1) mod 4 from the steps it has left, rem:
// among waves within a few steps of each other the one behind is issued first
// (except across a wrap of the four levels), and in the last four steps the
// order is exact, so that the waves finish close together.  Used only when
// every workgroup of the grid is resident at once: with more workgroups than
// that, a workgroup that finishes early makes room for a waiting one, which
// pacing would delay.
__device__ __forceinline__ void balance_priority(int rem) {
    switch ((rem - 1) & 3) {
        case 3: __builtin_amdgcn_s_setprio(3); break;
        case 2: __builtin_amdgcn_s_setprio(2); break;
        case 1: __builtin_amdgcn_s_setprio(1); break;
        default: __builtin_amdgcn_s_setprio(0); break;
    }
}

// One workgroup takes G consecutive 256-pair chunks, PPL of them per step
// (one pair of each per lane).  Software pipeline: the pairing and particle
// reads of step s + 1 are issued before the physics of step s, so their
// latency hides behind it (the physics reads nothing from global memory:
// the s(x) table is copied to LDS first).  Each wave writes its accepted
// pairs, with the particle values it read, to its own region of the stash
// (64 G slots) in the order it meets them; after the last step one look-back
// places the workgroup's slots (wave 0's, then wave 1's, ...) in the dense
// list, whose entry q names the stash slot of accepted pair q.
template <typename T, int PPL, bool O32>
__global__ __launch_bounds__(kChunk) void k_pair_compact(const CompactArgs<T> a) {
    __shared__ double s_sig[kSigTabSegments * kSigTabTerms];
    __shared__ int s_wcnt[kChunk / 64];
    __shared__ int s_prefix;
    __shared__ double s_rd[kChunk / 64];
    __shared__ long long s_ri[2 * (kChunk / 64)];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int64_t blk = blockIdx.x;
    const int G = a.chunks_per_block;
    // the s(x) table into LDS: every thread's reads issued before anything
    // waits, and stored below (a loop of read, wait, store would wait once
    // per round)
    constexpr int kSigRounds = kSigTabSegments * kSigTabTerms / kChunk;
    static_assert(kSigRounds * kChunk == kSigTabSegments * kSigTabTerms, "whole rounds");
    double sig_v[kSigRounds];
#pragma unroll
    for (int r = 0; r < kSigRounds; ++r) sig_v[r] = kSigTab[tid + r * kChunk];
    // chunk_cell of the workgroup's chunks and of the one after them, lane i
    // holding entry blk G + i (G < 64)
    const int64_t jc = blk * G + lane;
    const int cc = lane <= G && jc <= a.n_chunks ? a.chunk_cell[jc] : 0;
    const int32_t T_read = a.pair_off[a.n_cells];  // read with the control block, not after it
    StepControl* ctrl = a.ctrl;
    const CtrlView cv = ctrl_view(ctrl);
    const uint32_t E = cv.epoch;
    const uint64_t step = cv.step;
    const bool layout_ok = cv.layout_ok;
    const int32_t T_total = layout_ok ? T_read : 0;
    // (the s(x) table's reads, issued first, stored here)
#pragma unroll
    for (int r = 0; r < kSigRounds; ++r) s_sig[tid + r * kChunk] = sig_v[r];
    // steps of this workgroup: its chunks below min(n_chunks, ceil(T / kChunk))
    int64_t n_used = ((int64_t)T_total + kChunk - 1) / kChunk;
    if (n_used > a.n_chunks) n_used = a.n_chunks;
    int64_t n_mine = n_used - blk * G;
    n_mine = n_mine < 0 ? 0 : (n_mine > G ? G : n_mine);
    const int n_steps = (int)((n_mine + PPL - 1) / PPL);
    const int32_t slot0 = (int32_t)((blk * (kChunk / 64) + wave) * 64 * G);  // the wave's stash region
    StashPair<T>* stage = a.stash + slot0;
    int n_stage = 0;  // wave-uniform
    const uint64_t lanes_below = (1ull << lane) - 1ull;
    double sum_p = 0.0;
    long long n_clip = 0, n_inv = 0;
    // physics of one step; accepted pairs go to the wave's stash region
    auto physics = [&](const PairSlot(&sl)[PPL], const PairRaw<T>(&raw)[PPL]) {
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
            const PairOutcome o = pair_physics<T>(sl[q], raw[q], a.dt, a.density_norm, a.seed, step, s_sig);
            sum_p += o.P;
            n_clip += o.clipped ? 1 : 0;
            n_inv += o.invalid ? 1 : 0;
            const uint64_t mask = __ballot(o.accept);
            if (o.accept) stage[n_stage + __popcll(mask & lanes_below)] = make_stash<T>(sl[q], raw[q]);
            n_stage += __popcll(mask);
        }
    };
    // two register sets in turn (no copies, which would wait for the reads)
    PairSlot sl_a[PPL], sl_b[PPL];
    PairRaw<T> raw_a[PPL], raw_b[PPL];
    pair_fetch<T, PPL, O32>(a, n_steps > 0, blk * G, 0, cc, T_total, tid, sl_a, raw_a);
    __syncthreads();  // s_sig
    for (int st = 0; st < n_steps; st += 2) {
        pair_fetch<T, PPL, O32>(a, st + 1 < n_steps, blk * G + (st + 1) * PPL, (st + 1) * PPL, cc, T_total, tid, sl_b,
                           raw_b);
        if (a.balance) balance_priority(n_steps - st);
        physics(sl_a, raw_a);
        if (st + 1 >= n_steps) break;
        pair_fetch<T, PPL, O32>(a, st + 2 < n_steps, blk * G + (st + 2) * PPL, (st + 2) * PPL, cc, T_total, tid, sl_a,
                           raw_a);
        if (a.balance) balance_priority(n_steps - st - 1);
        physics(sl_b, raw_b);
    }
    __builtin_amdgcn_s_setprio(0);
    const double wp = wave_sum(sum_p);
    const long long wc = wave_sum_i(n_clip), wi = wave_sum_i(n_inv);
    if (lane == 0) {
        s_rd[wave] = wp;
        s_ri[2 * wave] = wc;
        s_ri[2 * wave + 1] = wi;
        s_wcnt[wave] = n_stage;
    }
    __syncthreads();
    int wbase = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kChunk / 64; ++w) {
        wbase += w < wave ? s_wcnt[w] : 0;
        total += s_wcnt[w];
    }
    const bool seg = a.n_seg > 0;  // uniform
    if (!seg && tid < 64) {
        const uint32_t ex =
            lookback_exclusive_wave<kPairStatusStride>(a.status, blk, E, (uint32_t)total, &ctrl->scan_fault_epoch);
        if (tid == 0) s_prefix = (int)ex;
    }
    if (tid == 0) {
        if (seg) a.seg_count[blk] = total;
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
    int32_t* dst = a.list + (seg ? blk * kChunk * G : (int64_t)s_prefix) + wbase;
    for (int i = lane; i < n_stage; i += 64) dst[i] = slot0 + i;
    if (!seg && tid == 0 && blk == (int64_t)gridDim.x - 1) ctrl->n_accepted = (uint32_t)(s_prefix + total);
}

// Segmented list: prefix sums over the pair workgroups' counts, computed by
// every collide workgroup instead of a look-back chain in the pair kernel
// (whose workgroups, finishing together, would wait for one another).
// Thread t of NT takes counts [P t, P (t + 1)), P = kSegMax / NT: seg_load
// reads them (issued only, so that other reads can join them), seg_scan
// writes the n <= kSegMax exclusive prefixes to s and returns the total.
// Both are called by every thread.  The count array has room for kSegMax
// entries whatever n, so that a thread reads its P counts with 16-byte loads
// and zeroes those past n (element by element, the reads sat in branches of
// their own, each waiting for the array's address).
constexpr int kSegMax = 4096;

template <int NT>
struct SegCounts {
    int32_t v[kSegMax / NT];
};

template <int NT>
__device__ __forceinline__ SegCounts<NT> seg_load(const int32_t* cnt, int n) {
    constexpr int kSegPerThread = kSegMax / NT;
    static_assert(kSegPerThread % 4 == 0, "16-byte reads");
    const int k0 = (int)threadIdx.x * kSegPerThread;
    int4 q[kSegPerThread / 4];
    if (k0 < n) {
#pragma unroll
        for (int j = 0; j < kSegPerThread / 4; ++j) q[j] = ((const int4*)(cnt + k0))[j];
    } else {
#pragma unroll
        for (int j = 0; j < kSegPerThread / 4; ++j) q[j] = make_int4(0, 0, 0, 0);
    }
    SegCounts<NT> c;
#pragma unroll
    for (int j = 0; j < kSegPerThread / 4; ++j) {
        const int i = 4 * j;
        c.v[i] = k0 + i < n ? q[j].x : 0;
        c.v[i + 1] = k0 + i + 1 < n ? q[j].y : 0;
        c.v[i + 2] = k0 + i + 2 < n ? q[j].z : 0;
        c.v[i + 3] = k0 + i + 3 < n ? q[j].w : 0;
    }
    return c;
}

template <int NT>
__device__ __forceinline__ int32_t seg_scan(SegCounts<NT> c, int n, int32_t* s, int32_t* s_wtot) {
    constexpr int kSegPerThread = kSegMax / NT;
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    const int k0 = tid * kSegPerThread;
    int32_t* v = c.v;
    int32_t run = 0;
#pragma unroll
    for (int i = 0; i < kSegPerThread; ++i) {
        const int32_t x = v[i];
        v[i] = run;
        run += x;
    }
    int32_t incl = run;  // inclusive scan of the thread totals over the wave
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
    }
    int32_t excl = incl - run, total;
    if constexpr (NT > 64) {
        if (lane == 63) s_wtot[wave] = incl;
        __syncthreads();
        int32_t wb = 0;
        total = 0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) {
            wb += w < wave ? s_wtot[w] : 0;
            total += s_wtot[w];
        }
        excl += wb;
    } else {
        total = __shfl(incl, 63, 64);
    }
#pragma unroll
    for (int i = 0; i < kSegPerThread; ++i)
        if (k0 + i < n) s[k0 + i] = excl + v[i];
    __syncthreads();
    return total;
}

// The segment holding dense position q is the last b with s[b] <= q (empty
// segments share their prefix with the next one).  seg_bsearch: binary
// search in [lo, hi] given s[lo] <= q.  seg_gallop: from b0 with s[b0] <= q,
// probes b0 + 1, + 2, + 4, ... first: within a wave the positions are
// consecutive, so that from the wave's first segment the answer is near.
__device__ __forceinline__ int seg_bsearch(const int32_t* s, int lo, int hi, int32_t q) {
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s[mid] <= q)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int seg_gallop(const int32_t* s, int n, int b0, int32_t q) {
    int lo = b0, hi = n - 1;
    for (int step = 1;; step <<= 1) {
        const int probe = b0 + step;
        if (probe >= n) break;
        if (s[probe] > q) {
            hi = probe - 1;
            break;
        }
        lo = probe;
    }
    return seg_bsearch(s, lo, hi, q);
}

// Network samplers resolve the pairs outside the network's domain in place
// with the plain sampler: the lanes of a wave that need it run it together.
// (Collecting them for separate dense passes was measured slower: the kernel
// is bound by the latency of one pass, not by issue.)
template <typename T, int SAMP>
__global__ __launch_bounds__(SAMP == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads) void k_collide_dense(
    const CompactArgs<T> a) {
    constexpr int NT = SAMP == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads;
    constexpr bool NET = SAMP != CS_SAMPLER_PLAIN;
    __shared__ NetLds<SAMP> s_net;
    __shared__ double s_d[2 * (NT / 64)];
    __shared__ long long s_fbc[NT / 64];
    __shared__ int32_t s_wtot[NT / 64];
    extern __shared__ int32_t s_seg[];  // segmented: the n_seg prefixes
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    // the network's copy, the control block and the segment counts are read
    // together (the counts whatever the layout), then the copy is stored
    // while the counts are still in flight; the scan's barriers publish it
    NetFetch<SAMP, NT> nf;
    nf.fetch(a.mlp);
    StepControl* ctrl = a.ctrl;
    const CtrlView cv = ctrl_view(ctrl);
    const uint64_t step = cv.step;
    const bool layout_ok = cv.layout_ok;
    const bool seg = a.n_seg > 0;  // uniform
    int64_t A;
    if (seg) {
        const SegCounts<NT> cnt = seg_load<NT>(a.seg_count, a.n_seg);
        nf.store(s_net);
        const int32_t total = seg_scan<NT>(cnt, a.n_seg, s_seg, s_wtot);
        A = layout_ok ? (int64_t)total : 0;
        if (blockIdx.x == 0 && tid == 0) ctrl->n_accepted = (uint32_t)A;
    } else {
        nf.store(s_net);
        if constexpr (NET) __syncthreads();
        A = layout_ok ? (int64_t)ctrl->n_accepted : 0;
    }
    const int64_t seg_len = (int64_t)kChunk * a.chunks_per_block;
    const int64_t stride = (int64_t)gridDim.x * NT;
    const int64_t n_iter = (A + stride - 1) / stride;  // uniform over the grid
    CollideSums sums;
    for (int64_t it = 0; it < n_iter; ++it) {
        const int64_t q = it * stride + (int64_t)blockIdx.x * NT + tid;
        const bool active = q < A;
        if (!__any(active)) break;
        // lane 0 holds the wave's smallest position, and is active if any
        // lane is: its segment, searched once per wave, starts every lane's
        // search
        const int b_wave = seg ? seg_bsearch(s_seg, 0, a.n_seg - 1, __builtin_amdgcn_readfirstlane((int32_t)q)) : 0;
        int32_t slot = 0;
        if (active) {
            int64_t li = q;
            if (seg) {
                const int b = seg_gallop(s_seg, a.n_seg, b_wave, (int32_t)q);
                li = b * seg_len + (q - s_seg[b]);
            }
            slot = a.list[li];
        }
        if constexpr (!NET)
            collide_stash<T>(a.pt, active, a.stash + slot, a.seed, step, sums);
        else
            collide_net<T, SAMP>(a.pt, active, FromStash<T>{a.stash + slot}, s_net, a.mlp, a.seed, step, sums);
    }
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
    const int64_t G = s.chunks_per_block;
    return s.n_chunks > 0 ? (s.n_chunks + G - 1) / G : 0;
}

// list entries: one segment of kChunk G per pair workgroup covers both the
// dense and the segmented layout
static int64_t compact_list_len(const StepShape& s) {
    const int64_t seg = compact_pair_blocks(s) * kChunk * s.chunks_per_block;
    return seg > s.n_chunks * kChunk ? seg : s.n_chunks * kChunk;
}

// stash slots: 64 G per wave of every pair workgroup (the largest entry
// type, so that one workspace serves either storage type)
static size_t compact_stash_bytes(const StepShape& s) {
    return sizeof(StashPair<double>) * (size_t)compact_pair_blocks(s) * kChunk * (size_t)s.chunks_per_block;
}

// per pair workgroup its accepted count, with room for the kSegMax counts
// that seg_load reads
static int64_t seg_count_len(const StepShape& s) {
    const int64_t n = compact_pair_blocks(s) + 1;
    return n > kSegMax ? n : kSegMax;
}

size_t compact_workspace_bytes(const StepShape& s) {
    size_t b = 0;
    b += al(sizeof(int32_t) * (s.n_cells + 1));
    b += al(sizeof(uint32_t) * 4 * (s.n_cells > 0 ? s.n_cells : 1));
    b += al(sizeof(int32_t) * (s.n_chunks + 1));
    b += al(sizeof(int32_t) * compact_list_len(s) + 8);
    b += al(sizeof(int32_t) * seg_count_len(s));
    b += al(compact_stash_bytes(s) + 16);
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
    b->list = (int32_t*)take(sizeof(int32_t) * compact_list_len(s) + 8);
    b->seg_count = (int32_t*)take(sizeof(int32_t) * seg_count_len(s));
    b->stash = take(compact_stash_bytes(s) + 16);
    b->chunk_prob = (double*)take(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b->chunk_clip = (int64_t*)take(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b->chunk_inv = (int64_t*)take(8 * (s.n_chunks > 0 ? s.n_chunks : 1));
    b->coll_eb = (double*)take(8 * s.n_collide_blocks);
    b->coll_ea = (double*)take(8 * s.n_collide_blocks);
    b->coll_fb = (int64_t*)take(8 * s.n_collide_blocks);
}

// Workgroups of k_pair_compact<T, PPL, O32> resident at once on the current
// device (its compute units times the kernel's occupancy), computed once.
template <typename T, int PPL, bool O32 = true>
static int64_t pair_resident_blocks() {
    static int64_t cached = -1;
    if (cached < 0) {
        int dev = 0, n_cu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void*>(&k_pair_compact<T, PPL, O32>), kChunk, 0) != hipSuccess)
            return 0;  // unknown: no pacing
        cached = (int64_t)n_cu * per_cu;
    }
    return cached;
}

int64_t compact_fit_chunks(cs_dtype dtype, int64_t ppl, int64_t n_chunks) {
    int64_t r;
    if (dtype == CS_F64)
        r = ppl == 1 ? pair_resident_blocks<double, 1>()
                     : ppl == 2 ? pair_resident_blocks<double, 2>() : pair_resident_blocks<double, 4>();
    else
        r = ppl == 1 ? pair_resident_blocks<float, 1>()
                     : ppl == 2 ? pair_resident_blocks<float, 2>() : pair_resident_blocks<float, 4>();
    if (r <= 0) r = 1024;
    int64_t g = (n_chunks + r - 1) / r;
    g = (g + ppl - 1) / ppl * ppl;
    if (g < ppl) g = ppl;
    if (g > kCompactMaxChunks) g = kCompactMaxChunks / ppl * ppl;
    return g;
}

// 32-bit byte offsets into the particle arrays whenever both species fit
// (at most 2^32 / sizeof(T) elements) and `wide` is 0; 64-bit indexing
// otherwise.
template <typename T, int PPL>
static hipError_t launch_pair_compact(CompactArgs<T> a, int64_t n_blocks, int64_t ne, int64_t ng, int wide,
                                      hipStream_t st) {
    constexpr int64_t kO32Max = ((int64_t)1 << 32) / (int64_t)sizeof(T);
    if (!wide && ne <= kO32Max && ng <= kO32Max) {
        a.balance = n_blocks <= pair_resident_blocks<T, PPL, true>() ? 1 : 0;
        k_pair_compact<T, PPL, true><<<(unsigned)n_blocks, kChunk, 0, st>>>(a);
    } else {
        a.balance = n_blocks <= pair_resident_blocks<T, PPL, false>() ? 1 : 0;
        k_pair_compact<T, PPL, false><<<(unsigned)n_blocks, kChunk, 0, st>>>(a);
    }
    return hipGetLastError();
}

template <typename T, int SAMP>
static hipError_t launch_compact_t(const StepShape& sh, const CompactBuffers& b, const StepParams& p, hipStream_t st) {
    auto mark = [&](int i) {
        if (p.events) (void)hipEventRecord(p.events[i], st);
    };
    mark(0);
    // prep status words first, then the pair workgroups' (kPairStatusStride apart)
    hipError_t e = launch_prep(sh, b.ctrl, b.status, b.pair_off, b.cell_keys, b.chunk_cell, p, st);
    if (e != hipSuccess) return e;
    mark(1);
    CompactArgs<T> a;
    a.pt = {(T*)p.e.x, (T*)p.e.y, (T*)p.e.z, (T*)p.e.w, (T*)p.g.x, (T*)p.g.y, (T*)p.g.z, (T*)p.g.w};
    a.off_e = p.off_e;
    a.off_g = p.off_g;
    a.n_cells = sh.n_cells;
    a.n_chunks = sh.n_chunks;
    a.chunks_per_block = (int32_t)sh.chunks_per_block;
    a.pair_off = b.pair_off;
    a.keys = b.cell_keys;
    a.chunk_cell = b.chunk_cell;
    a.dt = p.dt;
    a.density_norm = p.density_norm;
    a.seed = p.seed;
    a.ctrl = b.ctrl;
    a.status = b.status + sh.n_prep_blocks;
    a.list = b.list;
    a.seg_count = b.seg_count;
    a.stash = (StashPair<T>*)b.stash;
    a.chunk_prob = b.chunk_prob;
    a.chunk_clip = b.chunk_clip;
    a.chunk_inv = b.chunk_inv;
    a.coll_eb = b.coll_eb;
    a.coll_ea = b.coll_ea;
    a.coll_fb = b.coll_fb;
    a.stats = p.stats;
    a.mlp = p.net;
    constexpr int kCollideThreads = SAMP == CS_SAMPLER_PLAIN ? kDenseThreads : kDenseNetThreads;
    const int64_t n_pair_blocks = compact_pair_blocks(sh);
    // segmented list whenever a collide workgroup can scan the pair
    // workgroups' counts in one pass (at most kSegMax); else the pair
    // kernel's look-back
    a.n_seg = n_pair_blocks > 0 && n_pair_blocks <= kSegMax ? (int32_t)n_pair_blocks : 0;
    if (sh.n_chunks > 0) {
        if (sh.pairs_per_lane == 1)
            e = launch_pair_compact<T, 1>(a, n_pair_blocks, sh.ne, sh.ng, p.wide_index, st);
        else if (sh.pairs_per_lane == 2)
            e = launch_pair_compact<T, 2>(a, n_pair_blocks, sh.ne, sh.ng, p.wide_index, st);
        else
            e = launch_pair_compact<T, 4>(a, n_pair_blocks, sh.ne, sh.ng, p.wide_index, st);
        if (e != hipSuccess) return e;
    }
    mark(2);
    mark(3);
    k_collide_dense<T, SAMP><<<(unsigned)sh.n_collide_blocks, kCollideThreads, sizeof(int32_t) * (size_t)a.n_seg, st>>>(a);
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
