// cs_fused.hip -- the step as a scan kernel, a persistent step kernel and a
// finalize kernel.
//
//   k_prep_scan  one pass over the cells: validate offsets, pairs per cell
//                (min(N_e, N_g)), pairing keys, exclusive scan of the pair
//                counts by decoupled look-back, and the first cell of every
//                256-pair chunk.
//   k_step       persistent over chunks: each workgroup evaluates `chunks`
//                consecutive 256-pair chunks (pairing, x, s(x), P, accept),
//                appends accepted pairs in pair order to a queue in LDS, and
//                drains the queue densely (all lanes busy) whenever it holds
//                a full workgroup of pairs and at the end; per-workgroup partial
//                sums go to the workspace.
//   k_finalize_step  one workgroup reduces the partial sums in a fixed order
//                into cs_stats and advances the step epoch and device step.
//
// Step-to-step state lives in a small control block of the workspace (epoch,
// done counter, layout flag, device step).  The look-back status words and
// the layout flag carry the epoch of the step that wrote them, so nothing
// needs clearing between steps.
#include <hip/hip_runtime.h>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_lookback.h"
#include "cs_pair.h"

namespace cs {

// ---------------------------------------------------------------------------
// k_prep_scan
// ---------------------------------------------------------------------------
constexpr int kPrepThreads = 256;
constexpr int kPrepPerThread = 1;
constexpr int kPrepCells = kPrepThreads * kPrepPerThread;

struct PrepArgs {
    const int64_t *off_e, *off_g;
    int64_t n_cells, ne, ng, n_chunks;
    uint64_t seed, step;
    int use_device_step;  // 1: take the step from ctrl (graph replay)
    int32_t* pair_off;    // [n_cells + 1]
    uint32_t* keys;       // [4 n_cells]
    int32_t* chunk_cell;  // [n_chunks + 1]
    uint64_t* status;     // [n_prep_blocks]
    StepControl* ctrl;
};

__global__ __launch_bounds__(kPrepThreads) void k_prep_scan(const PrepArgs a) {
    __shared__ int s_scan[kPrepThreads / 64 + 1];
    __shared__ int s_prefix;
    // (not ctrl_view: block 0 may write the step word during this kernel)
    const uint32_t E = a.ctrl->epoch;
    const uint64_t step = a.use_device_step ? a.ctrl->step : a.step;
    const int64_t base = (int64_t)blockIdx.x * kPrepCells + (int64_t)threadIdx.x * kPrepPerThread;
    int cnt[kPrepPerThread];
    bool bad = false;
    int tsum = 0;
#pragma unroll
    for (int r = 0; r < kPrepPerThread; ++r) {
        const int64_t c = base + r;
        cnt[r] = 0;
        if (c < a.n_cells) {
            const int64_t a0 = a.off_e[c], a1 = a.off_e[c + 1], b0 = a.off_g[c], b1 = a.off_g[c + 1];
            bool b = a1 < a0 || b1 < b0;
            if (c == 0) b = b || a0 != 0 || b0 != 0;
            if (c == a.n_cells - 1) b = b || a1 != a.ne || b1 != a.ng;
            if (b) {
                bad = true;
            } else {
                const int64_t nmin = (a1 - a0) < (b1 - b0) ? (a1 - a0) : (b1 - b0);
                cnt[r] = (int)nmin;
                if (nmin > 0) {
                    const u32x4 k = draw(a.seed, (uint64_t)c, step, kPair);
                    a.keys[4 * c + 0] = k.a;
                    a.keys[4 * c + 1] = k.b;
                    a.keys[4 * c + 2] = k.c;
                    a.keys[4 * c + 3] = k.d;
                }
            }
        }
        tsum += cnt[r];
    }
    if (bad) atomicMax(&a.ctrl->layout_epoch, E);
    if (blockIdx.x == 0 && threadIdx.x == 0 && !a.use_device_step) a.ctrl->step = a.step;
    int block_total;
    const int tex = block_exclusive_scan(tsum, s_scan, &block_total);
    if (threadIdx.x < 64) {
        const uint32_t ex =
            lookback_exclusive_wave(a.status, blockIdx.x, E, (uint32_t)block_total, &a.ctrl->scan_fault_epoch);
        if (threadIdx.x == 0) s_prefix = (int)ex;
    }
    __syncthreads();
    int run = s_prefix + tex;
#pragma unroll
    for (int r = 0; r < kPrepPerThread; ++r) {
        const int64_t c = base + r;
        if (c < a.n_cells) {
            a.pair_off[c] = run;
            // chunks whose first pair lies in this cell start here
            if (cnt[r] > 0) {
                const int64_t j0 = ((int64_t)run + kChunk - 1) / kChunk;
                const int64_t j1 = ((int64_t)run + cnt[r] + kChunk - 1) / kChunk;
                for (int64_t j = j0; j < j1; ++j) a.chunk_cell[j] = (int32_t)c;
            }
        }
        run += cnt[r];
    }
    if (blockIdx.x == gridDim.x - 1) {
        // this block's inclusive prefix is the total pair count T
        const int T = s_prefix + block_total;
        if (threadIdx.x == 0) a.pair_off[a.n_cells] = T;
        const int64_t jt = ((int64_t)T + kChunk - 1) / kChunk;
        for (int64_t j = jt + threadIdx.x; j <= a.n_chunks; j += kPrepThreads)
            a.chunk_cell[j] = (int32_t)(a.n_cells - 1);
    }
}

// ---------------------------------------------------------------------------
// k_step
// ---------------------------------------------------------------------------
constexpr int kQueueCap = 2 * kChunk;  // holds < kChunk before a chunk adds <= kChunk

template <typename T>
struct FusedArgs {
    Particles<T> pt;
    const int64_t *off_e, *off_g;
    int64_t n_cells, n_chunks;
    int chunks_per_block;
    const int32_t* pair_off;
    const uint32_t* keys;
    const int32_t* chunk_cell;
    double dt, density_norm;
    uint64_t seed;
    StepControl* ctrl;
    BlockPartials part;
    cs_stats* stats;
    MlpDev mlp;  // network samplers only
};

// Resolve the n staged pairs at queue[0..n): the plain sampler, or the
// network (every entry of this stack lies in the network's domain).
template <typename T, int SAMP>
__device__ void drain(const FusedArgs<T>& a, const StagedPair<T>* queue, int n, uint64_t step, NetLds<SAMP>& s_net,
                      CollideSums& sums) {
    for (int base = 0; base < n; base += kChunk) {
        const int q = base + (int)threadIdx.x;
        // waves with no item skip the pass entirely
        if (__any(q < n)) {
            const bool active = q < n;
            const StagedPair<T>* e = queue + (active ? q : 0);
            if constexpr (SAMP == CS_SAMPLER_PLAIN)
                collide_staged<T>(a.pt, active, e, a.seed, step, sums);
            else
                collide_net<T, SAMP>(a.pt, active, FromStaged<T>{e}, s_net, a.mlp, a.seed, step, sums);
        }
    }
}

// Network samplers: the n pairs outside the network's domain, staged from
// the top of the queue down (queue[cap - 1 - q]), go to the plain sampler in
// dense passes.
template <typename T>
__device__ void drain_fallback(const FusedArgs<T>& a, const StagedPair<T>* queue, int n, uint64_t step,
                               CollideSums& sums) {
    for (int base = 0; base < n; base += kChunk) {
        const int q = base + (int)threadIdx.x;
        if (__any(q < n)) {
            const bool active = q < n;
            collide_staged<T>(a.pt, active, queue + (kQueueCap - 1 - (active ? q : 0)), a.seed, step, sums);
            sums.n_fallback += active ? 1 : 0;
        }
    }
}

template <typename T, int SAMP>
__global__ __launch_bounds__(kChunk) void k_step(const FusedArgs<T> a) {
    __shared__ StagedPair<T> s_queue[kQueueCap];
    __shared__ NetLds<SAMP> s_net;
    __shared__ int s_wcnt[2][kChunk / 64];
    __shared__ int s_qn, s_qf;
    __shared__ double s_red_d[3 * (kChunk / 64)];
    __shared__ long long s_red_i[4 * (kChunk / 64)];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    StepControl* ctrl = a.ctrl;
    const CtrlView cv = ctrl_view(ctrl);
    const uint32_t E = cv.epoch;
    const uint64_t step = cv.step;
    const bool layout_ok = cv.layout_ok;
    double sum_p = 0.0;
    long long n_clip = 0, n_inv = 0, n_coll = 0;
    CollideSums sums;
    if (tid == 0) s_qn = s_qf = 0;
    net_load<SAMP>(s_net, a.mlp);
    __syncthreads();
    if (layout_ok) {
        const int32_t T_total = a.pair_off[a.n_cells];
        const int64_t j_begin = (int64_t)blockIdx.x * a.chunks_per_block;
        int64_t j_end = j_begin + a.chunks_per_block;
        if (j_end > a.n_chunks) j_end = a.n_chunks;
        for (int64_t j = j_begin; j < j_end; ++j) {
            if (j * kChunk >= T_total) break;  // uniform over the block
            const int32_t t = (int32_t)(j * kChunk) + tid;
            const bool active = t < T_total;
            int c = 0;
            if (active) {
                int lo = a.chunk_cell[j], hi = a.chunk_cell[j + 1];
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (a.pair_off[mid] <= t)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                c = lo;
            }
            const PairOutcome o = pair_eval<T>(a.pt, active, a.off_e[c], a.off_e[c + 1], a.off_g[c], a.off_g[c + 1],
                                               a.keys + 4 * c, (uint32_t)(t - (active ? a.pair_off[c] : 0)), a.dt,
                                               a.density_norm, a.seed, step);
            sum_p += o.P;
            n_clip += o.clipped ? 1 : 0;
            n_inv += o.invalid ? 1 : 0;
            // accepted pairs are staged in LDS: from the bottom of the queue,
            // or (network samplers, x outside the network's domain) from the top
            bool to_fb = false;
            if constexpr (SAMP != CS_SAMPLER_PLAIN) to_fb = o.accept && !in_range((float)o.x, a.mlp.dom);
            const bool to_main = o.accept && !to_fb;
            const uint64_t lt = (1ull << lane) - 1ull;
            const uint64_t mask = __ballot(to_main), mask_fb = __ballot(to_fb);
            const int before = __popcll(mask & lt), before_fb = __popcll(mask_fb & lt);
            if (lane == 0) {
                s_wcnt[0][wave] = __popcll(mask);
                s_wcnt[1][wave] = __popcll(mask_fb);
            }
            __syncthreads();
            int wbase = 0, total = 0, wbase_fb = 0, total_fb = 0;
#pragma unroll
            for (int w = 0; w < kChunk / 64; ++w) {
                wbase += w < wave ? s_wcnt[0][w] : 0;
                total += s_wcnt[0][w];
                wbase_fb += w < wave ? s_wcnt[1][w] : 0;
                total_fb += s_wcnt[1][w];
            }
            const int qn = s_qn, qf = s_qf;
            if (o.accept) {
                StagedPair<T>& e = to_fb ? s_queue[kQueueCap - 1 - (qf + wbase_fb + before_fb)]
                                         : s_queue[qn + wbase + before];
                e.ie = o.ie;
                e.ig = o.ig;
                e.p[0] = a.pt.ex[o.ie];
                e.p[1] = a.pt.ey[o.ie];
                e.p[2] = a.pt.ez[o.ie];
                e.k[0] = a.pt.gx[o.ig];
                e.k[1] = a.pt.gy[o.ig];
                e.k[2] = a.pt.gz[o.ig];
                e.we = a.pt.ew[o.ie];
                e.wg = a.pt.gw[o.ig];
            }
            n_coll += o.accept ? 1 : 0;
            __syncthreads();
            // both stacks hold < kChunk entries together before a chunk adds
            // at most kChunk, so they never meet (kQueueCap = 2 kChunk)
            if (qn + total + qf + total_fb >= kChunk) {
                drain<T, SAMP>(a, s_queue, qn + total, step, s_net, sums);
                if constexpr (SAMP != CS_SAMPLER_PLAIN) drain_fallback<T>(a, s_queue, qf + total_fb, step, sums);
                __syncthreads();
                if (tid == 0) s_qn = s_qf = 0;
            } else if (tid == 0) {
                s_qn = qn + total;
                s_qf = qf + total_fb;
            }
            __syncthreads();
        }
        const int qn = s_qn, qf = s_qf;
        if (qn > 0) drain<T, SAMP>(a, s_queue, qn, step, s_net, sums);
        if constexpr (SAMP != CS_SAMPLER_PLAIN)
            if (qf > 0) drain_fallback<T>(a, s_queue, qf, step, sums);
    }
    // per-workgroup partials, fixed order: lanes (butterfly), then waves
    const double w_p = wave_sum(sum_p), w_eb = wave_sum(sums.e_before), w_ea = wave_sum(sums.e_after);
    const long long w_cl = wave_sum_i(n_clip), w_in = wave_sum_i(n_inv), w_co = wave_sum_i(n_coll);
    const long long w_fb = wave_sum_i(sums.n_fallback);
    if (lane == 0) {
        s_red_d[3 * wave + 0] = w_p;
        s_red_d[3 * wave + 1] = w_eb;
        s_red_d[3 * wave + 2] = w_ea;
        s_red_i[4 * wave + 0] = w_cl;
        s_red_i[4 * wave + 1] = w_in;
        s_red_i[4 * wave + 2] = w_co;
        s_red_i[4 * wave + 3] = w_fb;
    }
    __syncthreads();
    if (tid == 0) {
        double p = 0.0, eb = 0.0, ea = 0.0;
        long long cl = 0, in = 0, co = 0, fb = 0;
        for (int w = 0; w < kChunk / 64; ++w) {
            p += s_red_d[3 * w + 0];
            eb += s_red_d[3 * w + 1];
            ea += s_red_d[3 * w + 2];
            cl += s_red_i[4 * w + 0];
            in += s_red_i[4 * w + 1];
            co += s_red_i[4 * w + 2];
            fb += s_red_i[4 * w + 3];
        }
        const int b = blockIdx.x;
        a.part.prob[b] = p;
        a.part.e_before[b] = eb;
        a.part.e_after[b] = ea;
        a.part.clipped[b] = cl;
        a.part.invalid[b] = in;
        a.part.collided[b] = co;
        a.part.fallback[b] = fb;
    }
}

// ---------------------------------------------------------------------------
// k_finalize_step: one workgroup reduces the per-unit partial sums in a fixed
// order (thread stride, then lanes, then waves), writes cs_stats and advances
// the epoch and the device step counter.  Small on purpose: one accumulator
// per quantity keeps everything in registers.
// ---------------------------------------------------------------------------
constexpr int kFinalThreads = 256;

__global__ __launch_bounds__(kFinalThreads) void k_finalize_step(const FinalArgs a) {
    __shared__ double s_d[3][kFinalThreads / 64];
    __shared__ long long s_i[4][kFinalThreads / 64];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
    StepControl* ctrl = a.ctrl;
    const CtrlView cv = ctrl_view(ctrl);
    const uint32_t E = cv.epoch;
    const uint64_t step = cv.step;
    const int32_t np_read = a.pair_off[a.n_cells];  // (allocated for n_cells = 0 too)
    const int32_t n_pairs_raw = a.n_cells > 0 ? np_read : 0;
    const uint32_t n_acc_raw = ctrl->n_accepted;
    double sp = 0.0, eb = 0.0, ea = 0.0;
    long long cl = 0, in = 0, co = 0, fb = 0;
    // both partial sets in one pass, four entries of each per thread at a
    // time, every read of a batch issued before its sums (entries past an
    // array's end read as zeros, which leaves the sums unchanged: each thread
    // still adds its entries of an array in increasing order)
    const int64_t n_ab = a.n_a > a.n_b ? a.n_a : a.n_b;
    for (int64_t base = tid; base < n_ab; base += 4 * kFinalThreads) {
        double vp[4], ve[4], va[4];
        long long vc[4], vi[4], vo[4], vf[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int64_t i = base + (int64_t)k * kFinalThreads;
            const bool ia = i < a.n_a, ib = i < a.n_b;
            vp[k] = ia ? a.a_prob[i] : 0.0;
            vc[k] = ia ? a.a_clip[i] : 0;
            vi[k] = ia ? a.a_inv[i] : 0;
            vo[k] = ia && a.a_coll ? a.a_coll[i] : 0;
            ve[k] = ib ? a.b_eb[i] : 0.0;
            va[k] = ib ? a.b_ea[i] : 0.0;
            vf[k] = ib && a.b_fb ? a.b_fb[i] : 0;
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            sp += vp[k];
            cl += vc[k];
            in += vi[k];
            co += vo[k];
            eb += ve[k];
            ea += va[k];
            fb += vf[k];
        }
    }
    const bool layout_ok = cv.layout_ok;
    sp = wave_sum(sp);
    eb = wave_sum(eb);
    ea = wave_sum(ea);
    cl = wave_sum_i(cl);
    in = wave_sum_i(in);
    co = wave_sum_i(co);
    fb = wave_sum_i(fb);
    if (lane == 0) {
        s_d[0][wave] = sp;
        s_d[1][wave] = eb;
        s_d[2][wave] = ea;
        s_i[0][wave] = cl;
        s_i[1][wave] = in;
        s_i[2][wave] = co;
        s_i[3][wave] = fb;
    }
    __syncthreads();
    if (tid == 0) {
        cs_stats s = {};
        for (int w = 0; w < kFinalThreads / 64; ++w) {
            s.sum_prob += s_d[0][w];
            s.energy_before += s_d[1][w];
            s.energy_after += s_d[2][w];
            s.n_clipped += s_i[0][w];
            s.n_invalid += s_i[1][w];
            s.n_collided += s_i[2][w];
            s.n_fallback += s_i[3][w];
        }
        if (!a.a_coll) s.n_collided = (int64_t)n_acc_raw;
        s.n_pairs = n_pairs_raw;
        if (!layout_ok) {
            // no particle was touched: report the layout error only
            s = cs_stats{};
            s.layout_error = 1;
        }
        if (a.stats) *a.stats = s;
        ctrl->n_accepted = 0;
        ctrl->step = step + 1;
        ctrl->epoch = E + 1;
    }
}

hipError_t launch_finalize(const FinalArgs& f, hipStream_t st) {
    k_finalize_step<<<1, kFinalThreads, 0, st>>>(f);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// workspace and launcher
// ---------------------------------------------------------------------------
int64_t fused_prep_blocks(int64_t n_cells) { return (n_cells + kPrepCells - 1) / kPrepCells; }

static size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

size_t fused_workspace_bytes(const StepShape& s) {
    size_t b = 0;
    b += al(sizeof(int32_t) * (s.n_cells + 1));
    b += al(sizeof(uint32_t) * 4 * (s.n_cells > 0 ? s.n_cells : 1));
    b += al(sizeof(int32_t) * (s.n_chunks + 1));
    b += 7 * al(8 * s.n_step_blocks);
    return b;
}

void carve_fused_buffers(const Workspace& w, const StepShape& s, FusedBuffers* b) {
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
    b->part.prob = (double*)take(8 * s.n_step_blocks);
    b->part.e_before = (double*)take(8 * s.n_step_blocks);
    b->part.e_after = (double*)take(8 * s.n_step_blocks);
    b->part.clipped = (int64_t*)take(8 * s.n_step_blocks);
    b->part.invalid = (int64_t*)take(8 * s.n_step_blocks);
    b->part.collided = (int64_t*)take(8 * s.n_step_blocks);
    b->part.fallback = (int64_t*)take(8 * s.n_step_blocks);
}

hipError_t launch_prep(const StepShape& sh, StepControl* ctrl, uint64_t* status, int32_t* pair_off, uint32_t* keys,
                       int32_t* chunk_cell, const StepParams& p, hipStream_t st) {
    if (sh.n_cells <= 0) return hipSuccess;
    PrepArgs pa;
    pa.off_e = p.off_e;
    pa.off_g = p.off_g;
    pa.n_cells = sh.n_cells;
    pa.ne = sh.ne;
    pa.ng = sh.ng;
    pa.n_chunks = sh.n_chunks;
    pa.seed = p.seed;
    pa.step = p.step;
    pa.use_device_step = p.use_device_step;
    pa.pair_off = pair_off;
    pa.keys = keys;
    pa.chunk_cell = chunk_cell;
    pa.status = status;
    pa.ctrl = ctrl;
    k_prep_scan<<<(unsigned)fused_prep_blocks(sh.n_cells), kPrepThreads, 0, st>>>(pa);
    return hipGetLastError();
}

template <typename T, int SAMP>
static hipError_t launch_fused_t(const StepShape& sh, const FusedBuffers& b, const StepParams& p, hipStream_t st) {
    auto mark = [&](int i) {
        if (p.events) (void)hipEventRecord(p.events[i], st);
    };
    mark(0);
    hipError_t e = launch_prep(sh, b.ctrl, b.status, b.pair_off, b.cell_keys, b.chunk_cell, p, st);
    if (e != hipSuccess) return e;
    mark(1);
    FusedArgs<T> fa;
    fa.pt = {(T*)p.e.x, (T*)p.e.y, (T*)p.e.z, (T*)p.e.w, (T*)p.g.x, (T*)p.g.y, (T*)p.g.z, (T*)p.g.w};
    fa.off_e = p.off_e;
    fa.off_g = p.off_g;
    fa.n_cells = sh.n_cells;
    fa.n_chunks = sh.n_chunks;
    fa.chunks_per_block = sh.chunks_per_block;
    fa.pair_off = b.pair_off;
    fa.keys = b.cell_keys;
    fa.chunk_cell = b.chunk_cell;
    fa.dt = p.dt;
    fa.density_norm = p.density_norm;
    fa.seed = p.seed;
    fa.ctrl = b.ctrl;
    fa.part = b.part;
    fa.stats = p.stats;
    fa.mlp = p.net;
    k_step<T, SAMP><<<(unsigned)sh.n_step_blocks, kChunk, 0, st>>>(fa);
    mark(2);
    mark(3);
    mark(4);
    FinalArgs f = {};
    f.ctrl = b.ctrl;
    f.pair_off = b.pair_off;
    f.n_cells = sh.n_cells;
    f.a_prob = b.part.prob;
    f.a_clip = b.part.clipped;
    f.a_inv = b.part.invalid;
    f.a_coll = b.part.collided;
    f.n_a = sh.n_step_blocks;
    f.b_eb = b.part.e_before;
    f.b_ea = b.part.e_after;
    f.b_fb = b.part.fallback;
    f.n_b = sh.n_step_blocks;
    f.stats = p.stats;
    e = launch_finalize(f, st);
    mark(5);
    return e == hipSuccess ? hipGetLastError() : e;
}

template <typename T>
static hipError_t launch_fused_s(const StepShape& sh, const FusedBuffers& b, const StepParams& p, hipStream_t st) {
    switch (p.sampler) {
        case CS_SAMPLER_MLP_F32:
            return launch_fused_t<T, CS_SAMPLER_MLP_F32>(sh, b, p, st);
        case CS_SAMPLER_MLP_BF16:
            return launch_fused_t<T, CS_SAMPLER_MLP_BF16>(sh, b, p, st);
        case CS_SAMPLER_MLP_FP8:
            return launch_fused_t<T, CS_SAMPLER_MLP_FP8>(sh, b, p, st);
        default:
            return launch_fused_t<T, CS_SAMPLER_PLAIN>(sh, b, p, st);
    }
}

hipError_t launch_fused(const StepShape& sh, const FusedBuffers& b, const StepParams& p, hipStream_t st) {
    if (p.dtype == CS_F64) return launch_fused_s<double>(sh, b, p, st);
    return launch_fused_s<float>(sh, b, p, st);
}

// ---------------------------------------------------------------------------
// k_cell_baseline: the straightforward mapping, one workgroup per cell
// walking its pairs 256 at a time and resolving each accepted pair in the
// lane that found it (no compaction, so the sampler runs on mostly idle
// waves).  A baseline for the batched strategies; same per-pair code, so the
// same results.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kChunk) void k_cell_baseline(const FusedArgs<T> a) {
    __shared__ double s_red_d[3 * (kChunk / 64)];
    __shared__ long long s_red_i[3 * (kChunk / 64)];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int64_t c = blockIdx.x;
    StepControl* ctrl = a.ctrl;
    const CtrlView cv = ctrl_view(ctrl);
    const uint64_t step = cv.step;
    const bool layout_ok = cv.layout_ok;
    double sum_p = 0.0;
    long long n_clip = 0, n_inv = 0, n_coll = 0;
    CollideSums sums;
    if (layout_ok && c < a.n_cells) {
        const int32_t np = a.pair_off[c + 1] - a.pair_off[c];
        const int64_t e0 = a.off_e[c], e1 = a.off_e[c + 1], g0 = a.off_g[c], g1 = a.off_g[c + 1];
        for (int32_t base = 0; base < np; base += kChunk) {
            const int32_t i = base + tid;
            const bool active = i < np;
            const PairOutcome o = pair_eval<T>(a.pt, active, e0, e1, g0, g1, a.keys + 4 * c, (uint32_t)(active ? i : 0),
                                               a.dt, a.density_norm, a.seed, step);
            sum_p += o.P;
            n_clip += o.clipped ? 1 : 0;
            n_inv += o.invalid ? 1 : 0;
            n_coll += o.accept ? 1 : 0;
            collide_plain<T>(a.pt, o.accept, o.ie, o.ig, a.seed, step, sums);
        }
    }
    const double w_p = wave_sum(sum_p), w_eb = wave_sum(sums.e_before), w_ea = wave_sum(sums.e_after);
    const long long w_cl = wave_sum_i(n_clip), w_in = wave_sum_i(n_inv), w_co = wave_sum_i(n_coll);
    if (lane == 0) {
        s_red_d[3 * wave + 0] = w_p;
        s_red_d[3 * wave + 1] = w_eb;
        s_red_d[3 * wave + 2] = w_ea;
        s_red_i[3 * wave + 0] = w_cl;
        s_red_i[3 * wave + 1] = w_in;
        s_red_i[3 * wave + 2] = w_co;
    }
    __syncthreads();
    if (tid == 0) {
        double p = 0.0, eb = 0.0, ea = 0.0;
        long long cl = 0, in = 0, co = 0;
        for (int w = 0; w < kChunk / 64; ++w) {
            p += s_red_d[3 * w + 0];
            eb += s_red_d[3 * w + 1];
            ea += s_red_d[3 * w + 2];
            cl += s_red_i[3 * w + 0];
            in += s_red_i[3 * w + 1];
            co += s_red_i[3 * w + 2];
        }
        const int64_t b = blockIdx.x;
        a.part.prob[b] = p;
        a.part.e_before[b] = eb;
        a.part.e_after[b] = ea;
        a.part.clipped[b] = cl;
        a.part.invalid[b] = in;
        a.part.collided[b] = co;
        a.part.fallback[b] = 0;
    }
}

template <typename T>
static hipError_t launch_cell_t(const StepShape& sh, const FusedBuffers& b, const StepParams& p, hipStream_t st) {
    auto mark = [&](int i) {
        if (p.events) (void)hipEventRecord(p.events[i], st);
    };
    mark(0);
    hipError_t e = launch_prep(sh, b.ctrl, b.status, b.pair_off, b.cell_keys, b.chunk_cell, p, st);
    if (e != hipSuccess) return e;
    mark(1);
    FusedArgs<T> fa = {};
    fa.pt = {(T*)p.e.x, (T*)p.e.y, (T*)p.e.z, (T*)p.e.w, (T*)p.g.x, (T*)p.g.y, (T*)p.g.z, (T*)p.g.w};
    fa.off_e = p.off_e;
    fa.off_g = p.off_g;
    fa.n_cells = sh.n_cells;
    fa.n_chunks = sh.n_chunks;
    fa.chunks_per_block = 1;
    fa.pair_off = b.pair_off;
    fa.keys = b.cell_keys;
    fa.chunk_cell = b.chunk_cell;
    fa.dt = p.dt;
    fa.density_norm = p.density_norm;
    fa.seed = p.seed;
    fa.ctrl = b.ctrl;
    fa.part = b.part;
    fa.stats = p.stats;
    if (sh.n_cells > 0) k_cell_baseline<T><<<(unsigned)sh.n_cells, kChunk, 0, st>>>(fa);
    mark(2);
    mark(3);
    mark(4);
    FinalArgs f = {};
    f.ctrl = b.ctrl;
    f.pair_off = b.pair_off;
    f.n_cells = sh.n_cells;
    f.a_prob = b.part.prob;
    f.a_clip = b.part.clipped;
    f.a_inv = b.part.invalid;
    f.a_coll = b.part.collided;
    f.n_a = sh.n_cells > 0 ? sh.n_cells : 0;
    f.b_eb = b.part.e_before;
    f.b_ea = b.part.e_after;
    f.b_fb = b.part.fallback;
    f.n_b = f.n_a;
    f.stats = p.stats;
    e = launch_finalize(f, st);
    mark(5);
    return e == hipSuccess ? hipGetLastError() : e;
}

hipError_t launch_cell(const StepShape& sh, const FusedBuffers& b, const StepParams& p, hipStream_t st) {
    if (p.dtype == CS_F64) return launch_cell_t<double>(sh, b, p, st);
    return launch_cell_t<float>(sh, b, p, st);
}

}  // namespace cs
