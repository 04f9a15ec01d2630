// cs_step.hip -- kernels of one Compton step on gfx950 and their launcher.
//
// Data flow of a step (all on the caller's stream):
//   k_reset        clear the layout flag
//   k_cell_prep    per cell: validate offsets, pairs = min(N_e, N_g), pairing key
//   scan           pair offsets per cell (3-kernel exclusive scan)
//   k_chunk_cells  first cell of every 256-pair chunk (binary search)
//   k_pair         one lane per pair: pairing, x, s(x), P, accept; accepted
//                  pairs compacted per chunk with a wavefront ballot
//   scan           offsets of the accepted pairs per chunk
//   k_collide      one lane per accepted pair (dense): sample mu, scatter,
//                  back-boost, write back in place
//   k_finalize     fixed-order reduction of the per-chunk / per-block partials
// Every reduction has a fixed order, so a step is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_pair.h"

namespace cs {

// ---------------------------------------------------------------------------
// workspace carving
// ---------------------------------------------------------------------------
static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t step_workspace_bytes(const StepShape& s) {
    size_t b = 0;
    b += align_up(sizeof(int32_t));                               // flag
    b += align_up(sizeof(int32_t) * s.n_cells);                   // cell_np
    b += align_up(sizeof(int32_t) * (s.n_cells + 1));             // pair_off
    b += align_up(sizeof(uint32_t) * 4 * s.n_cells);              // keys
    b += align_up(sizeof(int32_t) * (s.n_chunks + 1));            // chunk_cell
    b += align_up(sizeof(int2) * s.n_chunks * kChunk);            // acc_list
    b += align_up(sizeof(int32_t) * s.n_chunks);                  // acc_cnt
    b += align_up(sizeof(int32_t) * (s.n_chunks + 1));            // acc_off
    b += align_up(sizeof(double) * s.n_chunks);                   // part_prob
    b += align_up(sizeof(int32_t) * s.n_chunks);                  // part_clip
    b += align_up(sizeof(int32_t) * s.n_chunks);                  // part_inv
    b += align_up(sizeof(double) * 2 * s.n_collide_blocks);       // part_energy
    b += align_up(sizeof(int32_t) * s.n_collide_blocks);          // part_fallback
    b += align_up(sizeof(int32_t) * s.scan_tmp_len);              // scan_tmp
    return b;
}

void carve_step_buffers(void* base, const StepShape& s, StepBuffers* b) {
    char* p = (char*)base;
    auto take = [&](size_t n) {
        char* r = p;
        p += align_up(n);
        return (void*)r;
    };
    b->flag = (int32_t*)take(sizeof(int32_t));
    b->cell_np = (int32_t*)take(sizeof(int32_t) * s.n_cells);
    b->pair_off = (int32_t*)take(sizeof(int32_t) * (s.n_cells + 1));
    b->cell_keys = (uint32_t*)take(sizeof(uint32_t) * 4 * s.n_cells);
    b->chunk_cell = (int32_t*)take(sizeof(int32_t) * (s.n_chunks + 1));
    b->acc_list = (int2*)take(sizeof(int2) * s.n_chunks * kChunk);
    b->acc_cnt = (int32_t*)take(sizeof(int32_t) * s.n_chunks);
    b->acc_off = (int32_t*)take(sizeof(int32_t) * (s.n_chunks + 1));
    b->part_prob = (double*)take(sizeof(double) * s.n_chunks);
    b->part_clip = (int32_t*)take(sizeof(int32_t) * s.n_chunks);
    b->part_inv = (int32_t*)take(sizeof(int32_t) * s.n_chunks);
    b->part_energy = (double*)take(sizeof(double) * 2 * s.n_collide_blocks);
    b->part_fallback = (int32_t*)take(sizeof(int32_t) * s.n_collide_blocks);
    b->scan_tmp = (int32_t*)take(sizeof(int32_t) * s.scan_tmp_len);
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (3 kernels); out has n + 1 entries, out[n] = total
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_scan_reduce(const int32_t* __restrict__ in, int64_t n,
                                                     int32_t* __restrict__ bsum) {
    __shared__ long long lds[256];
    const int64_t base = (int64_t)blockIdx.x * kScanItems;
    long long s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems / 256; ++r) {
        const int64_t i = base + r * 256 + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = block_sum_i(s, lds);
    if (threadIdx.x == 0) bsum[blockIdx.x] = (int32_t)s;
}

__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ bsum, int64_t nb) {
    __shared__ int lds[17];
    int carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const int v = i < nb ? bsum[i] : 0;
        int tot;
        const int ex = block_exclusive_scan(v, lds, &tot);
        if (i < nb) bsum[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) bsum[nb] = carry;
}

__global__ __launch_bounds__(256) void k_scan_apply(const int32_t* __restrict__ in, int64_t n,
                                                    const int32_t* __restrict__ bsum, int64_t nb,
                                                    int32_t* __restrict__ out) {
    __shared__ int lds[5];
    const int64_t base = (int64_t)blockIdx.x * kScanItems + (int64_t)threadIdx.x * (kScanItems / 256);
    int v[kScanItems / 256];
    int s = 0;
#pragma unroll
    for (int r = 0; r < kScanItems / 256; ++r) {
        const int64_t i = base + r;
        v[r] = i < n ? in[i] : 0;
        s += v[r];
    }
    int ex = block_exclusive_scan(s, lds, nullptr) + bsum[blockIdx.x];
#pragma unroll
    for (int r = 0; r < kScanItems / 256; ++r) {
        const int64_t i = base + r;
        if (i < n) out[i] = ex;
        ex += v[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = bsum[nb];
}

static hipError_t exclusive_scan(const int32_t* in, int64_t n, int32_t* out, int32_t* tmp, hipStream_t st) {
    const int64_t nb = (n + kScanItems - 1) / kScanItems;
    const int64_t nb1 = nb > 0 ? nb : 1;
    if (nb > 0) k_scan_reduce<<<dim3((unsigned)nb), dim3(256), 0, st>>>(in, n, tmp);
    k_scan_top<<<1, 1024, 0, st>>>(tmp, nb);
    k_scan_apply<<<dim3((unsigned)nb1), dim3(256), 0, st>>>(in, n, tmp, nb, out);
    return hipGetLastError();
}

static int64_t scan_tmp_needed(int64_t n) { return (n + kScanItems - 1) / kScanItems + 2; }

// ---------------------------------------------------------------------------
// step kernels
// ---------------------------------------------------------------------------
__global__ void k_reset(int32_t* flag) { *flag = 0; }

__global__ __launch_bounds__(256) void k_cell_prep(const int64_t* __restrict__ off_e,
                                                   const int64_t* __restrict__ off_g, int64_t n_cells,
                                                   int64_t ne, int64_t ng, uint64_t seed, uint64_t step,
                                                   int32_t* __restrict__ cell_np, uint32_t* __restrict__ keys,
                                                   int32_t* __restrict__ flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    const int64_t a0 = off_e[c], a1 = off_e[c + 1], b0 = off_g[c], b1 = off_g[c + 1];
    bool bad = a1 < a0 || b1 < b0;
    if (c == 0) bad = bad || a0 != 0 || b0 != 0;
    if (c == n_cells - 1) bad = bad || a1 != ne || b1 != ng;
    if (bad) {
        atomicOr(flag, 1);
        cell_np[c] = 0;
        return;
    }
    const int64_t nmin = (a1 - a0) < (b1 - b0) ? (a1 - a0) : (b1 - b0);
    cell_np[c] = (int32_t)nmin;
    if (nmin > 0) {
        const u32x4 r = draw(seed, (uint64_t)c, step, kPair);
        keys[4 * c + 0] = r.a;
        keys[4 * c + 1] = r.b;
        keys[4 * c + 2] = r.c;
        keys[4 * c + 3] = r.d;
    }
}

__global__ __launch_bounds__(256) void k_chunk_cells(const int32_t* __restrict__ pair_off, int64_t n_cells,
                                                     int64_t n_chunks, int32_t* __restrict__ chunk_cell) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j > n_chunks) return;
    const int64_t T = pair_off[n_cells];
    const int64_t t = j * kChunk;
    if (t >= T) {
        chunk_cell[j] = (int32_t)(n_cells - 1);
        return;
    }
    // largest c in [0, n_cells) with pair_off[c] <= t: the non-empty cell holding pair t
    int64_t lo = 0, hi = n_cells - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (pair_off[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    chunk_cell[j] = (int32_t)lo;
}

template <typename T>
struct PairArgs {
    Particles<T> pt;
    const int64_t *off_e, *off_g;
    int64_t n_cells;
    const int32_t* pair_off;
    const uint32_t* keys;
    const int32_t* chunk_cell;
    const int32_t* flag;
    double dt, density_norm;
    uint64_t seed, step;
    int2* acc_list;
    int32_t* acc_cnt;
    double* part_prob;
    int32_t* part_clip;
    int32_t* part_inv;
};

// Multi-kernel baseline, stage 1: one lane per pair, accepted pairs compacted
// per 256-pair chunk into its own list segment (pair order, no atomics).
template <typename T>
__global__ __launch_bounds__(kChunk) void k_pair(const PairArgs<T> a) {
    __shared__ double s_red[kChunk];
    __shared__ long long s_redi[kChunk];
    __shared__ int s_wcnt[kChunk / 64 + 1];
    const int j = blockIdx.x;
    const int tid = threadIdx.x;
    if (*a.flag) {
        if (tid == 0) {
            a.acc_cnt[j] = 0;
            a.part_prob[j] = 0.0;
            a.part_clip[j] = 0;
            a.part_inv[j] = 0;
        }
        return;
    }
    const int32_t T_total = a.pair_off[a.n_cells];
    const int32_t t = j * kChunk + tid;
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
    const PairOutcome o =
        pair_eval<T>(a.pt, active, a.off_e[c], a.off_e[c + 1], a.off_g[c], a.off_g[c + 1], a.keys + 4 * c,
                     (uint32_t)(t - (active ? a.pair_off[c] : 0)), a.dt, a.density_norm, a.seed, a.step);
    const uint64_t mask = __ballot(o.accept);
    const int lane = lane_id();
    const int wave = tid >> 6;
    const int before = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane == 0) s_wcnt[wave] = __popcll(mask);
    __syncthreads();
    int wbase = 0, total = 0;
    for (int w = 0; w < kChunk / 64; ++w) {
        if (w < wave) wbase += s_wcnt[w];
        total += s_wcnt[w];
    }
    if (o.accept) a.acc_list[(int64_t)j * kChunk + wbase + before] = make_int2(o.ie, o.ig);
    const double sp = block_sum(o.P, s_red);
    const long long sc = block_sum_i(o.clipped ? 1 : 0, s_redi);
    const long long si = block_sum_i(o.invalid ? 1 : 0, s_redi);
    if (tid == 0) {
        a.acc_cnt[j] = total;
        a.part_prob[j] = sp;
        a.part_clip[j] = (int32_t)sc;
        a.part_inv[j] = (int32_t)si;
    }
}

template <typename T>
struct CollideArgs {
    Particles<T> pt;
    const int2* acc_list;
    const int32_t* acc_off;
    int64_t n_chunks;
    const int32_t* flag;
    uint64_t seed, step;
    double* part_energy;
    int32_t* part_fallback;
};

// Multi-kernel baseline, stage 3: one lane per accepted pair, grid-stride.
template <typename T>
__global__ __launch_bounds__(256) void k_collide(const CollideArgs<T> a) {
    __shared__ double s_red[256];
    const int tid = threadIdx.x;
    CollideSums sums;
    if (!*a.flag) {
        const int64_t A = a.acc_off[a.n_chunks];
        const int64_t stride = (int64_t)gridDim.x * 256;
        const int64_t n_iter = (A + stride - 1) / stride;  // uniform over the grid
        for (int64_t it = 0; it < n_iter; ++it) {
            const int64_t q = it * stride + (int64_t)blockIdx.x * 256 + tid;
            const bool active = q < A;
            int2 pr = make_int2(0, 0);
            if (active) {
                int64_t lo = 0, hi = a.n_chunks - 1;  // largest j with acc_off[j] <= q
                while (lo < hi) {
                    const int64_t mid = (lo + hi + 1) >> 1;
                    if (a.acc_off[mid] <= q)
                        lo = mid;
                    else
                        hi = mid - 1;
                }
                pr = a.acc_list[lo * kChunk + (q - a.acc_off[lo])];
            }
            collide_plain<T>(a.pt, active, pr.x, pr.y, a.seed, a.step, sums);
        }
    }
    const double eb = block_sum(sums.e_before, s_red);
    const double ea = block_sum(sums.e_after, s_red);
    if (tid == 0) {
        a.part_energy[2 * blockIdx.x] = eb;
        a.part_energy[2 * blockIdx.x + 1] = ea;
        a.part_fallback[blockIdx.x] = 0;
    }
}

__global__ __launch_bounds__(256) void k_finalize(const int32_t* __restrict__ flag, const int32_t* __restrict__ pair_off,
                                                  int64_t n_cells, const int32_t* __restrict__ acc_off,
                                                  int64_t n_chunks, const double* __restrict__ part_prob,
                                                  const int32_t* __restrict__ part_clip,
                                                  const int32_t* __restrict__ part_inv,
                                                  const double* __restrict__ part_energy,
                                                  const int32_t* __restrict__ part_fallback, int64_t n_blocks,
                                                  cs_stats* __restrict__ out) {
    __shared__ double s_red[256];
    __shared__ long long s_redi[256];
    const int tid = threadIdx.x;
    const bool bad = *flag != 0;
    double sp = 0.0, eb = 0.0, ea = 0.0;
    long long clip = 0, inv = 0, fb = 0;
    if (!bad) {
        for (int64_t j = tid; j < n_chunks; j += 256) {
            sp += part_prob[j];
            clip += part_clip[j];
            inv += part_inv[j];
        }
        for (int64_t b = tid; b < n_blocks; b += 256) {
            eb += part_energy[2 * b];
            ea += part_energy[2 * b + 1];
            fb += part_fallback[b];
        }
    }
    sp = block_sum(sp, s_red);
    eb = block_sum(eb, s_red);
    ea = block_sum(ea, s_red);
    clip = block_sum_i(clip, s_redi);
    inv = block_sum_i(inv, s_redi);
    fb = block_sum_i(fb, s_redi);
    if (tid == 0) {
        cs_stats s = {};
        s.n_pairs = bad || n_cells == 0 ? 0 : pair_off[n_cells];
        s.n_collided = bad || n_chunks == 0 ? 0 : acc_off[n_chunks];
        s.n_clipped = clip;
        s.n_invalid = inv;
        s.n_fallback = fb;
        s.layout_error = bad ? 1 : 0;
        s.sum_prob = sp;
        s.energy_before = eb;
        s.energy_after = ea;
        *out = s;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void k_sample_plain(const T* __restrict__ x, const T* __restrict__ u, int64_t n,
                                                      T* __restrict__ mu_out, T* __restrict__ ratio_out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double xi = (double)x[i];
        const double v = angle_icdf_v((double)u[i], xi);
        mu_out[i] = (T)(1.0 - v);
        ratio_out[i] = (T)(1.0 / (1.0 + xi * v));
    }
}

// Rest-frame photon energy x of the pairs (electron i, photon i), FP64,
// cancellation-free (the step's own evaluation).
template <typename T>
__global__ __launch_bounds__(256) void k_pair_x(const T* __restrict__ px, const T* __restrict__ py,
                                                const T* __restrict__ pz, const T* __restrict__ kx,
                                                const T* __restrict__ ky, const T* __restrict__ kz, int64_t n,
                                                double* __restrict__ x_out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const d3 p = {(double)px[i], (double)py[i], (double)pz[i]};
        const d3 k = {(double)kx[i], (double)ky[i], (double)kz[i]};
        x_out[i] = pair_invariants(p, k).x;
    }
}

__global__ __launch_bounds__(256) void k_check_layout(const int64_t* __restrict__ off, int64_t n_cells, int64_t n,
                                                      int32_t* __restrict__ flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n_cells) return;
    bool bad = false;
    if (c == 0) bad = off[0] != 0;
    if (c == n_cells) bad = bad || off[n_cells] != n;
    if (c < n_cells) bad = bad || off[c + 1] < off[c];
    if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

template <typename T>
static hipError_t launch_step_t(const StepShape& sh, const StepBuffers& b, const StepParams& p, hipStream_t st) {
    auto mark = [&](int i) {
        if (p.events) (void)hipEventRecord(p.events[i], st);
    };
    mark(0);
    k_reset<<<1, 1, 0, st>>>(b.flag);
    if (sh.n_cells > 0) {
        k_cell_prep<<<blocks_for(sh.n_cells, 256), 256, 0, st>>>(p.off_e, p.off_g, sh.n_cells, sh.ne, sh.ng, p.seed,
                                                                 p.step, b.cell_np, b.cell_keys, b.flag);
        hipError_t e = exclusive_scan(b.cell_np, sh.n_cells, b.pair_off, b.scan_tmp, st);
        if (e != hipSuccess) return e;
    }
    if (sh.n_chunks > 0)
        k_chunk_cells<<<blocks_for(sh.n_chunks + 1, 256), 256, 0, st>>>(b.pair_off, sh.n_cells, sh.n_chunks,
                                                                         b.chunk_cell);
    mark(1);
    if (sh.n_chunks > 0) {
        PairArgs<T> pa;
        pa.pt = {(T*)p.e.x, (T*)p.e.y, (T*)p.e.z, (T*)p.e.w, (T*)p.g.x, (T*)p.g.y, (T*)p.g.z, (T*)p.g.w};
        pa.off_e = p.off_e;
        pa.off_g = p.off_g;
        pa.n_cells = sh.n_cells;
        pa.pair_off = b.pair_off;
        pa.keys = b.cell_keys;
        pa.chunk_cell = b.chunk_cell;
        pa.flag = b.flag;
        pa.dt = p.dt;
        pa.density_norm = p.density_norm;
        pa.seed = p.seed;
        pa.step = p.step;
        pa.acc_list = b.acc_list;
        pa.acc_cnt = b.acc_cnt;
        pa.part_prob = b.part_prob;
        pa.part_clip = b.part_clip;
        pa.part_inv = b.part_inv;
        k_pair<T><<<(unsigned)sh.n_chunks, kChunk, 0, st>>>(pa);
        mark(2);
        hipError_t e = exclusive_scan(b.acc_cnt, sh.n_chunks, b.acc_off, b.scan_tmp, st);
        if (e != hipSuccess) return e;
        mark(3);
        CollideArgs<T> ca;
        ca.pt = pa.pt;
        ca.acc_list = b.acc_list;
        ca.acc_off = b.acc_off;
        ca.n_chunks = sh.n_chunks;
        ca.flag = b.flag;
        ca.seed = p.seed;
        ca.step = p.step;
        ca.part_energy = b.part_energy;
        ca.part_fallback = b.part_fallback;
        k_collide<T><<<(unsigned)sh.n_collide_blocks, 256, 0, st>>>(ca);
        mark(4);
    } else {
        mark(2);
        mark(3);
        mark(4);
    }
    if (p.stats)
        k_finalize<<<1, 256, 0, st>>>(b.flag, b.pair_off, sh.n_cells, b.acc_off, sh.n_chunks, b.part_prob, b.part_clip,
                                      b.part_inv, b.part_energy, b.part_fallback,
                                      sh.n_chunks > 0 ? sh.n_collide_blocks : 0, p.stats);
    mark(5);
    return hipGetLastError();
}

hipError_t launch_step(const StepShape& sh, const StepBuffers& b, const StepParams& p, hipStream_t st) {
    if (p.dtype == CS_F64) return launch_step_t<double>(sh, b, p, st);
    return launch_step_t<float>(sh, b, p, st);
}

hipError_t launch_check_layout(const int64_t* off, int64_t n_cells, int64_t n, int32_t* flag, hipStream_t st) {
    k_reset<<<1, 1, 0, st>>>(flag);
    k_check_layout<<<blocks_for(n_cells + 1, 256), 256, 0, st>>>(off, n_cells, n, flag);
    return hipGetLastError();
}

hipError_t launch_sample_plain(cs_dtype dtype, const void* x, const void* u, int64_t n, void* mu, void* ratio,
                               hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    const unsigned grid = (unsigned)(nb < 65536 ? nb : 65536);
    if (dtype == CS_F64)
        k_sample_plain<double><<<grid, 256, 0, st>>>((const double*)x, (const double*)u, n, (double*)mu,
                                                     (double*)ratio);
    else
        k_sample_plain<float><<<grid, 256, 0, st>>>((const float*)x, (const float*)u, n, (float*)mu, (float*)ratio);
    return hipGetLastError();
}

hipError_t launch_pair_x(cs_dtype dtype, const cs_species& e, const cs_species& g, int64_t n, double* x_out,
                         hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    const unsigned grid = (unsigned)(nb < 65536 ? nb : 65536);
    if (dtype == CS_F64)
        k_pair_x<double><<<grid, 256, 0, st>>>((const double*)e.x, (const double*)e.y, (const double*)e.z,
                                               (const double*)g.x, (const double*)g.y, (const double*)g.z, n, x_out);
    else
        k_pair_x<float><<<grid, 256, 0, st>>>((const float*)e.x, (const float*)e.y, (const float*)e.z,
                                              (const float*)g.x, (const float*)g.y, (const float*)g.z, n, x_out);
    return hipGetLastError();
}

int64_t step_scan_tmp_len(int64_t n_cells, int64_t n_chunks) {
    const int64_t a = scan_tmp_needed(n_cells), b = scan_tmp_needed(n_chunks);
    return a > b ? a : b;
}

}  // namespace cs
