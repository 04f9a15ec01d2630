// cs_ntc.hip -- no-time-counter candidate selection (the NTC method of Bird
// that Sec. 3.1 names to shorten each cell's pair list) with the probability
// and bound of Sec. 3.2.
//
// Per cell c with N_e electrons, N_g photons and W the largest valid weight
// among them: P_max = 2 dt n W bounds the pair probability
// P = dt n max(w_e, w_g) s(x) flux (s <= 1, flux <= 2); the cell draws
// N_e N_g P_max candidates rounded stochastically, each an electron and a
// photon picked uniformly with replacement and accepted with probability
// P / P_max.  The candidates of a cell are taken in order, each on the
// momenta the earlier collisions of its cell left (Bird's sequential scheme).
//
// Data-parallel form.  A candidate's outcome depends only on its own two
// particles, so candidates that share no particle commute, and any order
// in which each candidate follows every earlier candidate of its cell that
// shares a particle with it gives the sequential result.  Rounds:
//   k_ntc_count    one wave per cell: W (wave max), P_max, the count
//   k_ntc_scan_*   candidate offsets (int64 exclusive scan over cells, the
//                  block offsets added by k_ntc_pick); the
//                  host reads the total (one stream synchronisation)
//   k_ntc_pick     one wave per cell: its candidates' electrons and
//                  photons.  A cell of at most 64 candidates is settled in
//                  the wave: candidates sharing no particle with an earlier
//                  one are evaluated (probability, accept) and the accepted
//                  ones listed; the others register for round 1 in the
//                  particles' "first toucher" words (atomicMax of (round
//                  tag << 32 | ~candidate): each word ends up holding the
//                  earliest candidate that touches the particle).  Larger
//                  cells register every candidate for round 0.
//   k_ntc_collide_list  the listed accepted candidates, one per lane:
//                  scattering and write-back (listing them first keeps the
//                  long collision path off the lanes that only evaluate)
//   k_ntc_round t  per unresolved candidate: ready when it is the earliest
//                  unresolved toucher of both its particles; ready ones are
//                  evaluated; round 0 (run only when a cell has more than
//                  64 candidates) lists its accepted ones for the dense
//                  collide, later rounds, with few candidates left, collide
//                  them in place; the others register for round t + 1 in
//                  the other word set (two sets alternate, so a round never
//                  reads a word that the same round writes); after the last
//                  round they mark their cell
//   k_ntc_serial   one wave per marked cell; its lane 0 resolves the
//                  cell's remaining candidates in order (long chains: a
//                  cell with one electron and many candidates)
//   k_ntc_reduce / k_ntc_final  fixed-order sums into cs_stats
// Tags grow by one per round and never repeat (a per-context epoch), so the
// touch words are never cleared between steps.
//
// Random numbers: Philox4x32-10 as elsewhere; the count from
// (cell, kNtcCount), candidate l of cell c from index (c << 32) | l with
// kNtcPick (electron (r0 N_e) >> 32, photon (r1 N_g) >> 32, acceptance
// uniform from r2, r3), kNtcScatter (u_mu, u_phi) and kNtcWeight.
#include <hip/hip_runtime.h>

#include "cs_block.h"
#include "cs_device.h"
#include "cs_internal.h"
#include "cs_pair.h"

namespace cs {

constexpr int kNtcThreads = 256;
constexpr int kNtcRounds = 3;
constexpr int kNtcScanPer = 4;                              // cells per thread in the scan
constexpr int kNtcScanBlock = kNtcThreads * kNtcScanPer;   // cells per scan workgroup
constexpr int kNtcRedPer = 2;                               // candidates per thread in the reduction
constexpr int64_t kNtcMaxCand = 2147483647;                 // candidates per step: below 2^31 - 1

// Control words of a step: flags and the total for the host, the list
// counts of the rounds.  Zero at the start of every step: zeroed when
// allocated and by k_ntc_final at the end of the previous step (they sit at
// the start of the per-cell scratch, whatever the cell count).
struct NtcCtl {
    long long total;
    int32_t layout_bad;
    int32_t too_many;
    int32_t has_large;  // a cell with more than 64 candidates
    int32_t pad;
};

struct NtcPart {
    double prob, eb, ea;
    long long coll, inv, clip;
};

template <typename T>
struct NtcArgs {
    Particles<T> pt;
    const int64_t *off_e, *off_g;
    int64_t n_cells, total;
    double dt, dn;
    uint64_t seed, step;
    uint32_t epoch;
    const int64_t* cand_off;  // [n_cells + 1] prefixes within each scan block
    int64_t* cand_full;       // [n_cells + 1] candidate offsets (written by k_ntc_pick)
    const double* p_max;      // [n_cells]
    int32_t *c_ie, *c_ig, *c_cell, *c_local;
    double* c_u;              // acceptance uniform of each candidate
    const long long* boff;    // block offsets of the candidate scan (cand_off holds block-local prefixes)
    uint8_t* status;  // bit 0 resolved; 2 collided, 4 invalid, 8 P > P_max
    double *r_ratio, *r_eb, *r_ea;
    unsigned long long *touch_e, *touch_g;  // [2][cap_e], [2][cap_g]
    int64_t cap_e, cap_g;
    uint8_t* pending;    // [n_cells]
    int32_t* list;       // round 0's accepted candidates, a 256-entry segment per round workgroup
    int32_t* seg_cnt;    // [round workgroups]: entries of each segment
    int64_t list_len, n_round_blocks;
    int32_t *pick_list, *pick_cnt;  // accepted candidates of the pick kernel: 256 per pick workgroup
};

__device__ __forceinline__ unsigned long long ntc_tag(uint32_t round_tag, int64_t j) {
    return ((unsigned long long)round_tag << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
}

template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_count(const T* ew, const T* gw, const int64_t* off_e,
                                                         const int64_t* off_g, int64_t n_cells, int64_t ne,
                                                         int64_t ng, double dt, double dn, uint64_t seed,
                                                         uint64_t step, int64_t* count, double* p_max,
                                                         uint8_t* pending, NtcCtl* ctl) {
    const int lane = lane_id();
    const int64_t c = (int64_t)blockIdx.x * (kNtcThreads / 64) + (threadIdx.x >> 6);
    if (c >= n_cells) return;
    if (lane == 0) pending[c] = 0;
    const int64_t e0 = off_e[c], e1 = off_e[c + 1], g0 = off_g[c], g1 = off_g[c + 1];
    const bool bad = e0 < 0 || e1 < e0 || e1 > ne || g0 < 0 || g1 < g0 || g1 > ng ||
                     (c == 0 && (e0 != 0 || g0 != 0)) || (c == n_cells - 1 && (e1 != ne || g1 != ng));
    if (bad) {
        if (lane == 0) {
            ctl->layout_bad = 1;
            count[c] = 0;
            p_max[c] = 0.0;
        }
        return;
    }
    // largest finite non-negative weight; four reads in flight per lane (a
    // maximum does not depend on the order)
    double w = 0.0;
    auto scan = [&](const T* arr, int64_t b, int64_t end) {
        double m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0;
        int64_t i = b + lane;
        for (; i + 192 < end; i += 256) {
            const double v0 = (double)arr[i], v1 = (double)arr[i + 64], v2 = (double)arr[i + 128],
                         v3 = (double)arr[i + 192];
            if (isfinite(v0) && v0 > m0) m0 = v0;
            if (isfinite(v1) && v1 > m1) m1 = v1;
            if (isfinite(v2) && v2 > m2) m2 = v2;
            if (isfinite(v3) && v3 > m3) m3 = v3;
        }
        for (; i < end; i += 64) {
            const double v = (double)arr[i];
            if (isfinite(v) && v > m0) m0 = v;
        }
        m0 = m0 > m1 ? m0 : m1;
        m2 = m2 > m3 ? m2 : m3;
        m0 = m0 > m2 ? m0 : m2;
        if (m0 > w) w = m0;
    };
    scan(ew, e0, e1);
    scan(gw, g0, g1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v = __shfl_xor(w, o, 64);
        w = v > w ? v : w;
    }
    if (lane == 0) {
        const int64_t nec = e1 - e0, ngc = g1 - g0;
        int64_t n = 0;
        double pm = 0.0;
        if (nec > 0 && ngc > 0) {
            pm = 2.0 * dt * dn * w;
            const double n_exp = (double)nec * (double)ngc * pm;
            if (!(n_exp < (double)kNtcMaxCand)) {
                ctl->too_many = 1;
            } else {
                const double fl = floor(n_exp);
                const u32x4 r = draw(seed, (uint64_t)c, step, kNtcCount);
                n = (int64_t)fl + (uniform53(r.a, r.b) < n_exp - fl ? 1 : 0);
                if (n > 64) ctl->has_large = 1;
            }
        }
        count[c] = n;
        p_max[c] = pm;
    }
}

__device__ __forceinline__ long long wave_incl_scan64(long long v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long t = __shfl_up(v, o, 64);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan of the workgroup's thread values (fixed order), and the total.
__device__ __forceinline__ long long block_excl_scan64(long long v, long long* lds, long long* total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const long long inc = wave_incl_scan64(v);
    if (lane == 63) lds[wave] = inc;
    __syncthreads();
    long long before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kNtcThreads / 64; ++w) {
        if (w < wave) before += lds[w];
        tot += lds[w];
    }
    __syncthreads();
    *total = tot;
    return before + inc - v;
}

// Local exclusive prefixes of the counts within each block of kNtcScanBlock
// cells, and the block sums.
__global__ __launch_bounds__(kNtcThreads) void k_ntc_scan_local(const int64_t* count, int64_t n_cells,
                                                              int64_t* cand_off, long long* bsum) {
    __shared__ long long s[kNtcThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kNtcScanBlock + (int64_t)threadIdx.x * kNtcScanPer;
    long long v[kNtcScanPer], t = 0;
#pragma unroll
    for (int q = 0; q < kNtcScanPer; ++q) {
        v[q] = base + q < n_cells ? count[base + q] : 0;
        t += v[q];
    }
    long long tot;
    long long run = block_excl_scan64(t, s, &tot);
#pragma unroll
    for (int q = 0; q < kNtcScanPer; ++q) {
        if (base + q < n_cells) cand_off[base + q] = run;
        run += v[q];
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// One workgroup: exclusive scan of the block sums (in place), the total.
__global__ __launch_bounds__(kNtcThreads) void k_ntc_scan_top(long long* bsum, int64_t n_blocks, int64_t n_cells,
                                                            int64_t* cand_off, NtcCtl* ctl) {
    __shared__ long long s[kNtcThreads / 64];
    long long carry = 0;
    for (int64_t b0 = 0; b0 < n_blocks; b0 += kNtcThreads) {
        const int64_t b = b0 + threadIdx.x;
        const long long v = b < n_blocks ? bsum[b] : 0;
        long long tot;
        const long long ex = block_excl_scan64(v, s, &tot);
        if (b < n_blocks) bsum[b] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) {
        cand_off[n_cells] = carry;
        ctl->total = carry;
        if (carry >= kNtcMaxCand) ctl->too_many = 1;
    }
}

// One wave per cell: the cell's candidates, 64 at a time.  A cell of at most
// 64 candidates is settled in the wave: a candidate that shares no particle
// with an earlier one of its cell is ready, and is evaluated here (the
// accepted ones listed in the workgroup's segment for the dense collide);
// the others register for round 1.  Larger cells register every candidate
// for round 0.
template <typename T>
__device__ __forceinline__ bool ntc_evaluate(const NtcArgs<T>& a, int64_t j, int32_t c, int32_t ie, int32_t ig);

template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_pick(const NtcArgs<T> a) {
    __shared__ int s_cnt[kNtcThreads / 64];
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * (kNtcThreads / 64) + wave;
    bool acc = false;
    int64_t j_acc = 0;
    if (c < a.n_cells) {
        // cand_off holds prefixes within each scan block: add the block offsets,
        // and keep the full offsets for the serial pass
        const int64_t j0 = a.cand_off[c] + a.boff[c / kNtcScanBlock];
        const int64_t j1 = c + 1 < a.n_cells ? a.cand_off[c + 1] + a.boff[(c + 1) / kNtcScanBlock] : a.total;
        if (lane == 0) {
            a.cand_full[c] = j0;
            if (c + 1 == a.n_cells) a.cand_full[c + 1] = j1;
        }
        const int64_t e0 = a.off_e[c], g0 = a.off_g[c];
        const uint64_t nec = (uint64_t)(a.off_e[c + 1] - e0), ngc = (uint64_t)(a.off_g[c + 1] - g0);
        const bool small = j1 - j0 <= 64;
        for (int64_t jb = j0; jb < j1; jb += 64) {
            const int64_t j = jb + lane;
            const bool act = j < j1;
            int32_t ie = -1, ig = -1;
            if (act) {
                const u32x4 r = draw(a.seed, ((uint64_t)c << 32) | (uint64_t)(j - j0), a.step, kNtcPick);
                ie = (int32_t)(e0 + (int64_t)(((uint64_t)r.a * nec) >> 32));
                ig = (int32_t)(g0 + (int64_t)(((uint64_t)r.b * ngc) >> 32));
                a.c_local[j] = (int32_t)(j - j0);
                a.c_u[j] = uniform53(r.c, r.d);
                a.c_ie[j] = ie;
                a.c_ig[j] = ig;
                a.c_cell[j] = (int32_t)c;
                a.status[j] = 0;
            }
            if (small) {
                const int n = (int)(j1 - j0);
                bool conflict = false;
                for (int m = 0; m < n; ++m) {
                    const int32_t ie_m = __shfl(ie, m, 64), ig_m = __shfl(ig, m, 64);
                    conflict = conflict || (m < lane && (ie_m == ie || ig_m == ig));
                }
                if (act && !conflict) {
                    acc = ntc_evaluate<T>(a, j, (int32_t)c, ie, ig);
                    j_acc = j;
                } else if (act) {
                    const unsigned long long tag = ntc_tag(a.epoch + 1u, j);
                    atomicMax(a.touch_e + a.cap_e + ie, tag);
                    atomicMax(a.touch_g + a.cap_g + ig, tag);
                }
            } else if (act) {
                const unsigned long long tag = ntc_tag(a.epoch, j);
                atomicMax(a.touch_e + ie, tag);
                atomicMax(a.touch_g + ig, tag);
            }
        }
    }
    // the workgroup's accepted candidates (small cells: at most one per lane)
    const unsigned long long m = __ballot(acc);
    if (lane == 0) s_cnt[wave] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kNtcThreads / 64; ++w) {
        before += w < wave ? s_cnt[w] : 0;
        tot += s_cnt[w];
    }
    if (acc) a.pick_list[(int64_t)blockIdx.x * kNtcThreads + before + __popcll(m & ((1ull << lane) - 1))] = (int32_t)j_acc;
    if (threadIdx.x == 0) a.pick_cnt[blockIdx.x] = tot;
}

// The probability of candidate j (cell c, particles ie, ig) on the current
// momenta and its accept/reject decision; writes its status and P / P_max
// and returns whether it collides (the collision itself: ntc_collide).
template <typename T>
__device__ __forceinline__ bool ntc_evaluate(const NtcArgs<T>& a, int64_t j, int32_t c, int32_t ie, int32_t ig) {
    const double u_c = a.c_u[j];
    const d3 p = load_p(a.pt, ie), k = load_k(a.pt, ig);
    const double we = (double)a.pt.ew[ie], wg = (double)a.pt.gw[ig];
    uint8_t st = 1;
    double ratio = -1.0;
    if (!finite_pair(p, we, k, wg)) {
        st |= 4;
    } else {
        const XFlux xf = x_flux(p, k, dot(p, p), dot(k, k));
        const double wmax = we > wg ? we : wg;
        const double P = xf.x > 0.0 ? a.dt * a.dn * wmax * sigma_ratio(xf.x) * xf.flux : 0.0;
        ratio = P / a.p_max[c];
        if (ratio > 1.0) st |= 8;
        if (u_c < ratio) st |= 2;
    }
    a.r_ratio[j] = ratio;
    a.status[j] = st;
    return (st & 2) != 0;
}

// Resolve the accepted candidate j: scattering angle from the plain
// sampler, both momenta updated under the weight rule.
template <typename T>
__device__ __forceinline__ void ntc_collide(const NtcArgs<T>& a, int64_t j, int32_t c, int32_t ie, int32_t ig) {
    const uint64_t idx = ((uint64_t)c << 32) | (uint64_t)a.c_local[j];
    const d3 p = load_p(a.pt, ie), k = load_k(a.pt, ig);
    const double we = (double)a.pt.ew[ie], wg = (double)a.pt.gw[ig];
    const PairInv inv = pair_invariants(p, k);
    const u32x4 s = draw(a.seed, idx, a.step, kNtcScatter);
    const double v = angle_icdf_v(uniform53(s.a, s.b), inv.x);
    const Scattered sc = scatter(p, k, inv, v, uniform53(s.c, s.d));
    bool upd_e = true, upd_g = true;
    if (we != wg) {
        const u32x4 q = draw(a.seed, idx, a.step, kNtcWeight);
        const double wmin = we < wg ? we : wg, wmax = we < wg ? wg : we;
        const bool heavier_moves = uniform53(q.a, q.b) < wmin / wmax;
        if (we > wg)
            upd_e = heavier_moves;
        else
            upd_g = heavier_moves;
    }
    if (upd_e) {
        a.pt.ex[ie] = (T)sc.p1.x;
        a.pt.ey[ie] = (T)sc.p1.y;
        a.pt.ez[ie] = (T)sc.p1.z;
    }
    if (upd_g) {
        a.pt.gx[ig] = (T)sc.k1.x;
        a.pt.gy[ig] = (T)sc.k1.y;
        a.pt.gz[ig] = (T)sc.k1.z;
    }
    a.r_eb[j] = sc.e_before;
    a.r_ea[j] = sc.e_after;
}

// Round t: ready candidates (earliest unresolved toucher of both their
// particles) are evaluated, and the accepted ones listed in the workgroup's
// segment for k_ntc_collide_list (round 0) or collide in place (later
// rounds); the others register for round t + 1, or
// after the last round mark their cell.
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_round(const NtcArgs<T> a, int t) {
    __shared__ int s_cnt[kNtcThreads / 64];
    const int64_t j = (int64_t)blockIdx.x * kNtcThreads + threadIdx.x;
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    bool acc = false;
    const uint8_t st = j < a.total ? a.status[j] : (uint8_t)1;
    if (!(st & 1)) {
        const int32_t ie = a.c_ie[j], ig = a.c_ig[j];
        const unsigned long long* te = a.touch_e + (t & 1) * a.cap_e;
        const unsigned long long* tg = a.touch_g + (t & 1) * a.cap_g;
        const unsigned long long mine = ntc_tag(a.epoch + (uint32_t)t, j);
        if (te[ie] == mine && tg[ig] == mine) {
            acc = ntc_evaluate<T>(a, j, a.c_cell[j], ie, ig);
            // after round 0 few candidates are left: they collide here
            if (t > 0 && acc) {
                ntc_collide<T>(a, j, a.c_cell[j], ie, ig);
                acc = false;
            }
        } else if (t + 1 < kNtcRounds) {
            const unsigned long long next = ntc_tag(a.epoch + (uint32_t)(t + 1), j);
            atomicMax(a.touch_e + ((t + 1) & 1) * a.cap_e + ie, next);
            atomicMax(a.touch_g + ((t + 1) & 1) * a.cap_g + ig, next);
        } else {
            a.pending[a.c_cell[j]] = 1;
        }
    }
    if (t != 0) return;  // (uniform) only round 0 lists its accepted candidates
    const unsigned long long m = __ballot(acc);
    if (lane == 0) s_cnt[wave] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kNtcThreads / 64; ++w) {
        before += w < wave ? s_cnt[w] : 0;
        tot += s_cnt[w];
    }
    int32_t* seg = a.list + (int64_t)blockIdx.x * kNtcThreads;
    if (acc) seg[before + __popcll(m & ((1ull << lane) - 1))] = (int32_t)j;
    if (threadIdx.x == 0) a.seg_cnt[blockIdx.x] = tot;
}

// Accepted candidates listed in segments of 256 (one per listing
// workgroup): workgroup b collides segment b, one entry per lane.
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_collide_list(const NtcArgs<T> a, const int32_t* list,
                                                                const int32_t* cnt) {
    const int n = cnt[blockIdx.x];
    if ((int)threadIdx.x >= n) return;
    const int64_t j = list[(int64_t)blockIdx.x * kNtcThreads + threadIdx.x];
    ntc_collide<T>(a, j, a.c_cell[j], a.c_ie[j], a.c_ig[j]);
}

// One wave per marked cell: the wave reads the statuses of 64 candidates at
// a time and lane 0 resolves the unresolved ones among them in order.
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_serial(const NtcArgs<T> a) {
    const int64_t c = (int64_t)blockIdx.x * (kNtcThreads / 64) + (threadIdx.x >> 6);
    if (c >= a.n_cells || !a.pending[c]) return;  // (uniform in the wave)
    const int lane = lane_id();
    const int64_t j0 = a.cand_full[c], j1 = a.cand_full[c + 1];
    for (int64_t jb = j0; jb < j1; jb += 64) {
        const int64_t j = jb + lane;
        unsigned long long m = __ballot(j < j1 && !(a.status[j] & 1));
        if (lane == 0) {
            while (m) {
                const int64_t q = jb + (__ffsll((long long)m) - 1);
                m &= m - 1;
                if (ntc_evaluate<T>(a, q, (int32_t)c, a.c_ie[q], a.c_ig[q]))
                    ntc_collide<T>(a, q, (int32_t)c, a.c_ie[q], a.c_ig[q]);
            }
        }
    }
    if (lane == 0) a.pending[c] = 0;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum a workgroup's per-thread partials in a fixed order (butterfly in each
// wave, then the waves in order); thread 0 gets the result.
__device__ __forceinline__ NtcPart block_sum_part(NtcPart v, NtcPart* lds) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    v.prob = wave_sum_d(v.prob);
    v.eb = wave_sum_d(v.eb);
    v.ea = wave_sum_d(v.ea);
    v.coll = wave_sum_ll(v.coll);
    v.inv = wave_sum_ll(v.inv);
    v.clip = wave_sum_ll(v.clip);
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    NtcPart r = {0.0, 0.0, 0.0, 0, 0, 0};
    if (threadIdx.x == 0)
        for (int w = 0; w < kNtcThreads / 64; ++w) {
            r.prob += lds[w].prob;
            r.eb += lds[w].eb;
            r.ea += lds[w].ea;
            r.coll += lds[w].coll;
            r.inv += lds[w].inv;
            r.clip += lds[w].clip;
        }
    return r;
}

__global__ __launch_bounds__(kNtcThreads) void k_ntc_reduce(const uint8_t* status, const double* ratio,
                                                          const double* eb, const double* ea, int64_t total,
                                                          NtcPart* part) {
    __shared__ NtcPart s[kNtcThreads / 64];
    NtcPart v = {0.0, 0.0, 0.0, 0, 0, 0};
    const int64_t base = (int64_t)blockIdx.x * kNtcThreads * kNtcRedPer + threadIdx.x;
    for (int q = 0; q < kNtcRedPer; ++q) {
        const int64_t j = base + (int64_t)q * kNtcThreads;
        if (j >= total) break;
        const uint8_t st = status[j];
        if (st & 4) {
            v.inv += 1;
            continue;
        }
        v.prob += ratio[j];
        v.clip += (st & 8) ? 1 : 0;
        if (st & 2) {
            v.coll += 1;
            v.eb += eb[j];
            v.ea += ea[j];
        }
    }
    const NtcPart r = block_sum_part(v, s);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ __launch_bounds__(kNtcThreads) void k_ntc_final(const NtcPart* part, int64_t n_part, int64_t total,
                                                         cs_stats* stats, NtcCtl* ctl) {
    __shared__ NtcPart s[kNtcThreads / 64];
    NtcPart v = {0.0, 0.0, 0.0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < n_part; b += kNtcThreads) {
        const NtcPart p = part[b];
        v.prob += p.prob;
        v.eb += p.eb;
        v.ea += p.ea;
        v.coll += p.coll;
        v.inv += p.inv;
        v.clip += p.clip;
    }
    const NtcPart r = block_sum_part(v, s);
    if (threadIdx.x == 0) {
        NtcCtl z = {};
        *ctl = z;
    }
    if (threadIdx.x == 0 && stats) {
        cs_stats o = {};
        o.n_pairs = total;
        o.n_collided = r.coll;
        o.n_clipped = r.clip;
        o.n_invalid = r.inv;
        o.sum_prob = r.prob;
        o.energy_before = r.eb;
        o.energy_after = r.ea;
        *stats = o;
    }
}

__global__ void k_ntc_stats_layout(cs_stats* stats) {
    cs_stats o = {};
    o.layout_error = 1;
    *stats = o;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

static hipError_t grow(void** buf, size_t* bytes, size_t want, hipStream_t st, bool* fresh = nullptr) {
    if (fresh) *fresh = false;
    if (*bytes >= want) return hipSuccess;
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    if (*buf) {
        e = hipFree(*buf);
        *buf = nullptr;
        *bytes = 0;
        if (e != hipSuccess) return e;
    }
    const size_t g = want + want / 4;
    e = hipMalloc(buf, g);
    if (e != hipSuccess) {
        *buf = nullptr;
        return e;
    }
    *bytes = g;
    if (fresh) *fresh = true;
    return hipSuccess;
}

void ntc_free(NtcState& s) {
    if (s.cell_ws) (void)hipFree(s.cell_ws);
    if (s.cand_ws) (void)hipFree(s.cand_ws);
    if (s.touch) (void)hipFree(s.touch);
    if (s.host) (void)hipHostFree(s.host);
    s = NtcState{};
}

template <typename T>
static hipError_t ntc_launch(NtcState& s, const cs_species& e, const cs_species& g, const int64_t* off_e,
                             const int64_t* off_g, int64_t n_cells, double dt, double dn, uint64_t seed,
                             uint64_t step, cs_stats* stats, hipStream_t st, NtcOutcome* out) {
    *out = NtcOutcome::kOk;
    // per-cell area: counts, offsets, P_max, marks, block sums, control
    const int64_t nb = (n_cells + kNtcScanBlock - 1) / kNtcScanBlock;
    const size_t b_count = align256(8 * (size_t)(n_cells > 0 ? n_cells : 1));
    const size_t b_off = align256(8 * (size_t)(n_cells + 1));
    const size_t b_pmax = b_count;
    const size_t b_pend = align256((size_t)(n_cells > 0 ? n_cells : 1));
    const size_t b_bsum = align256(8 * (size_t)(nb > 0 ? nb : 1));
    const size_t b_ctl = align256(sizeof(NtcCtl));
    bool fresh = false;
    hipError_t err =
        grow(&s.cell_ws, &s.cell_bytes, b_count + 2 * b_off + b_pmax + b_pend + b_bsum + b_ctl, st, &fresh);
    if (err != hipSuccess) return err;
    if (fresh) {  // the control words start at zero
        err = hipMemsetAsync(s.cell_ws, 0, s.cell_bytes, st);
        if (err != hipSuccess) return err;
    }
    // the control words first: their place does not depend on the cell count
    char* cw = (char*)s.cell_ws;
    NtcCtl* ctl = (NtcCtl*)cw;
    int64_t* count = (int64_t*)(cw += b_ctl);
    int64_t* cand_off = (int64_t*)(cw += b_count);
    double* p_max = (double*)(cw += b_off);
    uint8_t* pending = (uint8_t*)(cw += b_pmax);
    long long* bsum = (long long*)(cw += b_pend);
    int64_t* cand_full = (int64_t*)(cw += b_bsum);
    if (!s.host) {
        err = hipHostMalloc(&s.host, sizeof(NtcCtl), hipHostMallocDefault);
        if (err != hipSuccess) {
            s.host = nullptr;
            return err;
        }
    }
    // touch words: two sets per species, zero when (re)allocated
    if (s.cap_e < e.n || s.cap_g < g.n || s.touch == nullptr) {
        err = hipStreamSynchronize(st);
        if (err != hipSuccess) return err;
        if (s.touch) (void)hipFree(s.touch);
        s.touch = nullptr;
        s.cap_e = e.n > s.cap_e ? e.n + e.n / 4 : s.cap_e;
        s.cap_g = g.n > s.cap_g ? g.n + g.n / 4 : s.cap_g;
        if (s.cap_e < 1) s.cap_e = 1;
        if (s.cap_g < 1) s.cap_g = 1;
        const size_t tb = 2 * 8 * (size_t)(s.cap_e + s.cap_g);
        err = hipMalloc(&s.touch, tb);
        if (err != hipSuccess) {
            s.touch = nullptr;
            s.cap_e = s.cap_g = 0;
            return err;
        }
        err = hipMemsetAsync(s.touch, 0, tb, st);
        if (err != hipSuccess) return err;
        s.epoch = 1;
    }
    if (s.epoch > 0xFFFFFFFFu - 2 * kNtcRounds) {  // tags would wrap: clear and restart
        err = hipMemsetAsync(s.touch, 0, 2 * 8 * (size_t)(s.cap_e + s.cap_g), st);
        if (err != hipSuccess) return err;
        s.epoch = 1;
    }
    if (n_cells > 0) {
        k_ntc_count<T><<<(unsigned)((n_cells + 3) / 4), kNtcThreads, 0, st>>>(
            (const T*)e.w, (const T*)g.w, off_e, off_g, n_cells, e.n, g.n, dt, dn, seed, step, count, p_max, pending, ctl);
        k_ntc_scan_local<<<(unsigned)nb, kNtcThreads, 0, st>>>(count, n_cells, cand_off, bsum);
    }
    k_ntc_scan_top<<<1, kNtcThreads, 0, st>>>(bsum, nb, n_cells, cand_off, ctl);
    err = hipGetLastError();
    if (err == hipSuccess) err = hipMemcpyAsync(s.host, ctl, sizeof(NtcCtl), hipMemcpyDeviceToHost, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    if (err != hipSuccess) return err;
    const NtcCtl h = *(const NtcCtl*)s.host;
    if (h.layout_bad || (n_cells == 0 && (e.n != 0 || g.n != 0))) {
        *out = NtcOutcome::kLayout;
        if (stats) k_ntc_stats_layout<<<1, 1, 0, st>>>(stats);
        err = hipGetLastError();
        return err == hipSuccess ? hipMemsetAsync(ctl, 0, sizeof(NtcCtl), st) : err;
    }
    if (h.too_many) {
        *out = NtcOutcome::kTooMany;
        return hipMemsetAsync(ctl, 0, sizeof(NtcCtl), st);
    }
    const int64_t total = h.total;
    // per-candidate area
    const int64_t n_part = (total + kNtcThreads * kNtcRedPer - 1) / (kNtcThreads * kNtcRedPer);
    const size_t tc = (size_t)(total > 0 ? total : 1);
    const size_t b_i32 = align256(4 * tc), b_u8 = align256(tc), b_d = align256(8 * tc);
    const size_t b_part = align256(sizeof(NtcPart) * (size_t)(n_part > 0 ? n_part : 1));
    const int64_t n_rb = (total + kNtcThreads - 1) / kNtcThreads;
    const int64_t list_len = (n_rb > 0 ? n_rb : 1) * kNtcThreads;
    const int64_t n_pb = (n_cells + kNtcThreads / 64 - 1) / (kNtcThreads / 64);  // pick workgroups
    const size_t b_list = align256(4 * (size_t)list_len);
    const size_t b_seg = align256(4 * (size_t)(n_rb > 0 ? n_rb : 1));
    const size_t b_plist = align256(4 * (size_t)(n_pb > 0 ? n_pb : 1) * kNtcThreads);
    const size_t b_pcnt = align256(4 * (size_t)(n_pb > 0 ? n_pb : 1));
    err = grow(&s.cand_ws, &s.cand_bytes, 4 * b_i32 + b_u8 + 4 * b_d + b_part + b_list + b_seg + b_plist + b_pcnt,
               st);
    if (err != hipSuccess) return err;
    NtcArgs<T> a;
    a.pt = {(T*)e.x, (T*)e.y, (T*)e.z, (T*)e.w, (T*)g.x, (T*)g.y, (T*)g.z, (T*)g.w};
    a.off_e = off_e;
    a.off_g = off_g;
    a.n_cells = n_cells;
    a.total = total;
    a.dt = dt;
    a.dn = dn;
    a.seed = seed;
    a.step = step;
    a.epoch = s.epoch;
    a.cand_off = cand_off;
    a.boff = bsum;
    a.cand_full = cand_full;
    a.p_max = p_max;
    char* q = (char*)s.cand_ws;
    a.c_ie = (int32_t*)q;
    a.c_ig = (int32_t*)(q += b_i32);
    a.c_cell = (int32_t*)(q += b_i32);
    a.c_local = (int32_t*)(q += b_i32);
    a.status = (uint8_t*)(q += b_i32);
    a.r_ratio = (double*)(q += b_u8);
    a.r_eb = (double*)(q += b_d);
    a.r_ea = (double*)(q += b_d);
    a.c_u = (double*)(q += b_d);
    NtcPart* part = (NtcPart*)(q += b_d);
    a.list = (int32_t*)(q += b_part);
    a.seg_cnt = (int32_t*)(q += b_list);
    a.pick_list = (int32_t*)(q += b_seg);
    a.pick_cnt = (int32_t*)(q += b_plist);
    a.list_len = list_len;
    a.n_round_blocks = n_rb;
    a.touch_e = (unsigned long long*)s.touch;
    a.touch_g = a.touch_e + 2 * s.cap_e;
    a.cap_e = s.cap_e;
    a.cap_g = s.cap_g;
    a.pending = pending;
    s.epoch += kNtcRounds;
    if (total > 0) {
        const unsigned grid = (unsigned)((total + kNtcThreads - 1) / kNtcThreads);
        k_ntc_pick<T><<<(unsigned)n_pb, kNtcThreads, 0, st>>>(a);
        k_ntc_collide_list<T><<<(unsigned)n_pb, kNtcThreads, 0, st>>>(a, a.pick_list, a.pick_cnt);
        // round 0 only for cells of more than 64 candidates (the others were
        // settled in the pick kernel and registered for round 1)
        if (h.has_large) {
            k_ntc_round<T><<<grid, kNtcThreads, 0, st>>>(a, 0);
            k_ntc_collide_list<T><<<grid, kNtcThreads, 0, st>>>(a, a.list, a.seg_cnt);
        }
        for (int t = 1; t < kNtcRounds; ++t) k_ntc_round<T><<<grid, kNtcThreads, 0, st>>>(a, t);
        k_ntc_serial<T><<<(unsigned)n_pb, kNtcThreads, 0, st>>>(a);
        k_ntc_reduce<<<(unsigned)n_part, kNtcThreads, 0, st>>>(a.status, a.r_ratio, a.r_eb, a.r_ea, total, part);
    }
    k_ntc_final<<<1, kNtcThreads, 0, st>>>(part, n_part, total, stats, ctl);
    return hipGetLastError();
}

hipError_t ntc_step(NtcState& s, cs_dtype dtype, const cs_species& e, const cs_species& g, const int64_t* off_e,
                    const int64_t* off_g, int64_t n_cells, double dt, double dn, uint64_t seed, uint64_t step,
                    cs_stats* stats, hipStream_t st, NtcOutcome* out) {
    if (dtype == CS_F64) return ntc_launch<double>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, step, stats, st, out);
    return ntc_launch<float>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, step, stats, st, out);
}

}  // namespace cs
