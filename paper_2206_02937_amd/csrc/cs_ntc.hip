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
//                  block offsets added by k_ntc_pick) and the total, which
//                  stays on the device: the per-candidate launches are
//                  sized for a capacity fixed before the step (the context's
//                  grown capacity, or a graph's) and their workgroups past
//                  the total return at once; a step whose total exceeds the
//                  capacity changes nothing and flags its stats record
//   k_ntc_pick     one wave per cell: its candidates' electrons, photons
//                  and acceptance uniforms.  In a cell of at most 64
//                  candidates, those that share no particle with an earlier
//                  one are ready; the others register for round 1 in the
//                  particles' "first toucher" words (atomicMax of (round
//                  tag << 32 | ~candidate): each word ends up holding the
//                  earliest candidate that touches the particle).  Every
//                  candidate of a larger cell registers for round 0.
//   k_ntc_eval     round 0, one lane per candidate, one workgroup per
//                  segment of 1024 candidates (so the FP64 evaluation runs
//                  on full waves, not on a cell's few dozen lanes): ready
//                  candidates (a large cell's when it is the earliest
//                  registered toucher of both its particles) are evaluated
//                  (probability, accept); the accepted ones are compacted
//                  into the segment's collide list, the deferred ones (the
//                  large cells' others register for round 1 here) into its
//                  round-1 list
//   k_ntc_collide_list  round 0's accepted candidates, one per lane:
//                  scattering and write-back
//   k_ntc_round t  rounds 1 and 2 over the segments' lists: ready
//                  candidates are evaluated and, when accepted, collide in
//                  place (few are left); the others register for round 2 in
//                  the other word set (two sets alternate, so a round never
//                  reads a word that the same round writes) and go to the
//                  segment's round-2 list or, after round 2, mark their cell
//   k_ntc_serial   one wave per marked cell; its lane 0 resolves the
//                  cell's remaining candidates in order (long chains: a
//                  cell with one electron and many candidates)
//   k_ntc_reduce / k_ntc_final  fixed-order sums into cs_stats
// Compaction stays inside a workgroup (a prefix over its waves' ballots):
// no counter is shared between workgroups, and waves past a segment's list
// length return at once, so the waves that work are nearly full.
// Tags grow by one per round and never repeat (an epoch kept on the device
// beside the touch words and advanced by the last kernel of each step), so
// the touch words are cleared only when the epoch would wrap.  No kernel
// depends on a value read back by the host, so a step can be captured in a
// HIP graph; the step index then comes from a device word that each replay
// advances.
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
constexpr int kNtcRounds = 3;  // round 0 (k_ntc_eval), rounds 1 and 2 (k_ntc_round)
constexpr int kNtcScanPer = 4;                              // cells per thread in the scan
constexpr int kNtcScanBlock = kNtcThreads * kNtcScanPer;   // cells per scan workgroup
constexpr int kNtcRedPer = 2;                               // candidates per thread in the reduction
constexpr int64_t kNtcMaxCand = 2147483647;                 // candidates per step: below 2^31 - 1

// Control words of a step: the candidate total and flags.  Zero at the
// start of every step: zeroed when allocated and by k_ntc_final at the end
// of the previous step (they sit at the start of the per-cell scratch,
// whatever the cell count).
struct NtcCtl {
    long long total;
    int32_t layout_bad;
    int32_t too_many;   // 2^31 - 1 or more candidates
    int32_t overflow;   // more candidates than the launches were sized for
    int32_t go;         // none of the above: the step proceeds
    int32_t pad;
};
// Status bits before a candidate is resolved (bit 0 clear): registered for
// round 0 (a candidate of a cell with more than 64), or for round 1 (a
// small cell's candidate that shares a particle with an earlier one).
constexpr uint8_t kNtcLarge = 16;
constexpr uint8_t kNtcLater = 32;
// Candidates per segment: the evaluation kernel takes one segment per
// workgroup and compacts the segment's accepted candidates and the ones left
// for round 1 into the segment's part of two lists (no global counters).
constexpr int kNtcSeg = 1024;
constexpr int kNtcSub = kNtcSeg / kNtcThreads;  // collide and round workgroups per segment

// Persistent words at the start of the touch-word allocation (zeroed with
// the words): the tag epoch and the step index of graph replays.
struct NtcHead {
    uint32_t epoch;
    uint32_t pad;
    uint64_t step;
};
constexpr size_t kNtcHeadBytes = 256;

struct NtcPart {
    double prob, eb, ea;
    long long coll, inv, clip;
};

template <typename T>
struct NtcArgs {
    Particles<T> pt;
    const int64_t *off_e, *off_g;
    int64_t n_cells;
    int64_t total;   // filled on the device by ntc_live
    double dt, dn;
    uint64_t seed, step;  // step: the host's, or the device word's (dev_step)
    uint32_t epoch;       // filled on the device by ntc_live
    int32_t dev_step;
    const NtcCtl* ctl;
    const NtcHead* head;
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
    // per segment of kNtcSeg candidates: round 0's accepted candidates and
    // round 1's list (kNtcSeg entries each) with their lengths; round 2's
    // list in chunks of kNtcThreads (kNtcSub per segment) with theirs
    int32_t *lst_c, *lst_1, *lst_2;
    int32_t *cnt_c, *cnt_1, *cnt_2;
    int64_t n_seg;  // segments of the capacity
    int64_t cap;    // candidates the arrays hold
};

// The kernels below issue every read that does not depend on another one
// (the control words, the live values, their own inputs -- speculatively,
// clamped into the arrays) before they wait for any, and only then test
// whether the step proceeds: each read chain costs a memory round trip, and
// the waves of a launch run in few generations, so the round trips, not the
// arithmetic, set the kernels' length.

// The step's values that live on the device: the candidate total, the tag
// epoch and (graph replays) the step index.
template <typename T>
__device__ __forceinline__ NtcArgs<T> ntc_live(const NtcArgs<T>& in) {
    NtcArgs<T> a = in;
    a.total = in.ctl->total;
    a.epoch = in.head->epoch;
    if (in.dev_step) a.step = in.head->step;
    return a;
}

__device__ __forceinline__ unsigned long long ntc_tag(uint32_t round_tag, int64_t j) {
    return ((unsigned long long)round_tag << 32) | (unsigned long long)(0xFFFFFFFFu - (uint32_t)j);
}

template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_count(const T* ew, const T* gw, const int64_t* off_e,
                                                         const int64_t* off_g, int64_t n_cells, int64_t ne,
                                                         int64_t ng, double dt, double dn, uint64_t seed,
                                                         uint64_t step_host, const NtcHead* head, int dev_step,
                                                         int64_t* count, double* p_max, uint8_t* pending,
                                                         NtcCtl* ctl) {
    const int lane = lane_id();
    const int64_t c = (int64_t)blockIdx.x * (kNtcThreads / 64) + (threadIdx.x >> 6);
    if (c >= n_cells) return;
    const uint64_t step = dev_step ? head->step : step_host;
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

// One workgroup: exclusive scan of the block sums (in place), the total, and
// whether the step proceeds (a valid layout, fewer than 2^31 - 1
// candidates, at most `cap` of them).  When the tag epoch is about to wrap,
// the touch words are cleared and the epoch restarts at 0.
__global__ __launch_bounds__(kNtcThreads) void k_ntc_scan_top(long long* bsum, int64_t n_blocks, int64_t n_cells,
                                                            int64_t* cand_off, int64_t cap, NtcCtl* ctl,
                                                            NtcHead* head, unsigned long long* touch,
                                                            int64_t n_touch) {
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
    const bool wrap = head->epoch > 0xFFFFFFFFu - 2 * kNtcRounds;  // (uniform)
    if (wrap) {
        for (int64_t i = threadIdx.x; i < n_touch; i += kNtcThreads) touch[i] = 0ull;
        __syncthreads();  // every thread has read the epoch
    }
    if (threadIdx.x == 0) {
        if (wrap) head->epoch = 0;
        cand_off[n_cells] = carry;
        ctl->total = carry;
        int32_t too_many = ctl->too_many;
        if (carry >= kNtcMaxCand) too_many = 1;
        const int32_t overflow = carry > cap ? 1 : 0;
        ctl->too_many = too_many;
        ctl->overflow = overflow;
        ctl->go = (ctl->layout_bad | too_many | overflow) ? 0 : 1;
    }
}

// Compaction inside a workgroup of THREADS threads: the position of this
// thread among those with `take` set (in thread order) and their number.
template <int THREADS>
__device__ __forceinline__ int compact_slot(bool take, int* lds, int* total) {
    const int lane = lane_id(), wave = threadIdx.x >> 6;
    const unsigned long long m = __ballot(take);
    if (lane == 0) lds[wave] = __popcll(m);
    __syncthreads();
    int before = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < THREADS / 64; ++w) {
        before += w < wave ? lds[w] : 0;
        tot += lds[w];
    }
    *total = tot;
    return before + __popcll(m & ((1ull << lane) - 1));
}
__device__ __forceinline__ int seg_slot(bool take, int* lds, int* total) { return compact_slot<kNtcSeg>(take, lds, total); }
__device__ __forceinline__ int block_slot(bool take, int* lds, int* total) {
    return compact_slot<kNtcThreads>(take, lds, total);
}

// One wave per cell: the cell's candidates, 64 at a time: their electrons,
// photons and acceptance uniforms.  In a cell of at most 64 candidates, a
// candidate that shares no particle with an earlier one of its cell is
// ready (status 0); the others register for round 1 (kNtcLater).  Every
// candidate of a larger cell registers for round 0 (kNtcLarge).
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_pick(const NtcArgs<T> a_in) {
    const int lane = lane_id();
    const int64_t c = (int64_t)blockIdx.x * (kNtcThreads / 64) + (threadIdx.x >> 6);
    if (c >= a_in.n_cells) return;  // (uniform in the wave)
    const int32_t go = a_in.ctl->go;
    const NtcArgs<T> a = ntc_live(a_in);
    const bool last = c + 1 == a.n_cells;
    // cand_off holds prefixes within each scan block: add the block offsets,
    // and keep the full offsets for the serial pass
    const int64_t co0 = a.cand_off[c], bo0 = a.boff[c / kNtcScanBlock];
    const int64_t co1 = last ? 0 : a.cand_off[c + 1], bo1 = last ? 0 : a.boff[(c + 1) / kNtcScanBlock];
    const int64_t e0 = a.off_e[c], e1 = a.off_e[c + 1], g0 = a.off_g[c], g1 = a.off_g[c + 1];
    if (!go) return;  // (uniform) the step does not proceed
    const int64_t j0 = co0 + bo0;
    const int64_t j1 = last ? a.total : co1 + bo1;
    if (lane == 0) {
        a.cand_full[c] = j0;
        if (last) a.cand_full[c + 1] = j1;
    }
    const uint64_t nec = (uint64_t)(e1 - e0), ngc = (uint64_t)(g1 - g0);
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
        }
        if (small) {
            const int n = (int)(j1 - j0);
            bool conflict = false;
            for (int m = 0; m < n; ++m) {  // (m uniform: a lane read, not a permute)
                const int32_t ie_m = __builtin_amdgcn_readlane(ie, m), ig_m = __builtin_amdgcn_readlane(ig, m);
                conflict = conflict || (m < lane && (ie_m == ie || ig_m == ig));
            }
            if (act) a.status[j] = conflict ? kNtcLater : 0;
            if (act && conflict) {
                const unsigned long long tag = ntc_tag(a.epoch + 1u, j);
                atomicMax(a.touch_e + a.cap_e + ie, tag);
                atomicMax(a.touch_g + a.cap_g + ig, tag);
            }
        } else if (act) {
            a.status[j] = kNtcLarge;
            const unsigned long long tag = ntc_tag(a.epoch, j);
            atomicMax(a.touch_e + ie, tag);
            atomicMax(a.touch_g + ig, tag);
        }
    }
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

// Round 0, one workgroup per segment of kNtcSeg candidates, one lane per
// candidate: ready candidates (status 0, or a large cell's candidate that
// is the earliest registered toucher of both its particles) are evaluated,
// and the accepted ones compacted into the segment's collide list; the
// large cells' other candidates register for round 1, and they and the
// small cells' deferred ones are compacted into the segment's round-1 list.
template <typename T>
__global__ __launch_bounds__(kNtcSeg) void k_ntc_eval(const NtcArgs<T> a_in) {
    __shared__ int s_acc[kNtcSeg / 64], s_later[kNtcSeg / 64];
    const int64_t base = (int64_t)blockIdx.x * kNtcSeg;
    const int64_t j = base + threadIdx.x;
    const int64_t jc = j < a_in.cap ? j : a_in.cap - 1;
    const int32_t go = a_in.ctl->go;
    const NtcArgs<T> a = ntc_live(a_in);
    const uint8_t st = a.status[jc];
    const int32_t ie = a.c_ie[jc], ig = a.c_ig[jc], cell = a.c_cell[jc];
    if (!go || base >= a.total) return;  // (uniform) no step, or past the candidates
    bool acc = false, later = false;
    if (j < a.total) {
        bool ready = st == 0;
        if (st & kNtcLarge) {
            const unsigned long long mine = ntc_tag(a.epoch, j);
            ready = a.touch_e[ie] == mine && a.touch_g[ig] == mine;
            if (!ready) {
                const unsigned long long next = ntc_tag(a.epoch + 1u, j);
                atomicMax(a.touch_e + a.cap_e + ie, next);
                atomicMax(a.touch_g + a.cap_g + ig, next);
                later = true;
            }
        } else if (st & kNtcLater) {
            later = true;
        }
        if (ready) acc = ntc_evaluate<T>(a, j, cell, ie, ig);
    }
    int n_acc, n_later;
    const int pa = seg_slot(acc, s_acc, &n_acc);
    const int pl = seg_slot(later, s_later, &n_later);
    if (acc) a.lst_c[base + pa] = (int32_t)j;
    if (later) a.lst_1[base + pl] = (int32_t)j;
    if (threadIdx.x == 0) {
        a.cnt_c[blockIdx.x] = n_acc;
        a.cnt_1[blockIdx.x] = n_later;
    }
}

// Round 0's accepted candidates, one per lane (they share no particle, so
// their order does not matter).  Workgroups of kNtcThreads, kNtcSub per
// segment: a small workgroup whose waves have nothing to do frees its
// place at once, so the few waves that work spread over the chip.
// Workgroup b takes part b / n_seg of segment b % n_seg: the first parts
// (the ones most often busy, as lists fill from their start) are
// consecutive workgroups, which the dispatcher deals out over all XCDs.
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_collide_list(const NtcArgs<T> a_in) {
    const int64_t seg = blockIdx.x % a_in.n_seg;
    const int i = (int)(blockIdx.x / a_in.n_seg) * kNtcThreads + (int)threadIdx.x;
    const int32_t go = a_in.ctl->go;
    const NtcArgs<T> a = ntc_live(a_in);
    const int32_t n = a.cnt_c[seg];
    const int64_t j = a.lst_c[seg * kNtcSeg + i];  // (read whatever the count: i < kNtcSeg)
    if (!go || seg * kNtcSeg >= a.total || i >= n) return;
    ntc_collide<T>(a, j, a.c_cell[j], a.c_ie[j], a.c_ig[j]);
}

// Round t (1 or 2), one lane per list entry, workgroups of kNtcThreads:
// round 1 over the segments' round-1 lists (kNtcSub workgroups per
// segment, mapped as in k_ntc_collide_list), round 2 over the chunks of
// kNtcThreads entries that round 1 wrote.  A candidate that is the earliest registered toucher of both its
// particles is evaluated and, when accepted, collides in place (few
// candidates are left after round 0); in round 1 the others register for
// round 2 and are compacted into the workgroup's chunk of the round-2 list,
// in round 2 they mark their cell for the serial pass.
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_round(const NtcArgs<T> a_in, int t) {
    __shared__ int s_later[kNtcThreads / 64];
    const int64_t seg = blockIdx.x % a_in.n_seg;
    const int sub = (int)(blockIdx.x / a_in.n_seg) * kNtcThreads;
    const int64_t chunk = (int64_t)blockIdx.x * kNtcThreads;  // this workgroup's chunk of the lists
    const int32_t go = a_in.ctl->go;
    const NtcArgs<T> a = ntc_live(a_in);
    // entries of this workgroup: round 1, the part [sub, sub + kNtcThreads)
    // of the segment's list; round 2, its own chunk (read whatever the count)
    const int32_t cnt = t == 1 ? a.cnt_1[seg] : a.cnt_2[blockIdx.x];
    const int64_t j_l = t == 1 ? a.lst_1[seg * kNtcSeg + sub + threadIdx.x] : a.lst_2[chunk + threadIdx.x];
    if (!go || seg * kNtcSeg >= a.total) return;  // (uniform) no step, or past the candidates
    const int n = t == 1 ? min(cnt - sub, kNtcThreads) : cnt;
    if (n <= 0) {
        if (t == 1 && threadIdx.x == 0) a.cnt_2[blockIdx.x] = 0;
        return;  // (uniform)
    }
    bool later = false;
    int64_t j = 0;
    if ((int)threadIdx.x < n) {
        j = j_l;
        const int32_t ie = a.c_ie[j], ig = a.c_ig[j], c = a.c_cell[j];
        const unsigned long long* te = a.touch_e + (t & 1) * a.cap_e;
        const unsigned long long* tg = a.touch_g + (t & 1) * a.cap_g;
        const unsigned long long mine = ntc_tag(a.epoch + (uint32_t)t, j);
        if (te[ie] == mine && tg[ig] == mine) {
            if (ntc_evaluate<T>(a, j, c, ie, ig)) ntc_collide<T>(a, j, c, ie, ig);
        } else if (t + 1 < kNtcRounds) {
            const unsigned long long next = ntc_tag(a.epoch + (uint32_t)(t + 1), j);
            atomicMax(a.touch_e + ((t + 1) & 1) * a.cap_e + ie, next);
            atomicMax(a.touch_g + ((t + 1) & 1) * a.cap_g + ig, next);
            later = true;
        } else {
            a.pending[c] = 1;
        }
    }
    if (t + 1 < kNtcRounds) {  // (uniform: t == 1)
        int n_later;
        const int pl = block_slot(later, s_later, &n_later);
        if (later) a.lst_2[chunk + pl] = (int32_t)j;
        if (threadIdx.x == 0) a.cnt_2[blockIdx.x] = n_later;
    }
}

// One wave per marked cell: the wave reads the statuses of 64 candidates at
// a time and lane 0 resolves the unresolved ones among them in order.
template <typename T>
__global__ __launch_bounds__(kNtcThreads) void k_ntc_serial(const NtcArgs<T> a_in) {
    const int64_t c = (int64_t)blockIdx.x * (kNtcThreads / 64) + (threadIdx.x >> 6);
    if (c >= a_in.n_cells) return;  // (uniform in the wave)
    const int32_t go = a_in.ctl->go;
    const uint8_t pend = a_in.pending[c];
    if (!go || !pend) return;  // (uniform in the wave)
    const NtcArgs<T> a = ntc_live(a_in);
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
                                                          const double* eb, const double* ea, const NtcCtl* ctl,
                                                          int64_t cap, NtcPart* part) {
    __shared__ NtcPart s[kNtcThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kNtcThreads * kNtcRedPer + threadIdx.x;
    const int64_t total = ctl->total;
    const int32_t go = ctl->go;
    uint8_t st[kNtcRedPer];
    double rt[kNtcRedPer], b[kNtcRedPer], e[kNtcRedPer];
#pragma unroll
    for (int q = 0; q < kNtcRedPer; ++q) {  // (clamped into the arrays; used below the total only)
        const int64_t j = base + (int64_t)q * kNtcThreads;
        const int64_t jc = j < cap ? j : cap - 1;
        st[q] = status[jc];
        rt[q] = ratio[jc];
        b[q] = eb[jc];
        e[q] = ea[jc];
    }
    // (uniform) the step did not proceed, or a workgroup past the candidates
    if (!go || (int64_t)blockIdx.x * kNtcThreads * kNtcRedPer >= total) return;
    NtcPart v = {0.0, 0.0, 0.0, 0, 0, 0};
#pragma unroll
    for (int q = 0; q < kNtcRedPer; ++q) {
        const int64_t j = base + (int64_t)q * kNtcThreads;
        if (j >= total) break;
        if (st[q] & 4) {
            v.inv += 1;
            continue;
        }
        v.prob += rt[q];
        v.clip += (st[q] & 8) ? 1 : 0;
        if (st[q] & 2) {
            v.coll += 1;
            v.eb += b[q];
            v.ea += e[q];
        }
    }
    const NtcPart r = block_sum_part(v, s);
    if (threadIdx.x == 0) part[blockIdx.x] = r;
}

// The stats record from the reduction's partials, the control words
// cleared for the next step, the epoch and the step word advanced.
__global__ __launch_bounds__(kNtcThreads) void k_ntc_final(const NtcPart* part, cs_stats* stats, NtcCtl* ctl,
                                                         NtcHead* head) {
    __shared__ NtcPart s[kNtcThreads / 64];
    const NtcCtl c = *ctl;
    const int64_t total = c.total;
    const int64_t n_part = c.go ? (total + kNtcThreads * kNtcRedPer - 1) / (kNtcThreads * kNtcRedPer) : 0;
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
        head->epoch += kNtcRounds;
        head->step += 1;
    }
    if (threadIdx.x == 0 && stats) {
        cs_stats o = {};
        if (c.layout_bad) {
            o.layout_error = 1;
        } else if (!c.go) {  // too many candidates: nothing was changed
            o.n_pairs = c.too_many ? kNtcMaxCand : total;
            o.overflow = 1;
        } else {
            o.n_pairs = total;
            o.n_collided = r.coll;
            o.n_clipped = r.clip;
            o.n_invalid = r.inv;
            o.sum_prob = r.prob;
            o.energy_before = r.eb;
            o.energy_after = r.ea;
        }
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

// Device scratch of a step, laid out from sizes the host knows before the
// step: the cell count, the candidate capacity and the particle counts.
struct NtcLayout {
    int64_t nb, n_pb, n_seg, n_part;  // scan, pick, segment and reduction workgroups
    size_t b_count, b_off, b_pmax, b_pend, b_bsum, b_ctl, cell;
    size_t b_i32, b_u8, b_d, b_part, b_lst, b_cnt, cand;
};

static NtcLayout ntc_layout(int64_t n_cells, int64_t cap) {
    NtcLayout l;
    l.nb = (n_cells + kNtcScanBlock - 1) / kNtcScanBlock;
    l.n_pb = (n_cells + kNtcThreads / 64 - 1) / (kNtcThreads / 64);
    l.n_seg = (cap + kNtcSeg - 1) / kNtcSeg;
    l.n_part = (cap + kNtcThreads * kNtcRedPer - 1) / (kNtcThreads * kNtcRedPer);
    const size_t nc = (size_t)(n_cells > 0 ? n_cells : 1);
    l.b_count = align256(8 * nc);
    l.b_off = align256(8 * (nc + 1));
    l.b_pmax = l.b_count;
    l.b_pend = align256(nc);
    l.b_bsum = align256(8 * (size_t)(l.nb > 0 ? l.nb : 1));
    l.b_ctl = align256(sizeof(NtcCtl));
    l.cell = l.b_ctl + l.b_count + 2 * l.b_off + l.b_pmax + l.b_pend + l.b_bsum;
    const size_t tc = (size_t)(cap > 0 ? cap : 1);
    l.b_i32 = align256(4 * tc);
    l.b_u8 = align256(tc);
    l.b_d = align256(8 * tc);
    l.b_part = align256(sizeof(NtcPart) * (size_t)(l.n_part > 0 ? l.n_part : 1));
    l.b_lst = align256(4 * (size_t)(l.n_seg > 0 ? l.n_seg : 1) * kNtcSeg);
    l.b_cnt = align256(4 * (size_t)(l.n_seg > 0 ? l.n_seg : 1) * kNtcSub);
    l.cand = 4 * l.b_i32 + l.b_u8 + 4 * l.b_d + l.b_part + 3 * l.b_lst + 3 * l.b_cnt;
    return l;
}

static size_t touch_bytes(int64_t cap_e, int64_t cap_g) { return kNtcHeadBytes + 2 * 8 * (size_t)(cap_e + cap_g); }

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
    if (s.ev) (void)hipEventDestroy(s.ev);
    s = NtcState{};
}

// Scratch for a step of n_cells cells, `cap` candidates and ne / ng
// particles: the per-cell area (zeroed when fresh: its control words start
// at zero), the per-candidate area, and the touch words with their head
// (zeroed when (re)allocated).  Synchronises `st` when a buffer grows.
static hipError_t ntc_reserve(NtcState& s, int64_t n_cells, int64_t cap, int64_t ne, int64_t ng, hipStream_t st) {
    const NtcLayout l = ntc_layout(n_cells, cap);
    bool fresh = false;
    hipError_t err = grow(&s.cell_ws, &s.cell_bytes, l.cell, st, &fresh);
    if (err != hipSuccess) return err;
    if (fresh) {
        err = hipMemsetAsync(s.cell_ws, 0, s.cell_bytes, st);
        if (err != hipSuccess) return err;
    }
    if (cap > 0 || s.cand_ws == nullptr) {
        err = grow(&s.cand_ws, &s.cand_bytes, l.cand, st);
        if (err != hipSuccess) return err;
    }
    if (cap > s.cand_cap) s.cand_cap = cap;
    if (s.cap_e < ne || s.cap_g < ng || s.touch == nullptr) {
        err = hipStreamSynchronize(st);
        if (err != hipSuccess) return err;
        if (s.touch) (void)hipFree(s.touch);
        s.touch = nullptr;
        s.cap_e = ne > s.cap_e ? ne + ne / 4 : s.cap_e;
        s.cap_g = ng > s.cap_g ? ng + ng / 4 : s.cap_g;
        if (s.cap_e < 1) s.cap_e = 1;
        if (s.cap_g < 1) s.cap_g = 1;
        err = hipMalloc(&s.touch, touch_bytes(s.cap_e, s.cap_g));
        if (err != hipSuccess) {
            s.touch = nullptr;
            s.cap_e = s.cap_g = 0;
            return err;
        }
        err = hipMemsetAsync(s.touch, 0, touch_bytes(s.cap_e, s.cap_g), st);
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

// Queue one whole step for the candidate capacity s.cand_cap (no host
// synchronisation, no allocation, no memset: capturable).  With `host`
// set, the control words are copied there after the scan and `ev` is
// recorded behind the copy.
template <typename T>
static hipError_t ntc_enqueue(const NtcState& s, const cs_species& e, const cs_species& g, const int64_t* off_e,
                              const int64_t* off_g, int64_t n_cells, double dt, double dn, uint64_t seed,
                              uint64_t step, bool dev_step, cs_stats* stats, hipStream_t st, void* host,
                              hipEvent_t ev) {
    const int64_t cap = s.cand_cap;
    const NtcLayout l = ntc_layout(n_cells, cap);
    char* cw = (char*)s.cell_ws;
    NtcCtl* ctl = (NtcCtl*)cw;
    int64_t* count = (int64_t*)(cw += l.b_ctl);
    int64_t* cand_off = (int64_t*)(cw += l.b_count);
    double* p_max = (double*)(cw += l.b_off);
    uint8_t* pending = (uint8_t*)(cw += l.b_pmax);
    long long* bsum = (long long*)(cw += l.b_pend);
    int64_t* cand_full = (int64_t*)(cw += l.b_bsum);
    NtcHead* head = (NtcHead*)s.touch;
    unsigned long long* touch = (unsigned long long*)((char*)s.touch + kNtcHeadBytes);
    if (n_cells > 0) {
        k_ntc_count<T><<<(unsigned)((n_cells + 3) / 4), kNtcThreads, 0, st>>>(
            (const T*)e.w, (const T*)g.w, off_e, off_g, n_cells, e.n, g.n, dt, dn, seed, step, head, dev_step ? 1 : 0,
            count, p_max, pending, ctl);
        k_ntc_scan_local<<<(unsigned)l.nb, kNtcThreads, 0, st>>>(count, n_cells, cand_off, bsum);
    }
    k_ntc_scan_top<<<1, kNtcThreads, 0, st>>>(bsum, l.nb, n_cells, cand_off, cap, ctl, head, touch,
                                              2 * (s.cap_e + s.cap_g));
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    if (host) {
        err = hipMemcpyAsync(host, ctl, sizeof(NtcCtl), hipMemcpyDeviceToHost, st);
        if (err == hipSuccess) err = hipEventRecord(ev, st);
        if (err != hipSuccess) return err;
    }
    NtcArgs<T> a;
    a.pt = {(T*)e.x, (T*)e.y, (T*)e.z, (T*)e.w, (T*)g.x, (T*)g.y, (T*)g.z, (T*)g.w};
    a.off_e = off_e;
    a.off_g = off_g;
    a.n_cells = n_cells;
    a.total = 0;
    a.dt = dt;
    a.dn = dn;
    a.seed = seed;
    a.step = step;
    a.epoch = 0;
    a.dev_step = dev_step ? 1 : 0;
    a.ctl = ctl;
    a.head = head;
    a.cand_off = cand_off;
    a.boff = bsum;
    a.cand_full = cand_full;
    a.p_max = p_max;
    char* q = (char*)s.cand_ws;
    a.c_ie = (int32_t*)q;
    a.c_ig = (int32_t*)(q += l.b_i32);
    a.c_cell = (int32_t*)(q += l.b_i32);
    a.c_local = (int32_t*)(q += l.b_i32);
    a.status = (uint8_t*)(q += l.b_i32);
    a.r_ratio = (double*)(q += l.b_u8);
    a.r_eb = (double*)(q += l.b_d);
    a.r_ea = (double*)(q += l.b_d);
    a.c_u = (double*)(q += l.b_d);
    NtcPart* part = (NtcPart*)(q += l.b_d);
    a.lst_c = (int32_t*)(q += l.b_part);
    a.lst_1 = (int32_t*)(q += l.b_lst);
    a.lst_2 = (int32_t*)(q += l.b_lst);
    a.cnt_c = (int32_t*)(q += l.b_lst);
    a.cnt_1 = (int32_t*)(q += l.b_cnt);
    a.cnt_2 = (int32_t*)(q += l.b_cnt);
    a.n_seg = l.n_seg > 0 ? l.n_seg : 1;
    a.cap = cap > 0 ? cap : 1;
    a.touch_e = touch;
    a.touch_g = touch + 2 * s.cap_e;
    a.cap_e = s.cap_e;
    a.cap_g = s.cap_g;
    a.pending = pending;
    if (n_cells > 0) k_ntc_pick<T><<<(unsigned)l.n_pb, kNtcThreads, 0, st>>>(a);
    if (cap > 0) {
        // one workgroup per segment, up to the capacity; kNtcSub smaller ones per segment
        k_ntc_eval<T><<<(unsigned)l.n_seg, kNtcSeg, 0, st>>>(a);
        const unsigned grid = (unsigned)(l.n_seg * kNtcSub);
        k_ntc_collide_list<T><<<grid, kNtcThreads, 0, st>>>(a);
        for (int t = 1; t < kNtcRounds; ++t) k_ntc_round<T><<<grid, kNtcThreads, 0, st>>>(a, t);
    }
    if (n_cells > 0) k_ntc_serial<T><<<(unsigned)l.n_pb, kNtcThreads, 0, st>>>(a);
    if (cap > 0)
        k_ntc_reduce<<<(unsigned)l.n_part, kNtcThreads, 0, st>>>(a.status, a.r_ratio, a.r_eb, a.r_ea, ctl, a.cap,
                                                                 part);
    k_ntc_final<<<1, kNtcThreads, 0, st>>>(part, stats, ctl, head);
    return hipGetLastError();
}

template <typename T>
static hipError_t ntc_launch(NtcState& s, const cs_species& e, const cs_species& g, const int64_t* off_e,
                             const int64_t* off_g, int64_t n_cells, double dt, double dn, uint64_t seed,
                             uint64_t step, cs_stats* stats, hipStream_t st, NtcOutcome* out) {
    *out = NtcOutcome::kOk;
    if (n_cells == 0 && (e.n != 0 || g.n != 0)) {
        *out = NtcOutcome::kLayout;
        if (stats) k_ntc_stats_layout<<<1, 1, 0, st>>>(stats);
        return hipGetLastError();
    }
    hipError_t err = ntc_reserve(s, n_cells, s.cand_cap, e.n, g.n, st);
    if (err != hipSuccess) return err;
    if (!s.host) {
        err = hipHostMalloc(&s.host, sizeof(NtcCtl), hipHostMallocDefault);
        if (err != hipSuccess) {
            s.host = nullptr;
            return err;
        }
    }
    if (!s.ev) {
        err = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
        if (err != hipSuccess) {
            s.ev = nullptr;
            return err;
        }
    }
    // The whole step is queued at once; the host then waits only for the
    // scan's control words (the rest of the step runs meanwhile).  A step
    // with more candidates than the capacity changed nothing: the scratch
    // grows and the step is queued again (same inputs, same candidates).
    err = ntc_enqueue<T>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, step, false, stats, st, s.host, s.ev);
    if (err == hipSuccess) err = hipEventSynchronize(s.ev);
    if (err != hipSuccess) return err;
    const NtcCtl h = *(const NtcCtl*)s.host;
    if (h.layout_bad) {
        *out = NtcOutcome::kLayout;
        return hipSuccess;
    }
    if (h.too_many) {
        *out = NtcOutcome::kTooMany;
        return hipSuccess;
    }
    if (h.overflow) {
        err = ntc_reserve(s, n_cells, h.total + h.total / 4, e.n, g.n, st);
        if (err == hipSuccess)
            err = ntc_enqueue<T>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, step, false, stats, st, nullptr,
                                 nullptr);
    }
    return err;
}

hipError_t ntc_step(NtcState& s, cs_dtype dtype, const cs_species& e, const cs_species& g, const int64_t* off_e,
                    const int64_t* off_g, int64_t n_cells, double dt, double dn, uint64_t seed, uint64_t step,
                    cs_stats* stats, hipStream_t st, NtcOutcome* out) {
    if (dtype == CS_F64) return ntc_launch<double>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, step, stats, st, out);
    return ntc_launch<float>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, step, stats, st, out);
}

hipError_t ntc_prepare_graph(NtcState& s, int64_t n_cells, int64_t cap, int64_t ne, int64_t ng, hipStream_t st) {
    hipError_t err = ntc_reserve(s, n_cells, cap, ne, ng, st);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
    return err;
}

hipError_t ntc_capture(const NtcState& s, cs_dtype dtype, const cs_species& e, const cs_species& g,
                       const int64_t* off_e, const int64_t* off_g, int64_t n_cells, double dt, double dn,
                       uint64_t seed, cs_stats* stats, hipStream_t st) {
    if (dtype == CS_F64)
        return ntc_enqueue<double>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, 0, true, stats, st, nullptr, nullptr);
    return ntc_enqueue<float>(s, e, g, off_e, off_g, n_cells, dt, dn, seed, 0, true, stats, st, nullptr, nullptr);
}

__global__ void k_ntc_set_step(NtcHead* head, uint64_t step) {
    if (threadIdx.x == 0 && blockIdx.x == 0) head->step = step;
}

hipError_t ntc_set_step(const NtcState& s, uint64_t step, hipStream_t st) {
    k_ntc_set_step<<<1, 64, 0, st>>>((NtcHead*)s.touch, step);
    return hipGetLastError();
}

}  // namespace cs
