// cs_pair.h -- the per-pair work of a Compton step, shared by every kernel
// strategy (multi-kernel baseline and fused persistent kernel) so that all of
// them compute bitwise-identical results.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cs_device.h"
#include "cs_net.h"

namespace cs {

template <typename T>
struct Particles {
    T *ex, *ey, *ez, *ew;
    T *gx, *gy, *gz, *gw;
};

// The step's control words that every kernel after the scan reads at its
// start (epoch, step counter, layout and scan-fault epochs), all in one
// memory round trip: read one by one, with the layout test's short-circuit
// between two of them, they took several round trips in a row.
struct CtrlView {
    uint32_t epoch;
    uint64_t step;
    bool layout_ok;  // no layout error and no scan time-out in this step
};

__device__ __forceinline__ CtrlView ctrl_view(const StepControl* ctrl) {
    const uint32_t epoch = ctrl->epoch, layout_epoch = ctrl->layout_epoch, fault_epoch = ctrl->scan_fault_epoch;
    const uint64_t step = ctrl->step;
    CtrlView v;
    v.epoch = epoch;
    v.step = step;
    v.layout_ok = (layout_epoch != epoch) & (fault_epoch != epoch);
    return v;
}

struct PairOutcome {
    int32_t ie, ig;  // electron / photon index of the pair
    double x;        // rest-frame photon energy (0 when invalid)
    double P;        // collision probability (0 when invalid)
    bool accept;
    bool clipped;
    bool invalid;
};

__device__ __forceinline__ bool finite_pair(d3 p, double we, d3 k, double wg) {
    return isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(k.x) && isfinite(k.y) && isfinite(k.z) &&
           isfinite(we) && isfinite(wg) && we >= 0.0 && wg >= 0.0;
}

// The three phases of a pair's evaluation, split so that a kernel can issue
// the memory accesses of several pairs before it needs any of them:
//   pair_index   pairing (keyed in-cell bijection) -> electron/photon index
//   pair_load    the two particles' momenta and weights (storage type)
//   pair_physics rest-frame photon energy, Klein-Nishina cross-section,
//                probability, accept/reject
// pair_eval runs the three in a row.
struct PairSlot {
    int32_t ie, ig;  // particle indices (0 when inactive)
    uint32_t M;      // larger species count of the cell
    bool active;
};

template <typename T>
struct PairRaw {
    T p[3], k[3], we, wg;
};

// Pair number i of the cell with particle ranges [e0, e1), [g0, g1) and
// pairing key key4.
__device__ __forceinline__ PairSlot pair_index(bool active, int64_t e0, int64_t e1, int64_t g0, int64_t g1,
                                               uint32_t k0, uint32_t k1, uint32_t k2, uint32_t k3, uint32_t i) {
    PairSlot s;
    s.ie = 0;
    s.ig = 0;
    s.M = 0;
    s.active = active;
    if (active) {
        const uint32_t ne = (uint32_t)(e1 - e0), ng = (uint32_t)(g1 - g0);
        s.M = ne > ng ? ne : ng;
        FeistelKey key;
        key.k[0] = k0;
        key.k[1] = k1;
        key.k[2] = k2;
        key.k[3] = k3;
        key.bits = ceil_log2(s.M);
        if (ne <= ng) {
            s.ie = (int32_t)(e0 + i);
            s.ig = (int32_t)(g0 + shuffle_index(i, ng, key));
        } else {
            s.ig = (int32_t)(g0 + i);
            s.ie = (int32_t)(e0 + shuffle_index(i, ne, key));
        }
    }
    return s;
}

template <typename T>
__device__ __forceinline__ PairRaw<T> pair_load(const Particles<T>& a, const PairSlot& s) {
    PairRaw<T> r;
    if (s.active) {
        r.p[0] = a.ex[s.ie];
        r.p[1] = a.ey[s.ie];
        r.p[2] = a.ez[s.ie];
        r.k[0] = a.gx[s.ig];
        r.k[1] = a.gy[s.ig];
        r.k[2] = a.gz[s.ig];
        r.we = a.ew[s.ie];
        r.wg = a.gw[s.ig];
    } else {
        r.p[0] = r.p[1] = r.p[2] = r.k[0] = r.k[1] = r.k[2] = r.we = r.wg = (T)0;
    }
    return r;
}

// The reads of pair_load issued by every lane: inactive lanes read element 0
// (which exists whenever a pair does; pair_index leaves index 0 in inactive
// slots) and leave the values unused (the physics reads them only for active
// slots), so that the number of reads in flight does not depend on which
// lanes are active and no lane waits for them before they are used.  With
// O32 the byte offsets are formed as unsigned 32-bit values (one multiply
// instead of a 64-bit shift-add per array; the loads take the array base in
// scalar registers), valid while every species has at most 2^32 / sizeof(T)
// elements -- the caller checks that.
template <typename T, bool O32 = false>
__device__ __forceinline__ PairRaw<T> pair_load_all(const Particles<T>& a, const PairSlot& s) {
    PairRaw<T> r;
    if constexpr (O32) {
        const uint32_t oe = (uint32_t)s.ie * (uint32_t)sizeof(T), og = (uint32_t)s.ig * (uint32_t)sizeof(T);
        auto at = [](const T* b, uint32_t o) { return *(const T*)((const char*)b + (uint64_t)o); };
        r.p[0] = at(a.ex, oe);
        r.p[1] = at(a.ey, oe);
        r.p[2] = at(a.ez, oe);
        r.k[0] = at(a.gx, og);
        r.k[1] = at(a.gy, og);
        r.k[2] = at(a.gz, og);
        r.we = at(a.ew, oe);
        r.wg = at(a.gw, og);
    } else {
        r.p[0] = a.ex[s.ie];
        r.p[1] = a.ey[s.ie];
        r.p[2] = a.ez[s.ie];
        r.k[0] = a.gx[s.ig];
        r.k[1] = a.gy[s.ig];
        r.k[2] = a.gz[s.ig];
        r.we = a.ew[s.ie];
        r.wg = a.gw[s.ig];
    }
    return r;
}

// `sig_tab`: kSigTab or a copy of it (see sigma_ratio_tab).
template <typename T>
__device__ __forceinline__ PairOutcome pair_physics(const PairSlot& s, const PairRaw<T>& r, double dt,
                                                    double density_norm, uint64_t seed, uint64_t step,
                                                    const double* sig_tab = kSigTab) {
    PairOutcome o;
    o.ie = s.ie;
    o.ig = s.ig;
    o.x = 0.0;
    o.P = 0.0;
    o.accept = false;
    o.clipped = false;
    o.invalid = false;
    double x = 0.0, flux = 0.0, wmax = 0.0, tau = 0.0;
    bool compute = false;
    if (s.active) {
        const d3 p = {(double)r.p[0], (double)r.p[1], (double)r.p[2]};
        const d3 k = {(double)r.k[0], (double)r.k[1], (double)r.k[2]};
        const double we = (double)r.we, wg = (double)r.wg;
        if (!finite_pair(p, we, k, wg)) {
            o.invalid = true;
        } else {
            const XFlux xf = x_flux(p, k, dot(p, p), dot(k, k));
            x = xf.x;
            flux = xf.flux;
            tau = dt * density_norm * (double)s.M;
            wmax = we > wg ? we : wg;
            compute = x > 0.0;
        }
    }
    if (compute) {
        double P = tau * wmax * sigma_ratio_tab(x, sig_tab) * flux;
        if (P > 1.0) {
            o.clipped = true;
            P = 1.0;
        }
        o.P = P;
    }
    if (s.active && !o.invalid) {
        const u32x4 u = draw(seed, (uint64_t)o.ie, step, kCollide);
        o.accept = uniform53(u.a, u.b) < o.P;
    }
    o.x = x;
    return o;
}

template <typename T>
__device__ __forceinline__ PairOutcome pair_eval(const Particles<T>& a, bool active, int64_t e0, int64_t e1,
                                                 int64_t g0, int64_t g1, const uint32_t* key4, uint32_t i,
                                                 double dt, double density_norm, uint64_t seed, uint64_t step) {
    uint32_t k0 = 0, k1 = 0, k2 = 0, k3 = 0;
    if (active) {
        k0 = key4[0];
        k1 = key4[1];
        k2 = key4[2];
        k3 = key4[3];
    }
    const PairSlot s = pair_index(active, e0, e1, g0, g1, k0, k1, k2, k3, i);
    return pair_physics<T>(s, pair_load<T>(a, s), dt, density_norm, seed, step);
}

struct CollideSums {
    double e_before = 0.0, e_after = 0.0;
    long long n_fallback = 0;  // network samplers: samples the plain sampler answered
};

template <typename T>
__device__ __forceinline__ d3 load_p(const Particles<T>& a, int32_t i) {
    return {(double)a.ex[i], (double)a.ey[i], (double)a.ez[i]};
}
template <typename T>
__device__ __forceinline__ d3 load_k(const Particles<T>& a, int32_t i) {
    return {(double)a.gx[i], (double)a.gy[i], (double)a.gz[i]};
}

// Write back a resolved collision under the weight rule.
template <typename T>
__device__ __forceinline__ void write_back(const Particles<T>& a, int32_t ie, int32_t ig, double we, double wg,
                                           const Scattered& s, uint64_t seed, uint64_t step) {
    bool upd_e = true, upd_g = true;
    if (we != wg) {
        const u32x4 rc = draw(seed, (uint64_t)ie, step, kCollide);
        const double wmin = we < wg ? we : wg, wmx = we < wg ? wg : we;
        const bool heavier_moves = uniform53(rc.c, rc.d) < wmin / wmx;
        if (we > wg)
            upd_e = heavier_moves;
        else
            upd_g = heavier_moves;
    }
    if (upd_e) {
        a.ex[ie] = (T)s.p1.x;
        a.ey[ie] = (T)s.p1.y;
        a.ez[ie] = (T)s.p1.z;
    }
    if (upd_g) {
        a.gx[ig] = (T)s.k1.x;
        a.gy[ig] = (T)s.k1.y;
        a.gz[ig] = (T)s.k1.z;
    }
}

// Resolve the accepted pair (ie, ig) with particle values raw = (p, k, we, wg)
// in their storage type with the plain sampler and write it back.  Lanes
// with active == false run the sampler on a dummy x = 0 (the quickest case)
// and write nothing.
template <typename T>
__device__ __forceinline__ void collide_raw(const Particles<T>& a, bool active, int32_t ie, int32_t ig,
                                            const T (&raw)[8], uint64_t seed, uint64_t step, CollideSums& sums) {
    double x = 0.0;
    if (active) {
        const d3 p = {(double)raw[0], (double)raw[1], (double)raw[2]};
        const d3 k = {(double)raw[3], (double)raw[4], (double)raw[5]};
        x = x_flux(p, k, dot(p, p), dot(k, k)).x;
    }
    const u32x4 r = draw(seed, (uint64_t)ie, step, kScatter);
    const double v = angle_icdf_v(active ? uniform53(r.a, r.b) : 0.5, x);
    if (!active) return;
    const double u_phi = uniform53(r.c, r.d);
    const d3 p = {(double)raw[0], (double)raw[1], (double)raw[2]};
    const d3 k = {(double)raw[3], (double)raw[4], (double)raw[5]};
    const PairInv inv = pair_invariants(p, k);
    const Scattered s = scatter(p, k, inv, v, u_phi);
    write_back<T>(a, ie, ig, (double)raw[6], (double)raw[7], s, seed, step);
    sums.e_before += s.e_before;
    sums.e_after += s.e_after;
}

// The same with the particle values read from the arrays (once, before the
// sampler, kept in their storage type across it: 8 registers for FP32).
template <typename T>
__device__ __forceinline__ void collide_plain(const Particles<T>& a, bool active, int32_t ie, int32_t ig,
                                              uint64_t seed, uint64_t step, CollideSums& sums) {
    T raw[8] = {};
    if (active) {
        raw[0] = a.ex[ie];
        raw[1] = a.ey[ie];
        raw[2] = a.ez[ie];
        raw[3] = a.gx[ig];
        raw[4] = a.gy[ig];
        raw[5] = a.gz[ig];
        raw[6] = a.ew[ie];
        raw[7] = a.gw[ig];
    }
    collide_raw<T>(a, active, ie, ig, raw, seed, step, sums);
}

// An accepted pair kept in global memory between the pair and the collide
// kernels: its indices and the particle values the pair kernel read, in 16-
// byte units (3 for FP32, 5 for FP64), so that the collide kernel reads them
// in a few wide loads instead of gathering eight scattered elements.
template <typename T>
struct alignas(16) StashPair {
    T p[3], we;
    T k[3], wg;
    int32_t ie, ig, pad0, pad1;
};

template <typename T>
__device__ __forceinline__ StashPair<T> make_stash(const PairSlot& s, const PairRaw<T>& r) {
    StashPair<T> e;
    e.p[0] = r.p[0];
    e.p[1] = r.p[1];
    e.p[2] = r.p[2];
    e.we = r.we;
    e.k[0] = r.k[0];
    e.k[1] = r.k[1];
    e.k[2] = r.k[2];
    e.wg = r.wg;
    e.ie = s.ie;
    e.ig = s.ig;
    e.pad0 = 0;
    e.pad1 = 0;
    return e;
}

// collide_raw with the pair taken from a stash entry.
template <typename T>
__device__ __forceinline__ void collide_stash(const Particles<T>& a, bool active, const StashPair<T>* e,
                                              uint64_t seed, uint64_t step, CollideSums& sums) {
    T raw[8] = {};
    int32_t ie = 0, ig = 0;
    if (active) {
        const StashPair<T> v = *e;
        raw[0] = v.p[0];
        raw[1] = v.p[1];
        raw[2] = v.p[2];
        raw[3] = v.k[0];
        raw[4] = v.k[1];
        raw[5] = v.k[2];
        raw[6] = v.we;
        raw[7] = v.wg;
        ie = v.ie;
        ig = v.ig;
    }
    collide_raw<T>(a, active, ie, ig, raw, seed, step, sums);
}

// An accepted pair staged in LDS with its particle values.
template <typename T>
struct StagedPair {
    int32_t ie, ig;
    T p[3], k[3], we, wg;
};

// The same as collide_plain with the particle values taken from LDS.
template <typename T>
__device__ __forceinline__ void collide_staged(const Particles<T>& a, bool active, const StagedPair<T>* e,
                                               uint64_t seed, uint64_t step, CollideSums& sums) {
    double x = 0.0;
    int32_t ie = 0;
    if (active) {
        ie = e->ie;
        const d3 p = {(double)e->p[0], (double)e->p[1], (double)e->p[2]};
        const d3 k = {(double)e->k[0], (double)e->k[1], (double)e->k[2]};
        x = pair_invariants(p, k).x;
    }
    const u32x4 r = draw(seed, (uint64_t)ie, step, kScatter);
    const double v = angle_icdf_v(active ? uniform53(r.a, r.b) : 0.5, x);
    if (!active) return;
    const double u_phi = uniform53(r.c, r.d);
    const d3 p = {(double)e->p[0], (double)e->p[1], (double)e->p[2]};
    const d3 k = {(double)e->k[0], (double)e->k[1], (double)e->k[2]};
    const PairInv inv = pair_invariants(p, k);
    const Scattered s = scatter(p, k, inv, v, u_phi);
    write_back<T>(a, ie, e->ig, (double)e->we, (double)e->wg, s, seed, step);
    sums.e_before += s.e_before;
    sums.e_after += s.e_after;
}

// Where a collision's particle values come from: an LDS queue entry, a stash
// entry or the particle arrays.
template <typename T>
struct FromStaged {
    const StagedPair<T>* e;
    __device__ __forceinline__ void get(const Particles<T>&, int32_t& ie, int32_t& ig, d3& p, d3& k, double& we,
                                        double& wg) const {
        ie = e->ie;
        ig = e->ig;
        p = {(double)e->p[0], (double)e->p[1], (double)e->p[2]};
        k = {(double)e->k[0], (double)e->k[1], (double)e->k[2]};
        we = (double)e->we;
        wg = (double)e->wg;
    }
};
template <typename T>
struct FromStash {
    const StashPair<T>* e;
    __device__ __forceinline__ void get(const Particles<T>&, int32_t& ie, int32_t& ig, d3& p, d3& k, double& we,
                                        double& wg) const {
        const StashPair<T> v = *e;
        ie = v.ie;
        ig = v.ig;
        p = {(double)v.p[0], (double)v.p[1], (double)v.p[2]};
        k = {(double)v.k[0], (double)v.k[1], (double)v.k[2]};
        we = (double)v.we;
        wg = (double)v.wg;
    }
};
template <typename T>
struct FromArrays {
    int32_t ie, ig;
    __device__ __forceinline__ void get(const Particles<T>& a, int32_t& ie_, int32_t& ig_, d3& p, d3& k,
                                        double& we, double& wg) const {
        ie_ = ie;
        ig_ = ig;
        p = load_p(a, ie);
        k = load_k(a, ig);
        we = (double)a.ew[ie];
        wg = (double)a.gw[ig];
    }
};

// Resolve an accepted pair with the sampler network: the network maps the
// FP32-rounded (x, u) to (cos theta, eps'/eps), read as v = 1 - cos theta by
// net_reading_v; outside the network's x range the plain sampler answers
// (counted in n_fallback).  The
// same Philox draw as the plain sampler supplies u and the azimuth.  Must be
// called by the whole wave; lanes with active == false write nothing.
template <typename T, int SAMP, typename Src>
__device__ __forceinline__ void collide_net(const Particles<T>& a, bool active, const Src& src, NetLds<SAMP>& s_net,
                                            const MlpDev& m, uint64_t seed, uint64_t step, CollideSums& sums) {
    // Three phases, so that little is live while the network runs: (1) x and
    // the Philox draw from the pair's values, (2) the network for the wave,
    // (3) the pair's values fetched again (the same source: LDS, a stash entry
    // in cache, or the particle arrays) for the sampler's fallback and the
    // scatter.
    double x = 0.0;
    int32_t ie = 0, ig = 0;
    {
        d3 p = {0.0, 0.0, 0.0}, k = {0.0, 0.0, 0.0};
        double we = 0.0, wg = 0.0;
        if (active) {
            src.get(a, ie, ig, p, k, we, wg);
            x = pair_invariants(p, k).x;
        }
    }
    const u32x4 r = draw(seed, (uint64_t)ie, step, kScatter);
    const double u = uniform53(r.a, r.b);
    const float xf = (float)x, uf = (float)u;
    const bool inside = active && in_range(xf, m.dom);
    const bool fallback = active && !inside;
    float f1 = 0.0f, f2 = 0.0f;
    if (inside) features(xf, uf, m.dom, f1, f2);
    const float2 y = net_outputs<SAMP>(s_net, m, inside, f1, f2);
    double v = 0.0;
    if (__any(fallback)) {
        const double vf = angle_icdf_v(fallback ? u : 0.5, fallback ? x : 0.0);
        if (fallback) v = vf;
    }
    if (!active) return;
    if (inside) v = net_reading_v(xf, y.x, y.y);
    d3 p, k;
    double we, wg;
    src.get(a, ie, ig, p, k, we, wg);
    const PairInv inv = pair_invariants(p, k);
    const Scattered s = scatter(p, k, inv, v, uniform53(r.c, r.d));
    write_back<T>(a, ie, ig, we, wg, s, seed, step);
    sums.e_before += s.e_before;
    sums.e_after += s.e_after;
    sums.n_fallback += fallback ? 1 : 0;
}

}  // namespace cs
