// cs_device.h -- device-side arithmetic of the Compton step for gfx950.
//
// Counter-based random numbers, the in-cell pairing bijection, the
// Klein-Nishina cross-section and angular CDF, the inverse-CDF sampler and
// the rest-frame/lab kinematics.  All physics arithmetic is FP64 and written
// in forms free of catastrophic cancellation for gamma >> 1 (the Lorentz
// boosts and back-transforms), so that a FP32-stored plasma loses nothing
// beyond its storage rounding.
//
// Units: momenta in m_e c, energies in m_e c^2, s(x) = sigma_KN / sigma_T.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cs_sigma_table.h"

namespace cs {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32
// S-box, key advanced by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct u32x4 {
    uint32_t a, b, c, d;
};

// a ^ b ^ c in one v_bitop3_b32 (truth table 0x96); c must be wave-uniform
// (it is read from a scalar register).
__device__ __forceinline__ uint32_t xor3_uniform(uint32_t a, uint32_t b, uint32_t c) {
    uint32_t r;
    asm("v_bitop3_b32 %0, %1, %2, %3 bitop3:0x96" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// The key (k0, k1) must be wave-uniform (it is the seed everywhere here).
__device__ __forceinline__ u32x4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                          uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t m0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t m1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = xor3_uniform((uint32_t)(m1 >> 32), c1, k0);
        const uint32_t n2 = xor3_uniform((uint32_t)(m0 >> 32), c3, k1);
        c1 = (uint32_t)m1;
        c3 = (uint32_t)m0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Stream purposes (fourth counter word, low byte).
enum : uint32_t {
    kPair = 1,
    kCollide = 2,
    kScatter = 3,
    // no-time-counter candidate selection
    kNtcCount = 4,
    kNtcPick = 5,
    kNtcScatter = 6,
    kNtcWeight = 7
};

// counter = (index lo, index hi, step lo, step hi << 8 | purpose), key = seed.
__device__ __forceinline__ u32x4 draw(uint64_t seed, uint64_t index, uint64_t step, uint32_t purpose) {
    return philox10((uint32_t)index, (uint32_t)(index >> 32), (uint32_t)step,
                    ((uint32_t)(step >> 32) << 8) | purpose, (uint32_t)seed, (uint32_t)(seed >> 32));
}

// 53-bit uniform in [0, 1): top 27 bits of a, top 26 bits of b.
__device__ __forceinline__ double uniform53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * 0x1p-53;
}

// ---------------------------------------------------------------------------
// In-cell pairing: 4-round Feistel network over b = ceil(log2 M) bits with
// cycle-walking into [0, M) (Black & Rogaway 2002).  The left part has
// floor(b/2) bits and the right part the rest; a round maps (L, R) to
// (R, L ^ F(R)), so the widths trade places each round and are back after
// four.  Round function: MurmurHash3's 32-bit finaliser of (right part ^ key
// word), cut to the width of the left part.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

struct FeistelKey {
    uint32_t k[4];
    uint32_t bits;  // b = ceil(log2 M)
};

__device__ __forceinline__ uint32_t ceil_log2(uint32_t M) { return M <= 1 ? 0u : 32u - __clz(M - 1u); }

// The cycle-walk always ends: i lies on a cycle of the permutation of
// [0, 2^b), and that cycle returns to i, which is < M.
__device__ __forceinline__ uint32_t shuffle_index(uint32_t i, uint32_t M, const FeistelKey& key) {
    if (M <= 1u) return 0u;
    const uint32_t a = key.bits >> 1, c = key.bits - a;
    const uint32_t mask_a = (1u << a) - 1u, mask_c = (1u << c) - 1u;
    uint32_t v = i;
    do {
        uint32_t L = v >> c, R = v & mask_c;  // widths a, c
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
            const uint32_t R1 = L ^ (fmix32(R ^ key.k[r]) & mask_a);  // (L, R) -> (R, R1): widths c, a
            const uint32_t R2 = R ^ (fmix32(R1 ^ key.k[r + 1]) & mask_c);  // -> (R1, R2): widths a, c
            L = R1;
            R = R2;
        }
        v = (L << c) | R;
    } while (v >= M);
    return v;
}

// ---------------------------------------------------------------------------
// Klein-Nishina.  With a = 1 + x(1 - mu) the rest-frame angular density is
// f(mu) = a^-3 + a^-1 - (1 - mu^2) a^-2 (unnormalised), and
// s(x) = (3/8) int_{-1}^{1} f dmu.
// ---------------------------------------------------------------------------

// Upper tail of the angular integral, T(v) = int_{1-v}^{1} f dmu, by the
// three integrals in w = 1 - mu (a = 1 + x w; z = x v, A = 1 + z):
//   int a^-3 dw = v (2 + z) / (2 A^2),
//   int a^-1 dw = log1p(z) / x,
//   int w (2 - w) a^-2 dw = 2 phi2(z) / x^2 - phi3(z) / x^3,
//     phi2 = log1p(z) - z / (1 + z),  phi3 = z - 2 log1p(z) + z / (1 + z),
// and T = first + second - third.  With s = z / (2 + z) (so log1p(z) =
// 2 atanh(s)) and q = s / x = v / (2 + z), sigma = s^2:
//   log1p(z) / x = 2 q S1,            S1 = sum_{k>=0} sigma^k / (2k+1),
//   phi2 / x^2 = q^2 (2 / (1 + s) + s S2),  S2 = sum_{k>=0} 2 sigma^k / (2k+3),
//   phi3 / x^3 = q^3 S3,              S3 = sum_{k>=0} 8 (k+1) sigma^k / (2k+3).
// Every term of the three series is positive, so they lose nothing to
// cancellation at small x (where the closed form loses about 1/x^2 of its
// precision); they converge like sigma^k with sigma < 1/4 for z < 2.  The
// series branch serves x < 1; kTailTerms terms reach round-off at sigma
// just below 1/4, and a lane with a smaller sigma takes fewer (see
// tail_series).
constexpr int kTailChunk = 6;   // terms per Horner chunk
constexpr int kTailTerms = 30;  // five chunks
constexpr double kSeriesSwitch = 1.0;

struct TailCoeffs {
    double s1[kTailTerms], s2[kTailTerms], s3[kTailTerms];
};

constexpr TailCoeffs tail_series_coeffs() {
    TailCoeffs r{};
    for (int k = 0; k < kTailTerms; ++k) {
        const double kk = (double)k;
        r.s1[k] = 1.0 / (2.0 * kk + 1.0);
        r.s2[k] = 2.0 / (2.0 * kk + 3.0);
        r.s3[k] = 8.0 * (kk + 1.0) / (2.0 * kk + 3.0);
    }
    return r;
}

__constant__ constexpr TailCoeffs kTail = tail_series_coeffs();

typedef const __attribute__((address_space(4))) double* cdptr;  // constant (scalar-load) space

// a * b + c with c held in a scalar register pair: one v_fma_f64 that reads
// the coefficient directly (the compiler's own selection copies each scalar
// coefficient into vector registers first, two extra instructions per term).
__device__ __forceinline__ double fma_sgpr(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "s"(c));
    return r;
}

// t^N by repeated squaring (N known at compile time).
template <int N>
__device__ __forceinline__ double ipow(double t) {
    if constexpr (N == 1) {
        return t;
    } else if constexpr (N % 2 == 0) {
        const double h = ipow<N / 2>(t);
        return h * h;
    } else {
        return ipow<N - 1>(t) * t;
    }
}

// 1/a to about an ulp (hardware estimate and two Newton steps).
__device__ __forceinline__ double recip_approx(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = fma(fma(-a, r, 1.0), r, r);
    return fma(fma(-a, r, 1.0), r, r);
}

// sum_{k < 6 nch} c_k t^k for this lane's nch <= NC chunks of kTailChunk
// terms: the wave evaluates NC chunks (Horner each, from scalar registers),
// the lane zeroes those at or beyond its nch, and the chunks are combined
// from the top in powers of t^6.  A zeroed chunk leaves the combination at
// exactly 0 and fma(0, t^6, p) = p, so the lane's result is bit for bit its
// own nch-chunk sum, whatever NC its wave needs.
template <int NC>
__device__ __forceinline__ double poly_lane_chunks(cdptr c, double t, int nch) {
    double part[NC];
#pragma unroll
    for (int i = 0; i < NC; ++i) {
        const int lo = i * kTailChunk;
        double acc = c[lo + kTailChunk - 1];
#pragma unroll
        for (int k = lo + kTailChunk - 2; k >= lo; --k) acc = fma_sgpr(acc, t, c[k]);
        part[i] = i == 0 || i < nch ? acc : 0.0;
    }
    if constexpr (NC == 1) {
        return part[0];
    } else {
        const double tc = ipow<kTailChunk>(t);
        double r = part[NC - 1];
#pragma unroll
        for (int i = NC - 2; i >= 0; --i) r = fma(r, tc, part[i]);
        return r;
    }
}

// T(v) from the three series, each with this lane's nch chunks (the wave's
// NC >= nch evaluated).  The coefficient pointers pass through an empty asm
// so that the compiler reads the coefficients with scalar loads at each use
// instead of hoisting whole tables into vector registers across the
// sampler's iteration.
template <int NC>
__device__ __forceinline__ double tail_terms(double v, double z, double A, double s, double q, double sig,
                                             int nch) {
    cdptr S1 = (cdptr)kTail.s1, S2 = (cdptr)kTail.s2, S3 = (cdptr)kTail.s3;
    asm volatile("" : "+s"(S1), "+s"(S2), "+s"(S3));
    const double p1 = poly_lane_chunks<NC>(S1, sig, nch);
    const double p2 = poly_lane_chunks<NC>(S2, sig, nch);
    const double p3 = poly_lane_chunks<NC>(S3, sig, nch);
    const double iA = recip_approx(A);
    const double first = 0.5 * v * (2.0 + z) * iA * iA;
    const double inner = fma(s, p2, 2.0 * recip_approx(1.0 + s));
    return first + 2.0 * q * p1 - 2.0 * q * q * inner + q * q * q * p3;
}

// Series branch of T(v) for x < kSeriesSwitch.  Each lane takes as many
// terms as its own sigma needs for the truncated remainder to stay below
// 1e-17 of the sum: 6 terms up to sigma = 1.5e-3, 12 up to 0.035, 18 up to
// 0.112, else kTailTerms (sigma < 1/4).  The wave evaluates the chunks its
// largest need requires; a lane's result depends on its own sigma only
// (poly_lane_chunks), so it is the same whichever lanes share its wave --
// every kernel strategy, whose waves group the collisions differently,
// gives the same bits.
__device__ __forceinline__ double tail_series(double x, double v) {
    const double z = x * v;
    const double r = recip_approx(2.0 + z);
    const double s = z * r, q = v * r, sig = s * s;
    const double A = 1.0 + z;
    const int nch = sig <= 1.5e-3 ? 1 : (sig <= 0.035 ? 2 : (sig <= 0.112 ? 3 : kTailTerms / kTailChunk));
    if (__all(nch <= 1)) return tail_terms<1>(v, z, A, s, q, sig, nch);
    if (__all(nch <= 2)) return tail_terms<2>(v, z, A, s, q, sig, nch);
    if (__all(nch <= 3)) return tail_terms<3>(v, z, A, s, q, sig, nch);
    return tail_terms<kTailTerms / kTailChunk>(v, z, A, s, q, sig, nch);
}

// s(x) = sigma_KN(x) / sigma_T.  Below 2: the per-segment Taylor polynomial
// of cs_sigma_table.h, evaluated per lane (each lane loads its own segment's
// 12 coefficients; no lane waits for another's branch).  `tab` is kSigTab or
// a copy of it (e.g. in LDS): the same coefficients, the same result.  From
// 2 to 2^17 the second table (segment index and centre from the exponent and
// the top four mantissa bits); above, the closed form with log1p.
__device__ __forceinline__ double sigma_ratio_tab(double x, const double* tab) {
    if (x < kSigTabMax) {
        int j = (int)(x * kSigTabInvWidth);
        j = j < 0 ? 0 : (j > kSigTabSegments - 1 ? kSigTabSegments - 1 : j);
        const double t = x - ((double)j + 0.5) / kSigTabInvWidth;
        const double* a = tab + j * kSigTabTerms;
        double acc = a[kSigTabTerms - 1];
#pragma unroll
        for (int n = kSigTabTerms - 2; n >= 0; --n) acc = fma(acc, t, a[n]);
        return acc;
    }
    if (x < kSigTabHiMax) {
        // (hi >> 16) = (1023 + e) << 4 | m for x = 2^e (1 + m/16 + ...)
        const int hi = __double2hiint(x);
        const int j = (hi >> 16) - ((1023 + 1) << 4);
        const double t = x - __hiloint2double((hi & (int)0xFFFF0000) | 0x8000, 0);
        const double* a = kSigTabHi + j * kSigTabTerms;
        double acc = a[kSigTabTerms - 1];
#pragma unroll
        for (int n = kSigTabTerms - 2; n >= 0; --n) acc = fma(acc, t, a[n]);
        return acc;
    }
    const double l = log1p(2.0 * x);
    const double opx = 1.0 + x, o2x = 1.0 + 2.0 * x;
    return 0.75 * (opx / (x * x * x) * (2.0 * x * opx / o2x - l) + l / (2.0 * x) - (1.0 + 3.0 * x) / (o2x * o2x));
}

__device__ __forceinline__ double sigma_ratio(double x) { return sigma_ratio_tab(x, kSigTab); }

// Unnormalised angular density f at mu = 1 - v, for x >= 0.
__device__ __forceinline__ double angle_density_v(double v, double x) {
    const double a = 1.0 + x * v;
    const double ia = 1.0 / a;
    return ia * ia * ia + ia - v * (2.0 - v) * ia * ia;
}


// int_{1 - v}^{1} f dmu (upper tail), for 0 <= v <= 2.
//   series branch (x < kSeriesSwitch): as above;
//   closed branch: with a = 1 + x v and G' = f in a,
//   (1/x)[G(a) - G(1)] = (1/x)[ x v (2 + x v) / (2 a^2) + log1p(x v)
//                        - (-(x v) + (2x+2) log1p(x v) - (2x+1) x v / a) / x^2 ].
__device__ __forceinline__ double angle_tail(double v, double x) {
    if (x < kSeriesSwitch) return tail_series(x, v);
    const double xv = x * v;
    const double a = 1.0 + xv;
    const double L = log1p(xv);
    const double g = xv * (2.0 + xv) / (2.0 * a * a) + L -
                     (-xv + (2.0 * x + 2.0) * L - (2.0 * x + 1.0) * xv / a) / (x * x);
    return g / x;
}

// Thomson-limit inverse (x -> 0): root of (mu^3 + 3 mu + 4)/8 = u by Cardano;
// with q = 4u - 2 and A = cbrt(q + sqrt(q^2 + 1)) the root is A - 1/A.
__device__ __forceinline__ double thomson_root(double u) {
    const double q = 4.0 * u - 2.0;
    const double A = cbrt(q + sqrt(q * q + 1.0));
    return A - 1.0 / A;
}

// Inverse CDF of the rest-frame scattering angle, returned as v = 1 - mu so
// that forward scatters (mu -> 1) keep relative precision: the v with
// tail(v) = (1 - u) Z, Z = tail(2) = (8/3) s(x).
//
// Start: for x < 1/2 the Thomson root v0 = 1 - mu0 corrected to first order
// in x: with tail = v(2 - v + v^2/3) - x v^2 (2 - 4v/3 + v^2/2) + O(x^2) and
// Z = 8/3 - 16x/3 + O(x^2), v1 = [v0^2 (2 - 4 v0/3 + v0^2/2) - 16(1 - u)/3]
// / (2 - 2 v0 + v0^2); for x >= 1/2 the inverse of the large-x law
// F ~ ln((1+2x)/a) / ln(1+2x), a = 1 + x v.  Then Halley's iteration in v
// (slope: the density f; curvature: f' in closed form), safeguarded by a
// bisection bracket, falling back to a Newton step if Halley's denominator
// is not positive.  A Halley step below 1e-5 v (a Newton step below 1e-8 v)
// is accepted and ends the iteration: the error after it is at round-off
// (cubic convergence leaves about C v (1e-5)^3, quadratic C v (1e-8)^2, with
// C = O(1); against the converged root the accepted values stay within
// 2.2e-15 relative over x in [1e-4, 1e3]).  An exact zero residual ends it
// too.  Only the residual (the tail series or closed
// form) decides where the iteration lands, so the step sizes use reciprocal
// estimates refined to about an ulp.
__device__ __forceinline__ double angle_icdf_v(double u, double x) {
    const double Z = (8.0 / 3.0) * sigma_ratio(x);
    const double target = (1.0 - u) * Z;  // 1 - u is exact for u = k 2^-53
    double lo = 0.0, hi = 2.0;
    double v;
    if (x < 0.5) {
        const double v0 = 1.0 - thomson_root(u);
        const double v1 = (v0 * v0 * (2.0 - 4.0 / 3.0 * v0 + 0.5 * v0 * v0) - 16.0 / 3.0 * (1.0 - u)) /
                          (2.0 - 2.0 * v0 + v0 * v0);
        v = v0 + x * v1;
    } else {
        v = expm1((1.0 - u) * log1p(2.0 * x)) / x;
    }
    v = fmin(fmax(v, 0.0), 2.0);
    for (int it = 0; it < 60; ++it) {
        const double R = angle_tail(v, x) - target;  // > 0: v too large
        if (R == 0.0) break;
        if (R > 0.0)
            hi = v;
        else
            lo = v;
        // Halley step on the tail: slope f (the density) and curvature f'
        const double ia = recip_approx(1.0 + x * v);
        const double ia2 = ia * ia, ia3 = ia2 * ia;
        const double w = v * (2.0 - v);
        const double f = ia3 + ia - w * ia2;
        const double fp = -3.0 * x * ia3 * ia - x * ia2 - (2.0 - 2.0 * v) * ia2 + 2.0 * x * w * ia3;
        const double den = 2.0 * f * f - R * fp;
        const bool halley = den > 0.0;
        double next = halley ? v - 2.0 * R * f * recip_approx(den) : v - R * recip_approx(f);
        if (fabs(next - v) <= (halley ? 1e-5 : 1e-8) * next) {
            v = next;
            break;
        }
        if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
        v = next;
        if (hi - lo <= 1e-16 * hi) break;
    }
    return fmin(fmax(v, 0.0), 2.0);
}

// ---------------------------------------------------------------------------
// Kinematics (FP64, cancellation-free forms)
// ---------------------------------------------------------------------------
struct d3 {
    double x, y, z;
};

__device__ __forceinline__ double dot(d3 a, d3 b) { return fma(a.x, b.x, fma(a.y, b.y, a.z * b.z)); }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return {fma(a.y, b.z, -(a.z * b.y)), fma(a.z, b.x, -(a.x * b.z)), fma(a.x, b.y, -(a.y * b.x))};
}
__device__ __forceinline__ d3 axpy(double a, d3 x, d3 y) { return {fma(a, x.x, y.x), fma(a, x.y, y.y), fma(a, x.z, y.z)}; }
__device__ __forceinline__ d3 scale(double a, d3 x) { return {a * x.x, a * x.y, a * x.z}; }

// sqrt(a) for a normal, positive a: the hardware reciprocal square root
// refined by Goldschmidt's iteration with two residual corrections (within
// about an ulp; no scaling or special-case handling).
__device__ __forceinline__ double sqrt_normal(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    double g = a * y, h = 0.5 * y;
    const double r = fma(-h, g, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    double d = fma(-g, g, a);
    g = fma(d, h, g);
    d = fma(-g, g, a);
    return fma(d, h, g);
}

// n / d for normal d: the hardware reciprocal refined by two Newton steps,
// the quotient, and one residual correction (within about an ulp).
__device__ __forceinline__ double div_normal(double n, double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    const double q = n * r;
    return fma(fma(-d, q, n), r, q);
}

struct XFlux {
    double x, flux;  // rest-frame photon energy x = gamma eps - p.k, flux = x / (gamma eps)
};

// gamma eps = sqrt((1 + p.p) k.k) (one square root); x = gamma eps - p.k, and
// for p.k > 0 the cancellation-free x = (k.k + |p x k|^2) / (gamma eps + p.k)
// (gamma^2 eps^2 - (p.k)^2 = eps^2 + |p x k|^2).  Both cases share one
// division: flux = num / den with (num, den) = (gamma eps - p.k, gamma eps),
// resp. (k.k + |p x k|^2, gamma eps (gamma eps + p.k)), and then x = flux
// gamma eps in the second case.  pp = p.p, kk = k.k.  FAST: the square root
// and the division are the refined hardware estimates above, valid while
// their operands are normal numbers.
template <bool FAST>
__device__ __forceinline__ XFlux x_flux_impl(d3 p, d3 k, double pp, double kk) {
    const double a = (1.0 + pp) * kk;
    const double ge = FAST ? sqrt_normal(a) : sqrt(a);
    const double pk = dot(p, k);
    const bool fwd = pk > 0.0;
    const d3 c = cross(p, k);
    const double num = fwd ? kk + dot(c, c) : ge - pk;
    const double den = fwd ? ge * (ge + pk) : ge;
    XFlux r;
    r.flux = FAST ? div_normal(num, den) : num / den;
    r.x = fwd ? r.flux * ge : num;
    return r;
}

// The fast form wherever (1 + p.p) k.k lies in [1e-300, 1e300] (then every
// operand above is normal); the IEEE square root and division outside.
__device__ __forceinline__ XFlux x_flux(d3 p, d3 k, double pp, double kk) {
    if (kk == 0.0) return {0.0, 0.0};
    const double a = (1.0 + pp) * kk;
    if (a >= 1e-300 && a <= 1e300) return x_flux_impl<true>(p, k, pp, kk);
    return x_flux_impl<false>(p, k, pp, kk);
}

struct PairInv {
    double gamma, eps, x, flux;
};

__device__ __forceinline__ PairInv pair_invariants(d3 p, d3 k) {
    const double pp = dot(p, p), kk = dot(k, k);
    const XFlux xf = x_flux(p, k, pp, kk);
    PairInv r;
    r.gamma = sqrt(1.0 + pp);
    r.eps = sqrt(kk);
    r.x = xf.x;
    r.flux = xf.flux;
    return r;
}

struct Scattered {
    d3 p1, k1;
    double e_before, e_after;
};

// Resolve one collision.  Rest frame of the electron (velocity p/gamma):
// photon direction n from the decomposition of k along p_hat (perpendicular
// part unchanged, parallel part gamma k_par - |p| eps written without
// cancellation); scattered direction d = mu n + sin(theta)(cos(phi) e1 +
// sin(phi) e2) about the Duff et al. (JCGT 2017) orthonormal basis of n,
// with v = 1 - mu and sin(theta) = sqrt(v (2 - v));
// Compton shift x1 = x / (1 + x v); back-boost with the pre-collision
// p (parallel part x1 (gamma c + |p|), again cancellation-free); the
// electron takes p + k - k1.
__device__ __forceinline__ Scattered scatter(d3 p, d3 k, const PairInv& inv, double v, double u_phi) {
    const double gamma = inv.gamma, eps = inv.eps, x = inv.x;
    const double pp2 = dot(p, p);
    const double pp = sqrt(pp2);
    d3 n, ph;
    const bool moving = pp > 0.0;
    if (moving) {
        ph = scale(1.0 / pp, p);
        const double kpar = dot(k, ph);
        const d3 kperp = axpy(-kpar, ph, k);
        double kpar_r;
        if (kpar <= 0.0) {
            kpar_r = gamma * kpar - pp * eps;
        } else {
            const d3 c = cross(ph, k);
            kpar_r = (eps * eps - gamma * gamma * dot(c, c)) / (gamma * kpar + pp * eps);
        }
        n = axpy(kpar_r, ph, kperp);
    } else {
        ph = {0.0, 0.0, 0.0};
        n = k;
    }
    const double nn = 1.0 / sqrt(dot(n, n));
    n = scale(nn, n);
    // orthonormal basis (Duff et al. 2017)
    const double s = n.z >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (s + n.z);
    const double b = n.x * n.y * a;
    const d3 e1 = {1.0 + s * n.x * n.x * a, s * b, -s * n.x};
    const d3 e2 = {b, s + n.y * n.y * a, -n.y};
    double sphi, cphi;
    sincospi(2.0 * u_phi, &sphi, &cphi);
    const double mu = 1.0 - v;
    const double st = sqrt(v * (2.0 - v));
    d3 d = scale(mu, n);
    d = axpy(st * cphi, e1, d);
    d = axpy(st * sphi, e2, d);
    const double x1 = x / (1.0 + x * v);
    d3 k1;
    if (moving) {
        const double c = dot(d, ph);
        const d3 dperp = axpy(-c, ph, d);
        double par;
        if (c >= 0.0) {
            par = x1 * (gamma * c + pp);
        } else {
            const d3 cr = cross(ph, d);
            par = x1 * (1.0 - gamma * gamma * dot(cr, cr)) / (gamma * c - pp);
        }
        k1 = axpy(par, ph, scale(x1, dperp));
    } else {
        k1 = scale(x1, d);
    }
    Scattered r;
    r.k1 = k1;
    r.p1 = {(p.x + k.x) - k1.x, (p.y + k.y) - k1.y, (p.z + k.z) - k1.z};
    r.e_before = gamma + eps;
    r.e_after = sqrt(1.0 + dot(r.p1, r.p1)) + sqrt(dot(k1, k1));
    return r;
}

}  // namespace cs
