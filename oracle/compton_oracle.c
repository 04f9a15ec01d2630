/*
 * compton_oracle.c -- plain, slow, FP64 CPU oracle of the per-pair Compton
 * scattering Monte-Carlo step (TEST INFRASTRUCTURE ONLY).
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the GPU path.
 *
 * What it follows (Badiali et al., "Machine Learning-based models in
 * particle-in-cell codes for advanced physics extensions"):
 *   Sec. 3.1  the module's three steps: bin particles into collision cells and
 *             form a pair list per cell; for each pair compute the interaction
 *             probability and compare it with a random number; resolve every
 *             accepted collision and update both momenta.
 *   Sec. 3.2  the probability: boost the photon into the lepton rest frame,
 *             evaluate the Klein-Nishina cross-section there, carry the rate
 *             back to the lab frame; P_max = 2 sigma_T c dt max[w_e, w_gamma].
 * Everything the paper leaves to its reference on the Compton module (pairing
 * rule, exact normalisation, angle sampling, weight rule, RNG) follows the
 * readings listed in the design notes, restated next to each function here.
 *
 * Precision: every Lorentz boost and every lab-frame kinematic quantity is
 * evaluated in IEEE binary128 (__float128) from the definition, so that the
 * FP64 results below carry no cancellation error; the cross-section and the
 * angular CDF are evaluated in FP64 by a term-by-term integrated series below
 * x = 0.2 and by the closed form in binary128 above it.
 *
 * Units: momenta in m_e c, energies in m_e c^2, cross-sections as
 * s(x) = sigma_KN(x) / sigma_T.
 */
#include <math.h>
#include <quadmath.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 quad;

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11 "Parallel random numbers:  */
/* as easy as 1, 2, 3"): 10 rounds of the 4x32 S-box with the published       */
/* multipliers and Weyl key increments.                                        */
/* ------------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Stream purposes carried in the fourth counter word. */
enum { PURPOSE_PAIR = 1, PURPOSE_COLLIDE = 2, PURPOSE_SCATTER = 3,
       /* no-time-counter candidate selection */
       PURPOSE_NTC_COUNT = 4, PURPOSE_NTC_PICK = 5, PURPOSE_NTC_SCATTER = 6, PURPOSE_NTC_WEIGHT = 7 };

/* counter = (index lo, index hi, step lo, (step hi << 8) | purpose), key = seed */
static void draw(uint64_t seed, uint64_t index, uint64_t step, uint32_t purpose, uint32_t out[4])
{
    uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), (uint32_t)step,
                       ((uint32_t)(step >> 32) << 8) | purpose};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Uniform in [0, 1) from two 32-bit words: the top 27 bits of the first and
 * the top 26 bits of the second form a 53-bit integer, scaled by 2^-53. */
double oracle_uniform53(uint32_t a, uint32_t b)
{
    double hi = (double)(a >> 5);
    double lo = (double)(b >> 6);
    return (hi * 67108864.0 + lo) / 9007199254740992.0;
}

/* The two uniforms that resolve the collision of the pair whose electron has
 * index idx[i]: cos(theta) sampling (u_mu) and azimuth (u_phi). */
void oracle_scatter_uniforms(const int64_t* idx, int64_t n, uint64_t seed, uint64_t step, double* u_mu,
                             double* u_phi)
{
    for (int64_t i = 0; i < n; ++i) {
        uint32_t r[4];
        draw(seed, (uint64_t)idx[i], step, PURPOSE_SCATTER, r);
        u_mu[i] = oracle_uniform53(r[0], r[1]);
        u_phi[i] = oracle_uniform53(r[2], r[3]);
    }
}

/* ------------------------------------------------------------------------- */
/* Pairing: a keyed pseudo-random bijection of [0, M) (the in-cell shuffle).  */
/* A 4-round Feistel network over b = ceil(log2 M) bits, made a bijection of  */
/* [0, M) by cycle-walking (Black & Rogaway 2002).  The b bits split into a   */
/* left part of a = floor(b/2) bits and a right part of c = b - a bits; each  */
/* round replaces (L, R) by (R, L xor F_r(R)), so the two widths trade places */
/* every round and are back after four (for even b both halves are b/2 wide).*/
/* F_r mixes R with key word r through the MurmurHash3 32-bit finaliser and   */
/* keeps as many bits as L has.  The four key words are the Philox output for */
/* (index = cell id, step, purpose PAIR).                                      */
/* ------------------------------------------------------------------------- */
static uint32_t murmur_fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85EBCA6Bu;
    h ^= h >> 13;
    h *= 0xC2B2AE35u;
    h ^= h >> 16;
    return h;
}

uint64_t oracle_shuffle_index(uint64_t i, uint64_t M, uint64_t seed, uint64_t cell, uint64_t step)
{
    if (M <= 1) return 0;
    int bits = 0;
    while (((uint64_t)1 << bits) < M) ++bits;        /* bits = ceil(log2 M) */
    const int a = bits / 2, c = bits - a;             /* widths of L and R    */
    uint32_t keys[4];
    draw(seed, cell, step, PURPOSE_PAIR, keys);
    uint64_t v = i;
    do {
        uint64_t L = v >> c, R = v & (((uint64_t)1 << c) - 1);
        int wl = a, wr = c;                           /* current widths       */
        for (int r = 0; r < 4; ++r) {
            uint64_t f = murmur_fmix32((uint32_t)R ^ keys[r]) & (((uint64_t)1 << wl) - 1);
            uint64_t newL = R;
            uint64_t newR = L ^ f;
            L = newL;
            R = newR;
            int t = wl;
            wl = wr;
            wr = t;
        }
        v = (L << c) | R;                              /* wl = a, wr = c again */
    } while (v >= M);
    return v;
}

/* The whole permutation of [0, M) for one cell and step (out[i] = pi(i)). */
void oracle_shuffle_all(uint64_t M, uint64_t seed, uint64_t cell, uint64_t step, int64_t* out)
{
    for (uint64_t i = 0; i < M; ++i) out[i] = (int64_t)oracle_shuffle_index(i, M, seed, cell, step);
}

/* ------------------------------------------------------------------------- */
/* Klein-Nishina cross-section in units of sigma_T, s(x), x = rest-frame      */
/* photon energy.  The rest-frame angular density in mu = cos(theta) is,     */
/* up to a constant, f(mu) = a^-3 + a^-1 - (1 - mu^2) a^-2 with               */
/* a = 1 + x (1 - mu) (the Klein-Nishina formula); s(x) = 3/8 * int f dmu.    */
/* ------------------------------------------------------------------------- */

/* Upper bound on the number of terms of the small-x series: the k-th term is
 * O((2x)^k k) with 2x < 0.4, so 200 terms are far past round-off. */
#define SERIES_TERMS 200

/* The pdf series: with t = x (1 - mu), a^-n = sum_k C(k+n-1, n-1) (-t)^k, so
 * f(mu) = sum_k (-x)^k (1-mu)^k [ (k+1)(k+2)/2 + 1 - (k+1)(1 - mu^2) ].
 * Substituting v = 1 - mu (1 - mu^2 = v (2 - v)), the k-th term integrated
 * over v in [v0, 2] (mu in [-1, 1 - v0]) is
 *   J_k(v0) = A_k (2^{k+1} - v0^{k+1}) / (k+1)
 *           - (k+1) [ 2 (2^{k+2} - v0^{k+2}) / (k+2) - (2^{k+3} - v0^{k+3}) / (k+3) ],
 * A_k = (k+1)(k+2)/2 + 1.  The integrand is positive (v(2-v) <= 1 < A_k/(k+1)),
 * so the series in (-x)^k alternates with decreasing terms once (2x)^k k falls,
 * and the tail after a term is bounded by that term (Leibniz). */
/* int_{-1}^{1 - v0} f(mu) dmu by the series (valid for 2x < 1). */
static double series_partial_integral(double x, double v0)
{
    double sum = 0.0, xk = 1.0;
    double two_k1 = 2.0, v_k1 = v0; /* 2^{k+1}, v0^{k+1} at k = 0 */
    for (int k = 0; k < SERIES_TERMS; ++k) {
        double A = (double)(k + 1) * (double)(k + 2) / 2.0 + 1.0;
        double two_k2 = 2.0 * two_k1, two_k3 = 4.0 * two_k1;
        double v_k2 = v_k1 * v0, v_k3 = v_k2 * v0;
        double part_a = A * (two_k1 - v_k1) / (double)(k + 1);
        double part_b = (double)(k + 1) * (2.0 * (two_k2 - v_k2) / (double)(k + 2) -
                                          (two_k3 - v_k3) / (double)(k + 3));
        double term = xk * (part_a - part_b);
        sum += term;
        if (k > 2 && fabs(term) <= 1e-20 * fabs(sum)) break;
        xk *= -x;
        two_k1 *= 2.0;
        v_k1 *= v0;
    }
    return sum;
}

/* int_{1-v}^{1} f dmu by the same series, integrated term by term over
 * w = 1 - mu in [0, v]:
 *   sum_k (-x)^k [ A_k v^{k+1}/(k+1) - 2(k+1) v^{k+2}/(k+2) + (k+1) v^{k+3}/(k+3) ];
 * every term is small with v, so the upper tail keeps relative precision for
 * forward scatters (mu -> 1). */
static double series_upper_integral(double x, double v)
{
    double sum = 0.0, xk = 1.0, v_k1 = v;
    for (int k = 0; k < SERIES_TERMS; ++k) {
        double A = (double)(k + 1) * (double)(k + 2) / 2.0 + 1.0;
        double v_k2 = v_k1 * v, v_k3 = v_k2 * v;
        double term = xk * (A * v_k1 / (double)(k + 1) - 2.0 * (double)(k + 1) * v_k2 / (double)(k + 2) +
                            (double)(k + 1) * v_k3 / (double)(k + 3));
        sum += term;
        if (k > 2 && fabs(term) <= 1e-20 * fabs(sum)) break;
        xk *= -x;
        v_k1 *= v;
    }
    return sum;
}

/* G(a) with dG/da = f expressed in a (closed form antiderivative). */
static quad closed_G(quad a, quad x)
{
    return -1 / (2 * a * a) + logq(a) - (-a + (2 * x + 2) * logq(a) + (2 * x + 1) / a) / (x * x);
}

double oracle_sigma_ratio(double x)
{
    if (!(x >= 0.0)) return NAN;
    if (x < 0.2) {
        return 0.375 * series_partial_integral(x, 0.0);
    }
    /* Textbook closed form of sigma_KN / sigma_T, evaluated in binary128. */
    quad X = x;
    quad l = log1pq(2 * X);
    quad s = (quad)0.75 * ((1 + X) / (X * X * X) * (2 * X * (1 + X) / (1 + 2 * X) - l) +
                           l / (2 * X) - (1 + 3 * X) / ((1 + 2 * X) * (1 + 2 * X)));
    return (double)s;
}

/* Normalised angular density f(mu)/int f, i.e. dF/dmu. */
double oracle_angle_pdf(double mu, double x)
{
    double a = 1.0 + x * (1.0 - mu);
    double f = 1.0 / (a * a * a) + 1.0 / a - (1.0 - mu * mu) / (a * a);
    return f / (8.0 / 3.0 * oracle_sigma_ratio(x));
}

/* CDF of the rest-frame scattering cosine written in v = 1 - mu:
 * F(1 - v; x) = int_{-1}^{1-v} f / int_{-1}^{1} f, decreasing in v. */
double oracle_angle_cdf_v(double v, double x)
{
    if (v >= 2.0) return 0.0;
    if (v <= 0.0) return 1.0;
    if (x < 0.2) {
        double total = series_partial_integral(x, 0.0);
        return series_partial_integral(x, v) / total;
    }
    quad X = x, a = 1 + X * (quad)v, amax = 1 + 2 * X;
    quad num = closed_G(amax, X) - closed_G(a, X);
    quad den = closed_G(amax, X) - closed_G((quad)1, X);
    return (double)(num / den);
}

/* CDF F(mu; x) of the rest-frame scattering cosine. */
double oracle_angle_cdf(double mu, double x)
{
    if (mu <= -1.0) return 0.0;
    if (mu >= 1.0) return 1.0;
    return oracle_angle_cdf_v(1.0 - mu, x);
}

/* Upper tail 1 - F(1 - v; x), increasing in v, with relative precision at
 * small v. */
double oracle_angle_upper_v(double v, double x)
{
    if (v <= 0.0) return 0.0;
    if (v >= 2.0) return 1.0;
    if (x < 0.2) return series_upper_integral(x, v) / series_partial_integral(x, 0.0);
    quad X = x, a = 1 + X * (quad)v, amax = 1 + 2 * X;
    quad num = closed_G(a, X) - closed_G((quad)1, X);
    quad den = closed_G(amax, X) - closed_G((quad)1, X);
    return (double)(num / den);
}

/* Inverse CDF solved for v = 1 - mu (the scattering angle's natural variable:
 * forward scatters, mu -> 1, keep full relative precision in v and hence in
 * sin(theta) = sqrt(v (2 - v))), by plain bisection on [0, 2] down to
 * adjacent doubles.  For u >= 1/2 the bisection compares the upper tail with
 * 1 - u (exact for 53-bit uniforms), otherwise F with u. */
double oracle_angle_icdf_v(double u, double x)
{
    double lo = 0.0, hi = 2.0;
    const int upper = u >= 0.5;
    const double one_minus_u = 1.0 - u;
    for (int it = 0; it < 4000; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi || hi - lo <= 1e-17 * hi) break;
        int v_too_small = upper ? oracle_angle_upper_v(mid, x) < one_minus_u : oracle_angle_cdf_v(mid, x) > u;
        if (v_too_small)
            lo = mid;
        else
            hi = mid;
    }
    double elo, ehi;
    if (upper) {
        elo = one_minus_u - oracle_angle_upper_v(lo, x);
        ehi = oracle_angle_upper_v(hi, x) - one_minus_u;
    } else {
        elo = oracle_angle_cdf_v(lo, x) - u;
        ehi = u - oracle_angle_cdf_v(hi, x);
    }
    return (elo <= ehi) ? lo : hi;
}

double oracle_angle_icdf(double u, double x) { return 1.0 - oracle_angle_icdf_v(u, x); }

/* Plain sampler over arrays: mu = F^-1(u; x), r = eps'/eps = 1/(1 + x(1 - mu)). */
void oracle_sample_plain(const double* x, const double* u, int64_t n, double* mu_out, double* ratio_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double v = oracle_angle_icdf_v(u[i], x[i]);
        mu_out[i] = 1.0 - v;
        ratio_out[i] = 1.0 / (1.0 + x[i] * v);
    }
}

/* ------------------------------------------------------------------------- */
/* Lorentz boosts (binary128).                                                 */
/* ------------------------------------------------------------------------- */
static quad dot3(const quad a[3], const quad b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Boost the photon (eps, k) into the rest frame of an electron of momentum p:
 *   E' = gamma eps - p.k,   k' = k + (p.k / (gamma + 1) - eps) p.
 * Returns E' (= x); writes k'. */
static quad boost_to_rest(const quad p[3], quad gamma, const quad k[3], quad eps, quad kr[3])
{
    quad pk = dot3(p, k);
    quad c = pk / (gamma + 1) - eps;
    for (int i = 0; i < 3; ++i) kr[i] = k[i] + c * p[i];
    return gamma * eps - pk;
}

/* Boost a rest-frame photon (e1, q) back to the lab:
 *   eps1 = gamma e1 + p.q,   k1 = q + (p.q / (gamma + 1) + e1) p. */
static quad boost_to_lab(const quad p[3], quad gamma, const quad q[3], quad e1, quad k1[3])
{
    quad pq = dot3(p, q);
    quad c = pq / (gamma + 1) + e1;
    for (int i = 0; i < 3; ++i) k1[i] = q[i] + c * p[i];
    return gamma * e1 + pq;
}

/* Orthonormal basis around a unit vector n (Duff, Burgess, Christensen, Hery,
 * Kensler, Liani, Villemin, "Building an Orthonormal Basis, Revisited",
 * JCGT 6(1), 2017). */
static void onb(const quad n[3], quad e1[3], quad e2[3])
{
    quad s = n[2] >= 0 ? (quad)1 : (quad)-1;
    quad a = -1 / (s + n[2]);
    quad b = n[0] * n[1] * a;
    e1[0] = 1 + s * n[0] * n[0] * a;
    e1[1] = s * b;
    e1[2] = -s * n[0];
    e2[0] = b;
    e2[1] = s + n[1] * n[1] * a;
    e2[2] = -n[1];
}

/* Rest-frame photon energy x and flux factor (1 - beta . k_hat) of a pair. */
void oracle_pair_invariants(const double p_in[3], const double k_in[3], double* x_out, double* flux_out)
{
    quad p[3] = {p_in[0], p_in[1], p_in[2]}, k[3] = {k_in[0], k_in[1], k_in[2]}, kr[3];
    quad gamma = sqrtq(1 + dot3(p, p));
    quad eps = sqrtq(dot3(k, k));
    if (eps == 0) {
        *x_out = 0.0;
        *flux_out = 0.0;
        return;
    }
    quad x = boost_to_rest(p, gamma, k, eps, kr);
    *x_out = (double)x;
    *flux_out = (double)(x / (gamma * eps));
}

/* One resolved collision: given the pre-collision electron p and photon k,
 * the rest-frame scattering angle through v = 1 - cos(theta) and the azimuth
 * phi = 2 pi u_phi, compute the outgoing electron p1 and photon k1 (lab):
 *   1. boost the photon to the electron rest frame: energy x, direction n;
 *   2. scatter about n by (theta, phi) with the Compton shift x1 = x/(1+x v);
 *   3. boost the scattered photon back with the same (pre-collision) p;
 *   4. the electron takes p + k - k1 (momentum conservation).
 * Energies before/after are returned for the conservation check. */
static void scatter_event_v(const double p_in[3], const double k_in[3], quad V, double u_phi, double p_out[3],
                            double k_out[3], double* e_before, double* e_after)
{
    quad p[3] = {p_in[0], p_in[1], p_in[2]}, k[3] = {k_in[0], k_in[1], k_in[2]};
    quad gamma = sqrtq(1 + dot3(p, p));
    quad eps = sqrtq(dot3(k, k));
    quad kr[3], n[3], e1[3], e2[3], d[3], q1[3], k1[3], p1[3];
    quad x = boost_to_rest(p, gamma, k, eps, kr);
    quad kr_norm = sqrtq(dot3(kr, kr));
    for (int i = 0; i < 3; ++i) n[i] = kr[i] / kr_norm;
    onb(n, e1, e2);
    quad Mu = 1 - V;
    quad sin_theta = sqrtq(V * (2 - V));
    quad phi = 2 * M_PIq * (quad)u_phi;
    quad cphi = cosq(phi), sphi = sinq(phi);
    for (int i = 0; i < 3; ++i) d[i] = Mu * n[i] + sin_theta * (cphi * e1[i] + sphi * e2[i]);
    quad x1 = x / (1 + x * V);
    for (int i = 0; i < 3; ++i) q1[i] = x1 * d[i];
    quad eps1 = boost_to_lab(p, gamma, q1, x1, k1);
    for (int i = 0; i < 3; ++i) p1[i] = p[i] + k[i] - k1[i];
    for (int i = 0; i < 3; ++i) {
        p_out[i] = (double)p1[i];
        k_out[i] = (double)k1[i];
    }
    if (e_before) *e_before = (double)(gamma + eps);
    if (e_after) *e_after = (double)(sqrtq(1 + dot3(p1, p1)) + eps1);
}

/* The same with the scattering cosine mu given directly. */
void oracle_scatter_event(const double p_in[3], const double k_in[3], double mu, double u_phi,
                          double p_out[3], double k_out[3], double* e_before, double* e_after)
{
    scatter_event_v(p_in, k_in, 1 - (quad)mu, u_phi, p_out, k_out, e_before, e_after);
}

/* ------------------------------------------------------------------------- */
/* The step.                                                                   */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n_pairs;      /* candidate pairs formed                            */
    int64_t n_collided;   /* pairs with u < P                                  */
    int64_t n_clipped;    /* pairs whose P exceeded 1 (clipped to 1)           */
    int64_t n_invalid;    /* pairs skipped: non-finite input or weight < 0     */
    double sum_prob;      /* sum of P over valid pairs                         */
    double energy_before; /* sum over collided pairs of gamma + eps (before)  */
    double energy_after;  /* sum over collided pairs of gamma' + eps' (after) */
} oracle_stats;

typedef struct {
    int64_t n_pairs, n_collided, n_clipped, n_invalid;
    double sum_prob, energy_before, energy_after;
} cell_tally;

static double load_val(int dtype, const void* a, int64_t i)
{
    return dtype == 1 ? ((const double*)a)[i] : (double)((const float*)a)[i];
}

static void store_val(int dtype, void* a, int64_t i, double v)
{
    if (dtype == 1)
        ((double*)a)[i] = v;
    else
        ((float*)a)[i] = (float)v;
}

static int finite_nonneg_pair(const double p[3], double we, const double k[3], double wg)
{
    for (int i = 0; i < 3; ++i)
        if (!isfinite(p[i]) || !isfinite(k[i])) return 0;
    if (!isfinite(we) || !isfinite(wg)) return 0;
    if (we < 0.0 || wg < 0.0) return 0;
    return 1;
}

/* Process one collision cell (cells are independent). */
static void process_cell(int dtype, void* const E[4], void* const G[4], int64_t c, int64_t e0, int64_t ne,
                         int64_t g0, int64_t ng, double dt, double density_norm, uint64_t seed, uint64_t step,
                         cell_tally* t, double* diag_P, double* diag_u, double* diag_x, int64_t* diag_partner,
                         const double* mu_given)
{
    memset(t, 0, sizeof(*t));
    int64_t n_min = ne < ng ? ne : ng, n_max = ne < ng ? ng : ne;
    if (n_min == 0) return;
    /* Rate per pair: N_max partners are represented by the one partner drawn. */
    double tau = dt * density_norm * (double)n_max;
    for (int64_t i = 0; i < n_min; ++i) {
        int64_t ie, ig;
        if (ne <= ng) {
            ie = e0 + i;
            ig = g0 + (int64_t)oracle_shuffle_index((uint64_t)i, (uint64_t)ng, seed, (uint64_t)c, step);
        } else {
            ig = g0 + i;
            ie = e0 + (int64_t)oracle_shuffle_index((uint64_t)i, (uint64_t)ne, seed, (uint64_t)c, step);
        }
        t->n_pairs++;
        double p[3] = {load_val(dtype, E[0], ie), load_val(dtype, E[1], ie), load_val(dtype, E[2], ie)};
        double k[3] = {load_val(dtype, G[0], ig), load_val(dtype, G[1], ig), load_val(dtype, G[2], ig)};
        double we = load_val(dtype, E[3], ie), wg = load_val(dtype, G[3], ig);
        if (diag_partner) diag_partner[ie] = ig;
        if (!finite_nonneg_pair(p, we, k, wg)) {
            t->n_invalid++;
            continue;
        }
        /* Step 1: photon into the electron rest frame -> x, flux factor. */
        double x, flux;
        oracle_pair_invariants(p, k, &x, &flux);
        /* Step 2: Klein-Nishina cross-section, lab-frame probability. */
        double w_max = we > wg ? we : wg, w_min = we > wg ? wg : we;
        double P = (x > 0.0) ? tau * w_max * oracle_sigma_ratio(x) * flux : 0.0;
        if (P > 1.0) {
            t->n_clipped++;
            P = 1.0;
        }
        t->sum_prob += P;
        uint32_t r[4];
        draw(seed, (uint64_t)ie, step, PURPOSE_COLLIDE, r);
        double u_c = oracle_uniform53(r[0], r[1]);
        double u_w = oracle_uniform53(r[2], r[3]);
        if (diag_P) diag_P[ie] = P;
        if (diag_u) diag_u[ie] = u_c;
        if (diag_x) diag_x[ie] = x;
        /* Step 3: compare with a uniform number. */
        if (!(u_c < P)) continue;
        t->n_collided++;
        /* Step 4: resolve the collision. */
        uint32_t s[4];
        draw(seed, (uint64_t)ie, step, PURPOSE_SCATTER, s);
        double u_mu = oracle_uniform53(s[0], s[1]);
        double u_phi = oracle_uniform53(s[2], s[3]);
        /* The learned sampler stands in for the inverse-CDF step (Sec. 3.2):
         * when the caller supplies cos(theta) for this electron's pair, that
         * angle is used; otherwise the plain sampler draws it. */
        double v = (mu_given && !isnan(mu_given[ie])) ? 1.0 - mu_given[ie] : oracle_angle_icdf_v(u_mu, x);
        double p1[3], k1[3], eb, ea;
        scatter_event_v(p, k, (quad)v, u_phi, p1, k1, &eb, &ea);
        t->energy_before += eb;
        t->energy_after += ea;
        /* Weight rule: the lighter macro-particle always scatters, the heavier
         * one with probability w_min / w_max (both when the weights are equal). */
        int upd_e = 1, upd_g = 1;
        if (we != wg) {
            int heavier_moves = u_w < w_min / w_max;
            if (we > wg)
                upd_e = heavier_moves;
            else
                upd_g = heavier_moves;
        }
        if (upd_e)
            for (int d = 0; d < 3; ++d) store_val(dtype, E[d], ie, p1[d]);
        if (upd_g)
            for (int d = 0; d < 3; ++d) store_val(dtype, G[d], ig, k1[d]);
    }
}

/* Offsets must start at 0, be non-decreasing, and end at the particle count. */
static int check_offsets(const int64_t* off, int64_t n_cells, int64_t n)
{
    if (off[0] != 0 || off[n_cells] != n) return 0;
    for (int64_t c = 0; c < n_cells; ++c)
        if (off[c + 1] < off[c]) return 0;
    return 1;
}

/*
 * One Compton step over every cell (cells == NULL) or over the listed cells.
 * dtype: 0 = float32 storage, 1 = float64 storage.  Arrays are updated in
 * place.  Optional per-electron diagnostics (length ne, indexed by electron):
 * P, the uniform u_c, x and the partner photon index of the electron's pair.
 * mu_given (optional, length ne, indexed by electron): cos(theta) to use for
 * the pair of that electron when it collides, NaN for the plain sampler.
 * Returns 0, or 2 when the offsets are not a valid cell layout (nothing is
 * modified then), or 1 for other invalid arguments.
 */
int oracle_compton_step(int dtype, void* ex, void* ey, void* ez, void* ew, int64_t ne, void* gx, void* gy,
                        void* gz, void* gw, int64_t ng, const int64_t* cell_off_e, const int64_t* cell_off_g,
                        int64_t n_cells, const int64_t* cells, int64_t n_sel, double dt, double density_norm,
                        uint64_t seed, uint64_t step, oracle_stats* stats, double* diag_P, double* diag_u,
                        double* diag_x, int64_t* diag_partner, const double* mu_given)
{
    if (dtype != 0 && dtype != 1) return 1;
    if (n_cells < 0 || ne < 0 || ng < 0) return 1;
    if (!(dt > 0.0) || !isfinite(dt) || !(density_norm >= 0.0) || !isfinite(density_norm)) return 1;
    if (!check_offsets(cell_off_e, n_cells, ne) || !check_offsets(cell_off_g, n_cells, ng)) return 2;
    int64_t n_work = cells ? n_sel : n_cells;
    for (int64_t j = 0; cells && j < n_sel; ++j)
        if (cells[j] < 0 || cells[j] >= n_cells) return 1;
    void* E[4] = {ex, ey, ez, ew};
    void* G[4] = {gx, gy, gz, gw};
    cell_tally* tallies = (cell_tally*)calloc((size_t)(n_work > 0 ? n_work : 1), sizeof(cell_tally));
    if (!tallies) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n_work; ++j) {
        int64_t c = cells ? cells[j] : j;
        process_cell(dtype, E, G, c, cell_off_e[c], cell_off_e[c + 1] - cell_off_e[c], cell_off_g[c],
                     cell_off_g[c + 1] - cell_off_g[c], dt, density_norm, seed, step, &tallies[j], diag_P,
                     diag_u, diag_x, diag_partner, mu_given);
    }
    oracle_stats s;
    memset(&s, 0, sizeof(s));
    for (int64_t j = 0; j < n_work; ++j) {
        s.n_pairs += tallies[j].n_pairs;
        s.n_collided += tallies[j].n_collided;
        s.n_clipped += tallies[j].n_clipped;
        s.n_invalid += tallies[j].n_invalid;
        s.sum_prob += tallies[j].sum_prob;
        s.energy_before += tallies[j].energy_before;
        s.energy_after += tallies[j].energy_after;
    }
    free(tallies);
    if (stats) *stats = s;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* No-time-counter candidate selection (Sec. 3.1: the NTC method of Bird      */
/* shortens each cell's pair list; the probability of Sec. 3.2).              */
/* ------------------------------------------------------------------------- */
/*
 * Readings (the paper names the method and its bound only):
 *   - The interaction probability of one electron-photon pair over the step is
 *     P = dt n w_max s(x) flux (n = density_norm, w_max the larger of the two
 *     weights); summed over all N_e N_g pairs of a cell it is the expected
 *     number of collisions.  Since s <= 1 and flux <= 2, P never exceeds the
 *     cell's bound P_max = 2 dt n W, W the largest valid weight among the
 *     cell's particles (the paper's P_max with sigma_T c folded into n).
 *   - The cell draws N_cand = N_e N_g P_max candidates, rounded
 *     stochastically (floor, plus one with the fractional part's
 *     probability), each an electron and a photon picked uniformly with
 *     replacement, accepted with probability P / P_max.
 *   - Candidates are taken in order, each one seeing the momenta the earlier
 *     collisions of its cell left: Bird's sequential scheme.
 * Random numbers (Philox4x32-10, counter as above): the count from
 * draw(cell, COUNT); candidate l of cell c uses the index (c << 32) | l for
 * PICK (electron: (r0 N_e) >> 32, photon: (r1 N_g) >> 32, acceptance uniform
 * from r2, r3), SCATTER (u_mu, u_phi) and WEIGHT (the weight rule's uniform).
 */
static double cell_max_weight(int dtype, void* const E[4], void* const G[4], int64_t e0, int64_t ne, int64_t g0,
                              int64_t ng)
{
    double w = 0.0;
    for (int64_t i = 0; i < ne; ++i) {
        double v = load_val(dtype, E[3], e0 + i);
        if (isfinite(v) && v > w) w = v;
    }
    for (int64_t i = 0; i < ng; ++i) {
        double v = load_val(dtype, G[3], g0 + i);
        if (isfinite(v) && v > w) w = v;
    }
    return w;
}

/* Candidate count of one cell; -1 when it would reach 2^31. */
static int64_t ntc_cell_count(int dtype, void* const E[4], void* const G[4], int64_t c, int64_t e0, int64_t ne,
                              int64_t g0, int64_t ng, double dt, double density_norm, uint64_t seed, uint64_t step,
                              double* p_max_out)
{
    *p_max_out = 0.0;
    if (ne == 0 || ng == 0) return 0;
    double p_max = 2.0 * dt * density_norm * cell_max_weight(dtype, E, G, e0, ne, g0, ng);
    *p_max_out = p_max;
    double n_exp = (double)ne * (double)ng * p_max;
    if (!(n_exp < 2147483647.0)) return -1;
    double fl = floor(n_exp);
    uint32_t r[4];
    draw(seed, (uint64_t)c, step, PURPOSE_NTC_COUNT, r);
    return (int64_t)fl + (oracle_uniform53(r[0], r[1]) < n_exp - fl ? 1 : 0);
}

/* Candidate counts of every cell (-1 for a cell whose count would reach
 * 2^31).  Returns 0, or 2 for an invalid layout, 1 for other bad arguments. */
int oracle_ntc_counts(int dtype, void* ex, void* ey, void* ez, void* ew, int64_t ne, void* gx, void* gy, void* gz,
                      void* gw, int64_t ng, const int64_t* cell_off_e, const int64_t* cell_off_g, int64_t n_cells,
                      double dt, double density_norm, uint64_t seed, uint64_t step, int64_t* counts)
{
    if (dtype != 0 && dtype != 1) return 1;
    if (n_cells < 0 || ne < 0 || ng < 0) return 1;
    if (!(dt > 0.0) || !isfinite(dt) || !(density_norm >= 0.0) || !isfinite(density_norm)) return 1;
    if (!check_offsets(cell_off_e, n_cells, ne) || !check_offsets(cell_off_g, n_cells, ng)) return 2;
    void* E[4] = {ex, ey, ez, ew};
    void* G[4] = {gx, gy, gz, gw};
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cells; ++c) {
        double pm;
        counts[c] = ntc_cell_count(dtype, E, G, c, cell_off_e[c], cell_off_e[c + 1] - cell_off_e[c], cell_off_g[c],
                                   cell_off_g[c + 1] - cell_off_g[c], dt, density_norm, seed, step, &pm);
    }
    return 0;
}

/* Process the candidates of one cell in order.  Optional per-candidate
 * diagnostics at base (the cell's first candidate number): electron and
 * photon index, P / P_max and the acceptance uniform. */
static void ntc_cell(int dtype, void* const E[4], void* const G[4], int64_t c, int64_t e0, int64_t ne, int64_t g0,
                     int64_t ng, double dt, double density_norm, uint64_t seed, uint64_t step, int64_t n_cand,
                     double p_max, cell_tally* t, int64_t base, int64_t* d_ie, int64_t* d_ig, double* d_ratio,
                     double* d_u)
{
    for (int64_t l = 0; l < n_cand; ++l) {
        uint64_t idx = ((uint64_t)c << 32) | (uint64_t)l;
        uint32_t r[4];
        draw(seed, idx, step, PURPOSE_NTC_PICK, r);
        int64_t ie = e0 + (int64_t)(((uint64_t)r[0] * (uint64_t)ne) >> 32);
        int64_t ig = g0 + (int64_t)(((uint64_t)r[1] * (uint64_t)ng) >> 32);
        double u_c = oracle_uniform53(r[2], r[3]);
        t->n_pairs++;
        if (d_ie) {
            d_ie[base + l] = ie;
            d_ig[base + l] = ig;
            d_ratio[base + l] = -1.0;
            d_u[base + l] = u_c;
        }
        double p[3] = {load_val(dtype, E[0], ie), load_val(dtype, E[1], ie), load_val(dtype, E[2], ie)};
        double k[3] = {load_val(dtype, G[0], ig), load_val(dtype, G[1], ig), load_val(dtype, G[2], ig)};
        double we = load_val(dtype, E[3], ie), wg = load_val(dtype, G[3], ig);
        if (!finite_nonneg_pair(p, we, k, wg)) {
            t->n_invalid++;
            continue;
        }
        double x, flux;
        oracle_pair_invariants(p, k, &x, &flux);
        double w_max = we > wg ? we : wg, w_min = we > wg ? wg : we;
        double P = (x > 0.0) ? dt * density_norm * w_max * oracle_sigma_ratio(x) * flux : 0.0;
        double ratio = P / p_max;
        if (ratio > 1.0) t->n_clipped++;
        t->sum_prob += ratio;
        if (d_ratio) d_ratio[base + l] = ratio;
        if (!(u_c < ratio)) continue;
        t->n_collided++;
        uint32_t s[4];
        draw(seed, idx, step, PURPOSE_NTC_SCATTER, s);
        double v = oracle_angle_icdf_v(oracle_uniform53(s[0], s[1]), x);
        double p1[3], k1[3], eb, ea;
        scatter_event_v(p, k, (quad)v, oracle_uniform53(s[2], s[3]), p1, k1, &eb, &ea);
        t->energy_before += eb;
        t->energy_after += ea;
        int upd_e = 1, upd_g = 1;
        if (we != wg) {
            uint32_t q[4];
            draw(seed, idx, step, PURPOSE_NTC_WEIGHT, q);
            int heavier_moves = oracle_uniform53(q[0], q[1]) < w_min / w_max;
            if (we > wg)
                upd_e = heavier_moves;
            else
                upd_g = heavier_moves;
        }
        if (upd_e)
            for (int d = 0; d < 3; ++d) store_val(dtype, E[d], ie, p1[d]);
        if (upd_g)
            for (int d = 0; d < 3; ++d) store_val(dtype, G[d], ig, k1[d]);
    }
}

/*
 * One no-time-counter step over every cell, in place.  stats as for the
 * pairing step, with n_pairs = candidates, n_clipped = candidates whose
 * P / P_max exceeded 1 (never, by the bound) and sum_prob = the sum of
 * P / P_max over valid candidates (the expected collision count).  Optional
 * per-candidate diagnostics (length = total candidates, cell by cell): see
 * ntc_cell.  Returns 0, 2 for an invalid layout, 3 when a cell's or the
 * step's candidate count would reach 2^31, 1 for other bad arguments.
 */
int oracle_ntc_step(int dtype, void* ex, void* ey, void* ez, void* ew, int64_t ne, void* gx, void* gy, void* gz,
                    void* gw, int64_t ng, const int64_t* cell_off_e, const int64_t* cell_off_g, int64_t n_cells,
                    double dt, double density_norm, uint64_t seed, uint64_t step, oracle_stats* stats,
                    int64_t* d_ie, int64_t* d_ig, double* d_ratio, double* d_u)
{
    if (dtype != 0 && dtype != 1) return 1;
    if (n_cells < 0 || ne < 0 || ng < 0) return 1;
    if (!(dt > 0.0) || !isfinite(dt) || !(density_norm >= 0.0) || !isfinite(density_norm)) return 1;
    if (!check_offsets(cell_off_e, n_cells, ne) || !check_offsets(cell_off_g, n_cells, ng)) return 2;
    void* E[4] = {ex, ey, ez, ew};
    void* G[4] = {gx, gy, gz, gw};
    int64_t* counts = (int64_t*)calloc((size_t)(n_cells + 1), sizeof(int64_t));
    double* p_max = (double*)calloc((size_t)(n_cells + 1), sizeof(double));
    cell_tally* tallies = (cell_tally*)calloc((size_t)(n_cells > 0 ? n_cells : 1), sizeof(cell_tally));
    if (!counts || !p_max || !tallies) {
        free(counts);
        free(p_max);
        free(tallies);
        return 1;
    }
    /* every count first (the weights do not change during the step) */
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n_cells; ++c)
        counts[c] = ntc_cell_count(dtype, E, G, c, cell_off_e[c], cell_off_e[c + 1] - cell_off_e[c], cell_off_g[c],
                                   cell_off_g[c + 1] - cell_off_g[c], dt, density_norm, seed, step, &p_max[c]);
    int64_t total = 0;
    int bad = 0;
    for (int64_t c = 0; c < n_cells; ++c) {
        if (counts[c] < 0) bad = 1;
        total += counts[c] < 0 ? 0 : counts[c];
    }
    if (bad || total >= 2147483647) {
        free(counts);
        free(p_max);
        free(tallies);
        return 3;
    }
    int64_t* base = (int64_t*)calloc((size_t)(n_cells + 1), sizeof(int64_t));
    for (int64_t c = 0; c < n_cells; ++c) base[c + 1] = base[c] + counts[c];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t c = 0; c < n_cells; ++c)
        ntc_cell(dtype, E, G, c, cell_off_e[c], cell_off_e[c + 1] - cell_off_e[c], cell_off_g[c],
                 cell_off_g[c + 1] - cell_off_g[c], dt, density_norm, seed, step, counts[c], p_max[c], &tallies[c],
                 base[c], d_ie, d_ig, d_ratio, d_u);
    oracle_stats s;
    memset(&s, 0, sizeof(s));
    for (int64_t c = 0; c < n_cells; ++c) {
        s.n_pairs += tallies[c].n_pairs;
        s.n_collided += tallies[c].n_collided;
        s.n_clipped += tallies[c].n_clipped;
        s.n_invalid += tallies[c].n_invalid;
        s.sum_prob += tallies[c].sum_prob;
        s.energy_before += tallies[c].energy_before;
        s.energy_after += tallies[c].energy_after;
    }
    free(counts);
    free(p_max);
    free(tallies);
    free(base);
    if (stats) *stats = s;
    return 0;
}

/* Number of OpenMP threads the oracle runs with (1 without OpenMP). */
int oracle_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
