"""Pins of the oracle's boosts and collision kinematics: the invariant x
recomputed at 50 digits, the head-on closed form, the Compton energy-shift
formula for an electron at rest, the Compton invariant P.K = P.K1 + K.K1 of
every event (Minkowski products at 50 digits), energy and momentum
conservation, and the azimuthal symmetry of the scattered direction."""
import math

import mpmath as mp
import numpy as np
import pytest

mp.mp.dps = 50


def mink(a, b):
    """Minkowski product (E, p).(E', p') = E E' - p.p' in mpmath."""
    return a[0] * b[0] - sum(mp.mpf(float(a[i])) * mp.mpf(float(b[i])) for i in (1, 2, 3))


def four_electron(p):
    p = [mp.mpf(float(v)) for v in p]
    return [mp.sqrt(1 + sum(v * v for v in p))] + p


def four_photon(k):
    k = [mp.mpf(float(v)) for v in k]
    return [mp.sqrt(sum(v * v for v in k))] + k


def random_pairs(n, seed, gmax=100.0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        gam = math.exp(rng.uniform(0, math.log(gmax)))
        pm = math.sqrt(gam * gam - 1)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        eps = math.exp(rng.uniform(math.log(1e-5), math.log(10.0)))
        c = rng.normal(size=3)
        c /= np.linalg.norm(c)
        out.append((pm * d, eps * c, rng.random(), rng.random()))
    return out


def test_x_invariant_high_precision(orc):
    for p, k, _, _ in random_pairs(300, 1, gmax=1e4):
        x, flux = orc.pair_invariants(p, k)
        P = four_electron(p)
        K = four_photon(k)
        xr = mink(P, K)  # = gamma eps - p.k
        assert abs(x - float(xr)) <= 2e-16 * float(xr) * 4
        assert abs(flux - float(xr / (P[0] * K[0]))) <= 1e-15 * float(xr / (P[0] * K[0]))


def test_x_head_on_and_comoving():
    import oracle

    for gam in [1.5, 10.0, 1e3, 1e4]:
        pm = math.sqrt(gam * gam - 1)
        eps = 0.37
        x, flux = oracle.pair_invariants([0, 0, pm], [0, 0, -eps])
        assert abs(x - eps * (gam + pm)) <= 4e-16 * x
        assert abs(flux - (1 + pm / gam)) <= 4e-16 * flux
        x, flux = oracle.pair_invariants([0, 0, pm], [0, 0, eps])
        exact = eps / (gam + pm)  # eps (gamma - p), without cancellation
        assert abs(x - exact) <= 4e-16 * exact
    x, flux = oracle.pair_invariants([0.3, 0.1, 0.0], [0, 0, 0])
    assert x == 0.0 and flux == 0.0


def test_electron_at_rest_reduces_to_compton_formula(orc):
    rng = np.random.default_rng(5)
    for _ in range(200):
        eps = math.exp(rng.uniform(math.log(1e-4), math.log(100)))
        kd = rng.normal(size=3)
        kd /= np.linalg.norm(kd)
        k = eps * kd
        mu = rng.uniform(-1, 1)
        p1, k1, eb, ea = orc.scatter_event([0.0, 0.0, 0.0], k, mu, rng.random())
        e1 = np.linalg.norm(k1)
        # textbook: eps' = eps / (1 + eps (1 - cos theta)), cos theta = k_hat . k1_hat
        assert abs(e1 - eps / (1 + eps * (1 - mu))) <= 4e-16 * e1
        assert abs(np.dot(kd, k1) / e1 - mu) <= 2e-15
        assert np.allclose(p1, k - k1, rtol=0, atol=4e-16 * eps)


@pytest.mark.parametrize("seed", [2, 3])
def test_compton_invariant_and_conservation(orc, seed):
    for p, k, uf, up in random_pairs(150, seed, gmax=1e3):
        x, _ = orc.pair_invariants(p, k)
        mu = 2 * uf - 1
        p1, k1, eb, ea = orc.scatter_event(p, k, mu, up)
        P, K, P1, K1 = four_electron(p), four_photon(k), four_electron(p1), four_photon(k1)
        pk, pk1, kk1 = mink(P, K), mink(P, K1), mink(K, K1)
        # the outputs are rounded to doubles, so each product carries an
        # absolute error ~ ulp of its energy term E E'
        scale = P[0] * K[0] + P[0] * K1[0] + K[0] * K1[0]
        assert abs(pk - pk1 - kk1) <= 1e-15 * scale
        # energy: (gamma + eps) before equals (gamma' + eps') after
        e_before = P[0] + K[0]
        e_after = P1[0] + K1[0]
        assert abs(e_after - e_before) <= 2e-15 * e_before
        assert abs(eb - float(e_before)) <= 2e-16 * eb and abs(ea - float(e_after)) <= 4e-16 * ea
        # momentum: p1 + k1 = p + k to rounding of the outputs
        tot = np.abs(p) + np.abs(k) + np.abs(k1)
        assert np.all(np.abs(p1 + k1 - p - k) <= 2.3e-16 * tot * 2)
        # Compton shift in the rest frame: the rest-frame photon energy after
        # the event is x1 = x / (1 + x (1 - mu)) = P.K1
        assert abs(float(pk1) - x / (1 + x * (1 - mu))) <= 1e-15 * float(P[0] * K1[0])


def test_azimuth_is_uniform_about_incoming_direction(orc):
    """For a fixed rest-frame polar angle, the scattered lab directions of an
    electron at rest fill a cone around k uniformly in phi."""
    k = np.array([0.3, -0.2, 0.9])
    kd = k / np.linalg.norm(k)
    e1 = np.cross(kd, [1, 0, 0])
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(kd, e1)
    angles = []
    for u in np.linspace(0, 1, 2000, endpoint=False):
        _, k1, _, _ = orc.scatter_event([0, 0, 0], k, 0.2, u)
        d = k1 / np.linalg.norm(k1)
        angles.append(math.atan2(np.dot(d, e2), np.dot(d, e1)) % (2 * math.pi))
    a = np.sort(np.array(angles))
    gaps = np.diff(np.concatenate([a, [a[0] + 2 * math.pi]]))
    assert np.allclose(gaps, 2 * math.pi / 2000, rtol=1e-9)
