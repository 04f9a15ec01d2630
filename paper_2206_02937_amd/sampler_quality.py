"""Distance between the network sampler's and the plain sampler's output
distributions (the acceptance measure of the learned sampler).

* ks_distance: two-sample Kolmogorov-Smirnov statistic sup |F_a - F_b| of
  two samples (here: cos(theta) or the energy ratio from the network and from
  the plain sampler on the same (x, u) inputs).
* plasma_inputs: (x, u) pairs whose x follows the rest-frame photon energy of
  a plasma's electron-photon pairs (the invariant P.K in units of m_e c^2,
  evaluated by the library, cs_pair_x), pairing randomly drawn electrons with
  randomly drawn photons (the momenta are drawn independently, so any pairing
  gives the same distribution).
* per_x_distance: the deterministic D(x) at fixed x with stratified
  u_k = (k + 1/2) / m: the plain sampler's outputs are the exact quantiles of
  the angular distribution there, so D(x) is the sup distance of the
  network's conditional CDF from the exact one (up to 1/m).
"""
import numpy as np


def ks_distance(a, b):
    """Two-sample KS statistic of 1-D samples a and b."""
    a = np.sort(np.asarray(a, dtype=np.float64).ravel())
    b = np.sort(np.asarray(b, dtype=np.float64).ravel())
    if a.size == 0 or b.size == 0:
        raise ValueError("empty sample")
    t = np.concatenate([a, b])
    fa = np.searchsorted(a, t, side="right") / a.size
    fb = np.searchsorted(b, t, side="right") / b.size
    return float(np.max(np.abs(fa - fb)))


def plasma_inputs(ctx, p, n, seed=0):
    """n (x, u) pairs drawn from the pairs of plasma p (x as float64 numpy,
    computed on the device by the library; u uniform)."""
    import torch

    rng = np.random.default_rng([seed, 11])
    m = min(p.e["x"].size, p.g["x"].size)
    idx = rng.integers(0, m, size=n)
    e = {c: torch.from_numpy(np.ascontiguousarray(p.e[c][idx])).cuda() for c in "xyzw"}
    g = {c: torch.from_numpy(np.ascontiguousarray(p.g[c][idx])).cuda() for c in "xyzw"}
    x = ctx.pair_x(e, g).cpu().numpy()
    return x, rng.random(n)


def stratified_u(m):
    return (np.arange(m) + 0.5) / m


def log_spaced_x(n=61, x_min=1e-4, x_max=1e2):
    return np.logspace(np.log10(x_min), np.log10(x_max), n)
