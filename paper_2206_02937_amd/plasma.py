"""Seeded synthetic plasmas and sampler inputs shaped like the paper's workloads.

This module holds input generators only: momentum distributions, cell layouts
and random (x, u) sets.  It contains none of the scattering arithmetic, and
both the GPU library's tests and the CPU oracle take their inputs from here.

Units: momenta in m_e c, photon energies in m_e c^2.  Particles are stored as
structure-of-arrays per species (x, y, z momentum components and the
macro-particle weight w), sorted by collision cell, with int64 CSR offsets of
length n_cells + 1 per species.

The paper's own workloads (Sec. 3.2, Sec. 3.3) are OSIRIS runs whose data is
not available; these generators stand in for them with the distributions
named in the workload descriptions below.
"""
from dataclasses import dataclass, field

import numpy as np

# dt values: chosen so that the mean collision probability of the initial
# state is 0.05; each was computed once over the seeded initial plasma with
# the FP64 reference cross-section (script: tests/golden/derive_dt.py).
DT_SINGLE_CELL = 0.051594173859536484
DT_GRID = 0.05284409308615999
DT_UNEVEN = 0.019678706187464638
DT_POWERLAW = 0.050011220840244015


@dataclass
class Plasma:
    name: str
    e: dict            # electrons: x, y, z, w
    g: dict            # photons:   x, y, z, w
    off_e: np.ndarray  # int64, n_cells + 1
    off_g: np.ndarray
    dt: float
    density_norm: float
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return self.off_e.size - 1

    @property
    def n_pairs(self):
        ne = np.diff(self.off_e)
        ng = np.diff(self.off_g)
        return int(np.minimum(ne, ng).sum())

    def copy(self):
        return Plasma(self.name, {k: v.copy() for k, v in self.e.items()},
                      {k: v.copy() for k, v in self.g.items()}, self.off_e.copy(), self.off_g.copy(),
                      self.dt, self.density_norm, self.seed, dict(self.meta))

    def astype(self, dtype):
        out = self.copy()
        out.e = {k: np.ascontiguousarray(v, dtype=dtype) for k, v in out.e.items()}
        out.g = {k: np.ascontiguousarray(v, dtype=dtype) for k, v in out.g.items()}
        return out

    def nbytes(self):
        return sum(v.nbytes for v in self.e.values()) + sum(v.nbytes for v in self.g.values())


# ----------------------------------------------------------------------------
# distributions
# ----------------------------------------------------------------------------
def isotropic(rng, n):
    """Unit vectors uniform on the sphere: cos = 2u - 1, phi = 2 pi u."""
    c = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * np.pi * rng.random(n)
    s = np.sqrt(np.maximum(0.0, 1.0 - c * c))
    return s * np.cos(phi), s * np.sin(phi), c


def maxwell_juttner_momentum(rng, n, theta):
    """|p| drawn from the Maxwell-Juttner distribution
    f(p) ~ p^2 exp(-gamma/theta), by Sobol's rejection method as reviewed by
    Zenitani (2015, Phys. Plasmas 22, 042116): with X1..X4 uniform on (0, 1],
    u = -theta ln(X1 X2 X3), eta = -theta ln(X1 X2 X3 X4); accept p = u when
    eta^2 - u^2 > 1."""
    out = np.empty(0)
    while out.size < n:
        m = int((n - out.size) * 2.2) + 64
        X = 1.0 - rng.random((4, m))  # (0, 1]
        u = -theta * np.log(X[0] * X[1] * X[2])
        eta = -theta * np.log(X[0] * X[1] * X[2] * X[3])
        out = np.concatenate([out, u[eta * eta - u * u > 1.0]])
    return out[:n]


def power_law_gamma(rng, n, g_min=1.0, g_max=1e4):
    """gamma with density ~ gamma^-2 on [g_min, g_max] (inverse CDF)."""
    u = rng.random(n)
    a, b = 1.0 / g_min, 1.0 / g_max
    return 1.0 / (a - u * (a - b))


def blackbody_energy(rng, n, T):
    """Photon energies from a Planck spectrum f(eps) ~ eps^2 / (exp(eps/T) - 1):
    eps^2 / (e^y - 1) = sum_n eps^2 e^{-n y}, so pick n with weight n^-3 and
    draw y from a Gamma(3) law scaled by 1/n."""
    n_max = 100000
    k = np.arange(1, n_max + 1, dtype=np.float64)
    w = k ** -3.0
    w /= w.sum()
    nn = rng.choice(k, size=n, p=w)
    y = rng.gamma(3.0, 1.0, size=n) / nn
    return T * y


def log_uniform(rng, n, lo, hi):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=n))


def _species(px, py, pz, w, dtype):
    return {"x": np.ascontiguousarray(px, dtype=dtype), "y": np.ascontiguousarray(py, dtype=dtype),
            "z": np.ascontiguousarray(pz, dtype=dtype), "w": np.ascontiguousarray(w, dtype=dtype)}


def _electrons_from_pmag(rng, pmag, dtype):
    ux, uy, uz = isotropic(rng, pmag.size)
    return _species(pmag * ux, pmag * uy, pmag * uz, np.ones(pmag.size), dtype)


def _photons_from_energy(rng, eps, dtype):
    ux, uy, uz = isotropic(rng, eps.size)
    return _species(eps * ux, eps * uy, eps * uz, np.ones(eps.size), dtype)


def _uniform_offsets(n_cells, per_cell):
    return np.arange(n_cells + 1, dtype=np.int64) * per_cell


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def single_cell(seed=0, n=16384, dtype=np.float64):
    """0D single cell: n electrons with gamma = 10 and n photons with
    eps = 1e-3, both isotropic, unit weights; FP64 storage."""
    rng = np.random.default_rng([seed, 1])
    pmag = np.full(n, np.sqrt(99.0))
    e = _electrons_from_pmag(rng, pmag, dtype)
    g = _photons_from_energy(rng, np.full(n, 1e-3), dtype)
    off = np.array([0, n], dtype=np.int64)
    return Plasma("single_cell_16384_fp64", e, g, off, off.copy(), DT_SINGLE_CELL, 1.0 / n, seed,
                  {"cells": 1, "per_cell": n})


def grid(seed=0, nx=64, ny=64, per_cell=256, dtype=np.float32, theta=0.5, dt=DT_GRID):
    """2D grid of nx*ny cells with per_cell electrons and photons each:
    electrons Maxwell-Juttner at kT = theta m_e c^2, isotropic; photons
    isotropic with eps log-uniform in [1e-4, 1e-1].  FP32 storage."""
    rng = np.random.default_rng([seed, 2])
    n_cells = nx * ny
    n = n_cells * per_cell
    e = _electrons_from_pmag(rng, maxwell_juttner_momentum(rng, n, theta), dtype)
    g = _photons_from_energy(rng, log_uniform(rng, n, 1e-4, 1e-1), dtype)
    off = _uniform_offsets(n_cells, per_cell)
    return Plasma(f"grid_{nx}x{ny}x{per_cell}_fp32", e, g, off, off.copy(), dt, 1.0 / per_cell, seed,
                  {"cells": n_cells, "per_cell": per_cell})


def uneven(seed=0, side=256, mean=64, peak=20.0, area_frac=0.02, dtype=np.float32):
    """side*side cells with Poisson pair counts of mean `mean`, plus a
    Gaussian density bump of `peak` times the background at its centre,
    covering `area_frac` of the cells (radius R, Gaussian sigma R/2).
    Electron and photon counts are equal per cell; distributions as grid()."""
    rng = np.random.default_rng([seed, 4])
    R = np.sqrt(area_frac * side * side / np.pi)
    s = R / 2.0
    iy, ix = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    r2 = (ix + 0.5 - side / 2.0) ** 2 + (iy + 0.5 - side / 2.0) ** 2
    lam = np.full(side * side, float(mean))
    inside = (r2 <= R * R).ravel()
    lam[inside] = mean * (1.0 + (peak - 1.0) * np.exp(-r2.ravel()[inside] / (2.0 * s * s)))
    counts = rng.poisson(lam).astype(np.int64)
    n = int(counts.sum())
    e = _electrons_from_pmag(rng, maxwell_juttner_momentum(rng, n, 0.5), dtype)
    g = _photons_from_energy(rng, log_uniform(rng, n, 1e-4, 1e-1), dtype)
    off = np.zeros(side * side + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    return Plasma(f"uneven_{side}x{side}_poisson{mean}_bump{int(peak)}x_fp32", e, g, off, off.copy(),
                  DT_UNEVEN, 1.0 / mean, seed,
                  {"cells": side * side, "max_cell": int(counts.max()), "bump_radius": R})


def power_law(seed=0, n_cells=65536, per_cell=256, dtype=np.float32):
    """Precision stress: electrons with gamma ~ gamma^-2 on [1, 1e4],
    isotropic; photons from a blackbody at T = 1e-6 m_e c^2, isotropic."""
    rng = np.random.default_rng([seed, 5])
    n = n_cells * per_cell
    gam = power_law_gamma(rng, n)
    pmag = np.sqrt(np.maximum(gam * gam - 1.0, 0.0))
    e = _electrons_from_pmag(rng, pmag, dtype)
    g = _photons_from_energy(rng, blackbody_energy(rng, n, 1e-6), dtype)
    off = _uniform_offsets(n_cells, per_cell)
    return Plasma(f"powerlaw_{n_cells}x{per_cell}_fp32", e, g, off, off.copy(), DT_POWERLAW, 1.0 / per_cell,
                  seed, {"cells": n_cells, "per_cell": per_cell})


def sampler_inputs(n, seed=0, x_min=1e-4, x_max=1e2):
    """Sampler training / benchmark inputs: x log-uniform in [x_min, x_max],
    u uniform in [0, 1)."""
    rng = np.random.default_rng([seed, 3])
    return log_uniform(rng, n, x_min, x_max), rng.random(n)


def beam_gas(seed=0, p_e=100.0, eps=2.5, n_cells=1024, per_cell=256, dtype=np.float32, dt=1.0):
    """Inverse-Compton beam in a photon gas (the paper's Sec. 3.3 benchmark):
    in every cell per_cell electrons of momentum p_e along +z and per_cell
    photons of energy eps with isotropic directions; unit weights.  With
    density_norm = 1 / per_cell the pair probability of a step is
    dt s(x)(1 - beta . k_hat): of order 1 % for p_e = 100 and dt = 1."""
    rng = np.random.default_rng([seed, 7])
    n = n_cells * per_cell
    e = _species(np.zeros(n), np.zeros(n), np.full(n, float(p_e)), np.ones(n), dtype)
    g = _photons_from_energy(rng, np.full(n, float(eps)), dtype)
    off = _uniform_offsets(n_cells, per_cell)
    return Plasma(f"beam_gas_pe{p_e:g}_eps{eps:g}_{n_cells}x{per_cell}", e, g, off, off.copy(), dt, 1.0 / per_cell,
                  seed, {"cells": n_cells, "per_cell": per_cell, "p_e": p_e, "eps": eps})


def make(name, seed=0):
    if name == "single_cell":
        return single_cell(seed)
    if name == "grid":
        return grid(seed)
    if name == "grid_large":
        return grid(seed, nx=128, ny=128, per_cell=256)
    if name == "uneven":
        return uneven(seed)
    if name == "power_law":
        return power_law(seed)
    if name.startswith("beam_gas_"):
        return beam_gas(seed, p_e=float(name[len("beam_gas_"):]))
    raise KeyError(name)
