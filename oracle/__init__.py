"""FP64 CPU oracle of the Compton-scattering Monte-Carlo step and of the
sampler MLP -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_2206_02937_amd``) and never imports it.

This module is a thin ctypes wrapper over ``liboracle.so`` (plain C, see
``compton_oracle.c``); the MLP oracle lives in ``mlp_oracle.py`` (numpy FP64)
the cell-binning oracle in ``binning.py`` and the probability-network
oracle in ``pnet_oracle.py``.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# CS_ORACLE_LIB selects another build of the same source (the sanitized one)
_LIB_PATH = os.environ.get("CS_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")
_lib = None


class OracleStats(C.Structure):
    _fields_ = [
        ("n_pairs", C.c_int64),
        ("n_collided", C.c_int64),
        ("n_clipped", C.c_int64),
        ("n_invalid", C.c_int64),
        ("sum_prob", C.c_double),
        ("energy_before", C.c_double),
        ("energy_after", C.c_double),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


def lib():
    """Load liboracle.so, building it with gcc first if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    L = C.CDLL(_LIB_PATH)
    d, i64, u32, u64, vp = C.c_double, C.c_int64, C.c_uint32, C.c_uint64, C.c_void_p
    dp = C.POINTER(C.c_double)
    L.oracle_philox4x32_10.argtypes = [C.POINTER(u32), C.POINTER(u32), C.POINTER(u32)]
    L.oracle_philox4x32_10.restype = None
    L.oracle_uniform53.argtypes = [u32, u32]
    L.oracle_uniform53.restype = d
    L.oracle_shuffle_index.argtypes = [u64, u64, u64, u64, u64]
    L.oracle_shuffle_index.restype = u64
    L.oracle_shuffle_all.argtypes = [u64, u64, u64, u64, vp]
    L.oracle_shuffle_all.restype = None
    L.oracle_sigma_ratio.argtypes = [d]
    L.oracle_sigma_ratio.restype = d
    L.oracle_angle_pdf.argtypes = [d, d]
    L.oracle_angle_pdf.restype = d
    L.oracle_angle_cdf.argtypes = [d, d]
    L.oracle_angle_cdf.restype = d
    L.oracle_angle_icdf.argtypes = [d, d]
    L.oracle_angle_icdf.restype = d
    L.oracle_angle_icdf_v.argtypes = [d, d]
    L.oracle_angle_icdf_v.restype = d
    L.oracle_angle_cdf_v.argtypes = [d, d]
    L.oracle_angle_cdf_v.restype = d
    L.oracle_sample_plain.argtypes = [dp, dp, i64, dp, dp]
    L.oracle_sample_plain.restype = None
    L.oracle_pair_invariants.argtypes = [dp, dp, dp, dp]
    L.oracle_pair_invariants.restype = None
    L.oracle_scatter_event.argtypes = [dp, dp, d, d, dp, dp, dp, dp]
    L.oracle_scatter_event.restype = None
    L.oracle_compton_step.argtypes = [
        C.c_int, vp, vp, vp, vp, i64, vp, vp, vp, vp, i64, vp, vp, i64, vp, i64,
        d, d, u64, u64, C.POINTER(OracleStats), vp, vp, vp, vp, vp,
    ]
    L.oracle_compton_step.restype = C.c_int
    L.oracle_ntc_counts.argtypes = [C.c_int] + [vp] * 4 + [i64] + [vp] * 4 + [i64, vp, vp, i64, d, d, u64, u64, vp]
    L.oracle_ntc_counts.restype = C.c_int
    L.oracle_ntc_step.argtypes = ([C.c_int] + [vp] * 4 + [i64] + [vp] * 4 + [i64, vp, vp, i64, d, d, u64, u64,
                                  C.POINTER(OracleStats)] + [vp] * 4)
    L.oracle_ntc_step.restype = C.c_int
    L.oracle_scatter_uniforms.argtypes = [vp, i64, u64, u64, dp, dp]
    L.oracle_scatter_uniforms.restype = None
    L.oracle_num_threads.argtypes = []
    L.oracle_num_threads.restype = C.c_int
    L.oracle_set_num_threads.argtypes = [C.c_int]
    L.oracle_set_num_threads.restype = None
    _lib = L
    return L


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


# ----------------------------------------------------------------------------
# scalar helpers
# ----------------------------------------------------------------------------
def philox4x32_10(ctr, key):
    """Philox4x32-10 block: ctr = 4 words, key = 2 words -> 4 words."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().oracle_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniform53(a, b):
    return lib().oracle_uniform53(int(a) & 0xFFFFFFFF, int(b) & 0xFFFFFFFF)


def shuffle_index(i, M, seed, cell, step):
    """Image of i under the in-cell pairing bijection of [0, M)."""
    return int(lib().oracle_shuffle_index(int(i), int(M), int(seed), int(cell), int(step)))


def shuffle_all(M, seed, cell, step):
    """The whole in-cell pairing permutation of [0, M) as an int64 array."""
    out = np.empty(int(M), dtype=np.int64)
    lib().oracle_shuffle_all(int(M), int(seed), int(cell), int(step), out.ctypes.data)
    return out


def sigma_ratio(x):
    """sigma_KN(x) / sigma_T (vectorised over numpy input)."""
    f = lib().oracle_sigma_ratio
    if np.isscalar(x):
        return f(float(x))
    x = np.asarray(x, dtype=np.float64)
    return np.array([f(float(v)) for v in x.ravel()]).reshape(x.shape)


def angle_pdf(mu, x):
    return lib().oracle_angle_pdf(float(mu), float(x))


def angle_cdf(mu, x):
    f = lib().oracle_angle_cdf
    if np.isscalar(mu):
        return f(float(mu), float(x))
    mu = np.asarray(mu, dtype=np.float64)
    return np.array([f(float(m), float(x)) for m in mu.ravel()]).reshape(mu.shape)


def angle_icdf(u, x):
    return lib().oracle_angle_icdf(float(u), float(x))


def angle_icdf_v(u, x):
    """v = 1 - mu solving F(1 - v; x) = u (relative precision for forward scatters)."""
    return lib().oracle_angle_icdf_v(float(u), float(x))


def angle_cdf_v(v, x):
    return lib().oracle_angle_cdf_v(float(v), float(x))


def sample_plain(x, u):
    """Plain inverse-CDF sampler: (x, u) -> (mu, eps'/eps), FP64."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert x.shape == u.shape
    mu = np.empty_like(x)
    r = np.empty_like(x)
    lib().oracle_sample_plain(_dptr(x), _dptr(u), x.size, _dptr(mu), _dptr(r))
    return mu, r


def pair_invariants(p, k):
    """(x, 1 - beta.k_hat) for one electron momentum p and photon momentum k."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    x = C.c_double()
    fl = C.c_double()
    lib().oracle_pair_invariants(_dptr(p), _dptr(k), C.byref(x), C.byref(fl))
    return x.value, fl.value


def scatter_event(p, k, mu, u_phi):
    """Resolve one collision: returns (p1, k1, energy_before, energy_after)."""
    p = np.ascontiguousarray(p, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    p1 = np.empty(3)
    k1 = np.empty(3)
    eb = C.c_double()
    ea = C.c_double()
    lib().oracle_scatter_event(_dptr(p), _dptr(k), float(mu), float(u_phi), _dptr(p1), _dptr(k1),
                               C.byref(eb), C.byref(ea))
    return p1, k1, eb.value, ea.value


def num_threads():
    return int(lib().oracle_num_threads())


def set_num_threads(n):
    lib().oracle_set_num_threads(int(n))


# ----------------------------------------------------------------------------
# the step
# ----------------------------------------------------------------------------
class OracleError(RuntimeError):
    pass


def scatter_uniforms(idx, seed, step):
    """(u_mu, u_phi) of the collisions of the pairs whose electrons are idx."""
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    u_mu = np.empty(idx.size)
    u_phi = np.empty(idx.size)
    lib().oracle_scatter_uniforms(idx.ctypes.data, idx.size, int(seed), int(step), _dptr(u_mu), _dptr(u_phi))
    return u_mu, u_phi


def compton_step(e, g, off_e, off_g, dt, density_norm, seed, step, cells=None, diagnostics=False, mu_given=None):
    """One Compton step, in place, on host numpy arrays.

    ``e`` / ``g``: dicts with keys x, y, z, w (same dtype, float32 or float64,
    C-contiguous); ``off_e`` / ``off_g``: int64 cell offsets (n_cells + 1).
    ``cells``: optional int64 array of cell ids to process (others untouched).
    ``mu_given``: optional float64 array over electrons: cos(theta) to use
    when that electron's pair collides (NaN: the plain sampler draws it).
    Returns the stats dict, plus per-electron diagnostics (P, u, x, partner)
    when ``diagnostics`` is true.
    """
    dtype = e["x"].dtype
    if dtype == np.float64:
        code = 1
    elif dtype == np.float32:
        code = 0
    else:
        raise OracleError("storage dtype must be float32 or float64")
    arrs = [e[c] for c in "xyzw"] + [g[c] for c in "xyzw"]
    for a in arrs:
        if a.dtype != dtype or not a.flags.c_contiguous:
            raise OracleError("species arrays must share one dtype and be contiguous")
    ne = e["x"].size
    ng = g["x"].size
    off_e = np.ascontiguousarray(off_e, dtype=np.int64)
    off_g = np.ascontiguousarray(off_g, dtype=np.int64)
    n_cells = off_e.size - 1
    if off_g.size != n_cells + 1:
        raise OracleError("offset arrays differ in length")
    sel = None
    if cells is not None:
        sel = np.ascontiguousarray(cells, dtype=np.int64)
    st = OracleStats()
    diag = None
    ptrs = [None] * 4
    if diagnostics:
        diag = {
            "P": np.full(ne, -1.0),
            "u": np.full(ne, -1.0),
            "x": np.full(ne, -1.0),
            "partner": np.full(ne, -1, dtype=np.int64),
        }
        ptrs = [diag[k].ctypes.data for k in ("P", "u", "x", "partner")]
    mg = None
    if mu_given is not None:
        mg = np.ascontiguousarray(mu_given, dtype=np.float64)
        if mg.size != ne:
            raise OracleError("mu_given must have one entry per electron")
    rc = lib().oracle_compton_step(
        code, *[a.ctypes.data for a in arrs[:4]], ne, *[a.ctypes.data for a in arrs[4:]], ng,
        off_e.ctypes.data, off_g.ctypes.data, n_cells,
        sel.ctypes.data if sel is not None else None, sel.size if sel is not None else 0,
        float(dt), float(density_norm), int(seed), int(step), C.byref(st), *ptrs,
        mg.ctypes.data if mg is not None else None)
    if rc == 2:
        raise OracleError("cell offsets are not a valid layout")
    if rc != 0:
        raise OracleError(f"invalid argument (code {rc})")
    out = st.as_dict()
    if diagnostics:
        return out, diag
    return out


# the no-time-counter step
# ----------------------------------------------------------------------------
def _species_args(e, g, off_e, off_g):
    dtype = e["x"].dtype
    if dtype not in (np.float32, np.float64):
        raise OracleError("storage dtype must be float32 or float64")
    arrs = [e[c] for c in "xyzw"] + [g[c] for c in "xyzw"]
    for a in arrs:
        if a.dtype != dtype or not a.flags.c_contiguous:
            raise OracleError("species arrays must share one dtype and be contiguous")
    off_e = np.ascontiguousarray(off_e, dtype=np.int64)
    off_g = np.ascontiguousarray(off_g, dtype=np.int64)
    if off_g.size != off_e.size:
        raise OracleError("offset arrays differ in length")
    code = 1 if dtype == np.float64 else 0
    head = [code, *[a.ctypes.data for a in arrs[:4]], e["x"].size, *[a.ctypes.data for a in arrs[4:]], g["x"].size,
            off_e.ctypes.data, off_g.ctypes.data, off_e.size - 1]
    return head, (off_e, off_g)


def _ntc_rc(rc):
    if rc == 2:
        raise OracleError("cell offsets are not a valid layout")
    if rc == 3:
        raise OracleError("candidate count reaches 2^31")
    if rc != 0:
        raise OracleError(f"invalid argument (code {rc})")


def ntc_counts(e, g, off_e, off_g, dt, density_norm, seed, step):
    """Candidate count of every cell under no-time-counter selection
    (N_e N_g P_max rounded stochastically; -1 where it would reach 2^31)."""
    head, keep = _species_args(e, g, off_e, off_g)
    counts = np.zeros(max(head[-1], 1), dtype=np.int64)
    _ntc_rc(lib().oracle_ntc_counts(*head, float(dt), float(density_norm), int(seed), int(step), counts.ctypes.data))
    return counts[:head[-1]]


def ntc_step(e, g, off_e, off_g, dt, density_norm, seed, step, diagnostics=False):
    """One no-time-counter Compton step (Bird's candidate selection, each
    cell's candidates taken in order), in place on host numpy arrays (the
    layout of compton_step).  Returns the stats dict (n_pairs = candidates,
    sum_prob = sum of P / P_max), plus with ``diagnostics`` per-candidate
    arrays ie, ig, ratio (P / P_max, -1 for invalid pairs), u (acceptance
    uniform) and cell, candidates ordered cell by cell."""
    head, keep = _species_args(e, g, off_e, off_g)
    ptrs = [None] * 4
    diag = None
    if diagnostics:
        counts = ntc_counts(e, g, off_e, off_g, dt, density_norm, seed, step)
        if np.any(counts < 0):
            raise OracleError("candidate count reaches 2^31")
        n = int(counts.sum())
        diag = {"ie": np.zeros(max(n, 1), dtype=np.int64), "ig": np.zeros(max(n, 1), dtype=np.int64),
                "ratio": np.zeros(max(n, 1)), "u": np.zeros(max(n, 1))}
        ptrs = [diag[k].ctypes.data for k in ("ie", "ig", "ratio", "u")]
    st = OracleStats()
    _ntc_rc(lib().oracle_ntc_step(*head, float(dt), float(density_norm), int(seed), int(step), C.byref(st), *ptrs))
    out = st.as_dict()
    if diagnostics:
        diag = {k: v[:n] for k, v in diag.items()}
        diag["cell"] = np.repeat(np.arange(counts.size, dtype=np.int64), counts)
        return out, diag
    return out
