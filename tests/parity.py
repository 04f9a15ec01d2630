"""Helpers for GPU-vs-oracle parity of one Compton step.

Per-event error metric (a reading; the tolerances are the workload's 1e-12 for
FP64 storage and 1e-5 for FP32 storage):
    electrons  |p_gpu - p_ref| / gamma_ref
    photons    |k_gpu - k_ref| / eps_ref
Pairs whose acceptance is decided within rounding (|u - P| <= delta P, delta
equal to the tolerance) are "ambiguous": both particles of such a pair are
left out of the per-event comparison and counted; the count must stay small
against its expectation 2 delta sum(P).  Every particle the oracle leaves
bitwise untouched (invalid inputs included, NaN payloads and all) must be
bitwise unchanged on the GPU.  Every other particle of the compared set is
compared: a GPU value that is not finite where the oracle's is finite counts
as an infinite error, and the number compared must equal the size of the set.
"""
import numpy as np

TOL = {np.float64: 1e-12, np.float32: 1e-5}


def tolerance(dtype):
    return TOL[np.dtype(dtype).type]


def run_oracle(orc, p, state_e, state_g, step, cells=None):
    """Oracle step on a host copy of the given state; returns (after_e,
    after_g, stats, diagnostics)."""
    e = {k: v.copy() for k, v in state_e.items()}
    g = {k: v.copy() for k, v in state_g.items()}
    st, diag = orc.compton_step(e, g, p.off_e, p.off_g, p.dt, p.density_norm, p.seed, step, cells=cells,
                                diagnostics=True)
    return e, g, st, diag


def _bits(d):
    """Bit patterns of the three momentum components (n x 3 unsigned ints)."""
    cols = []
    for c in "xyz":
        a = np.ascontiguousarray(d[c])
        cols.append(a.view(np.uint64 if a.dtype.itemsize == 8 else np.uint32))
    return np.stack(cols, axis=1)


def _vec(d):
    return np.stack([d["x"], d["y"], d["z"]], axis=1).astype(np.float64)


def _event_errors(gpu, ref, scale):
    """|gpu - ref| / scale per particle; 0 where the two are bitwise equal,
    inf where the GPU value is not finite but the oracle's is (or the scale
    is not a positive finite number while the two differ)."""
    g, r = _vec(gpu), _vec(ref)
    same = np.all(_bits(gpu) == _bits(ref), axis=1)
    with np.errstate(invalid="ignore", divide="ignore", over="ignore"):
        err = np.linalg.norm(g - r, axis=1) / scale
    ok = np.isfinite(err) & np.all(np.isfinite(g), axis=1)
    err = np.where(ok, err, np.inf)
    return np.where(same, 0.0, err)


def compare(before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, diag, dtype, e_mask=None, g_mask=None):
    """Return a dict with max errors, ambiguous count and its expectation.
    e_mask / g_mask restrict the comparison to the processed particles."""
    delta = tolerance(dtype)
    ne = before_e["x"].size
    ng = before_g["x"].size
    e_mask = np.ones(ne, bool) if e_mask is None else e_mask.copy()
    g_mask = np.ones(ng, bool) if g_mask is None else g_mask.copy()
    P, u, partner = diag["P"], diag["u"], diag["partner"]
    paired = P >= 0
    amb = paired & (np.abs(u - P) <= delta * np.maximum(P, 0))
    e_mask &= ~amb
    g_mask[partner[amb]] = False

    pr, kr = _vec(ref_e), _vec(ref_g)
    with np.errstate(invalid="ignore", over="ignore"):
        gam = np.sqrt(1.0 + (pr * pr).sum(1))
        eps = np.sqrt((kr * kr).sum(1))
    # a photon of zero energy keeps its (zero) momentum: absolute error there
    err_e = _event_errors(gpu_e, ref_e, gam)
    err_g = _event_errors(gpu_g, ref_g, np.where(eps > 0, eps, 1.0))
    # untouched by the oracle (bit for bit) -> bitwise unchanged on the GPU
    same_e = np.all(_bits(ref_e) == _bits(before_e), axis=1) & e_mask
    same_g = np.all(_bits(ref_g) == _bits(before_g), axis=1) & g_mask
    bad_e = ~np.all(_bits(gpu_e)[same_e] == _bits(before_e)[same_e], axis=1)
    bad_g = ~np.all(_bits(gpu_g)[same_g] == _bits(before_g)[same_g], axis=1)
    return {
        "max_err_e": float(err_e[e_mask].max()) if e_mask.any() else 0.0,
        "max_err_g": float(err_g[g_mask].max()) if g_mask.any() else 0.0,
        "n_ambiguous": int(amb.sum()),
        "expected_ambiguous": float(2 * delta * P[paired].sum()),
        "untouched_changed": int(bad_e.sum() + bad_g.sum()),
        "n_compared_e": int(np.isfinite(err_e[e_mask]).sum()),
        "n_compared_g": int(np.isfinite(err_g[g_mask]).sum()),
        "n_expected_e": int(e_mask.sum()),
        "n_expected_g": int(g_mask.sum()),
    }


def assert_parity(res, dtype, what=""):
    tol = tolerance(dtype)
    assert res["untouched_changed"] == 0, (what, res)
    assert res["n_compared_e"] == res["n_expected_e"], (what, res)
    assert res["n_compared_g"] == res["n_expected_g"], (what, res)
    assert res["max_err_e"] <= tol, (what, res)
    assert res["max_err_g"] <= tol, (what, res)
    assert res["n_ambiguous"] <= 10 * res["expected_ambiguous"] + 3, (what, res)


def cell_masks(p, cells):
    me = np.zeros(p.e["x"].size, bool)
    mg = np.zeros(p.g["x"].size, bool)
    for c in cells:
        me[p.off_e[c]:p.off_e[c + 1]] = True
        mg[p.off_g[c]:p.off_g[c + 1]] = True
    return me, mg
