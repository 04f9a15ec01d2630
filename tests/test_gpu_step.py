"""GPU parity of the Compton step (through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs and the same Philox stream, and
the step's edge cases: ragged and uneven cells, unequal species counts, empty
cells, invalid inputs, bad layouts, determinism."""
import math
import sys

import numpy as np
import pytest

from paper_2206_02937_amd import plasma

from . import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2206_02937_amd import compton

    c = compton.Context(0)
    yield c
    c.close()


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_step(ctx, p, e_dev, g_dev, oe, og, step):
    import torch

    from paper_2206_02937_amd import compton

    stats = ctx.stats_buffer()
    ctx.step(e_dev, g_dev, oe, og, p.dt, p.density_norm, p.seed, step, stats=stats)
    torch.cuda.synchronize()
    return compton.decode_stats(stats)


def step_and_compare(ctx, orc, p, steps, cells=None, check_stats=True):
    """Run `steps` GPU steps; before each, snapshot the GPU state, run the
    oracle from that snapshot (all cells or the listed ones), compare."""
    from paper_2206_02937_amd import compton

    e_dev, g_dev, oe, og = compton.to_device(p)
    dtype = p.e["x"].dtype
    out = []
    for s in steps:
        before_e, before_g = compton.to_host(e_dev), compton.to_host(g_dev)
        _log(f"  step {s}: gpu")
        st = gpu_step(ctx, p, e_dev, g_dev, oe, og, s)
        after_e, after_g = compton.to_host(e_dev), compton.to_host(g_dev)
        _log(f"  step {s}: oracle")
        ref_e, ref_g, ost, diag = parity.run_oracle(orc, p, before_e, before_g, s, cells=cells)
        me = mg = None
        if cells is not None:
            me, mg = parity.cell_masks(p, cells)
        res = parity.compare(before_e, before_g, after_e, after_g, ref_e, ref_g, diag, dtype, me, mg)
        _log(f"  step {s}: {res} collided gpu={st['n_collided']} oracle={ost['n_collided']}")
        parity.assert_parity(res, dtype, f"step {s}")
        if check_stats and cells is None:
            assert st["layout_error"] == 0
            assert st["n_pairs"] == ost["n_pairs"]
            assert abs(st["n_collided"] - ost["n_collided"]) <= res["n_ambiguous"]
            assert st["n_clipped"] == ost["n_clipped"] and st["n_invalid"] == ost["n_invalid"]
            assert abs(st["sum_prob"] - ost["sum_prob"]) <= 1e-12 * max(1.0, ost["sum_prob"])
            if res["n_ambiguous"] == 0:
                tol = 1e-13 * max(1.0, ost["energy_before"])
                assert abs(st["energy_before"] - ost["energy_before"]) <= tol
                assert abs(st["energy_after"] - ost["energy_after"]) <= tol
        out.append((st, ost, res))
    return out


def test_single_cell_fp64_parity(ctx, orc):
    """0D cell, 16384 pairs, FP64: per-event 1e-12 over three steps."""
    p = plasma.single_cell(seed=0)
    res = step_and_compare(ctx, orc, p, [0, 1, 2])
    assert all(r[0]["n_collided"] > 600 for r in res)


def test_grid_fp32_ragged_parity(ctx, orc):
    """FP32 storage, 6x5 cells of 200 pairs: chunks of 256 straddle cells."""
    p = plasma.grid(seed=1, nx=6, ny=5, per_cell=200)
    step_and_compare(ctx, orc, p, [0, 7])


def test_grid_fp64_storage_parity(ctx, orc):
    p = plasma.grid(seed=2, nx=4, ny=4, per_cell=256, dtype=np.float64)
    step_and_compare(ctx, orc, p, [3])


def test_grid_full_size_sampled_cells(ctx, orc):
    """The full 64x64x256 FP32 grid in the benchmark's launch configuration;
    the oracle checks 192 sampled cells element by element."""
    p = plasma.grid(seed=0)
    rng = np.random.default_rng(0)
    cells = np.sort(rng.choice(p.n_cells, 192, replace=False))
    step_and_compare(ctx, orc, p, [0, 1], cells=cells)


def test_uneven_cells_parity(ctx, orc):
    """Poisson cell counts with a density bump (a small version of the uneven
    workload), including empty cells."""
    p = plasma.uneven(seed=3, side=24, mean=3, peak=20.0, area_frac=0.05)
    n_empty = int((np.diff(p.off_e) == 0).sum())
    assert n_empty > 0, n_empty
    step_and_compare(ctx, orc, p, [0, 1])


def test_uneven_full_size_sampled_cells(ctx, orc):
    p = plasma.uneven(seed=0)
    counts = np.diff(p.off_e)
    big = np.argsort(counts)[-20:]
    rng = np.random.default_rng(1)
    cells = np.unique(np.concatenate([big, rng.choice(p.n_cells, 200, replace=False)]))
    step_and_compare(ctx, orc, p, [0], cells=cells)


def test_power_law_sampled_cells(ctx, orc):
    """Precision stress: gamma up to 1e4, blackbody photons, 2^24 pairs FP32."""
    p = plasma.power_law(seed=0)
    rng = np.random.default_rng(2)
    cells = np.sort(rng.choice(p.n_cells, 128, replace=False))
    step_and_compare(ctx, orc, p, [0], cells=cells)


def _unequal_plasma(dtype=np.float64):
    rng = np.random.default_rng(9)
    counts_e = np.array([5, 0, 17, 300, 3, 1, 0, 40, 513])
    counts_g = np.array([9, 4, 17, 10, 3, 0, 0, 600, 2])
    ne, ng = int(counts_e.sum()), int(counts_g.sum())
    pm = plasma.maxwell_juttner_momentum(rng, ne, 0.5)
    ux, uy, uz = plasma.isotropic(rng, ne)
    eps = plasma.log_uniform(rng, ng, 1e-3, 1.0)
    vx, vy, vz = plasma.isotropic(rng, ng)
    e = {"x": pm * ux, "y": pm * uy, "z": pm * uz, "w": rng.uniform(0.5, 2.0, ne)}
    g = {"x": eps * vx, "y": eps * vy, "z": eps * vz, "w": rng.uniform(0.5, 2.0, ng)}
    e = {k: v.astype(dtype) for k, v in e.items()}
    g = {k: v.astype(dtype) for k, v in g.items()}
    off_e = np.concatenate([[0], np.cumsum(counts_e)]).astype(np.int64)
    off_g = np.concatenate([[0], np.cumsum(counts_g)]).astype(np.int64)
    return plasma.Plasma("unequal", e, g, off_e, off_g, 0.4, 0.05, 11)


def test_unequal_species_and_weights(ctx, orc):
    """N_e != N_gamma, empty cells, unequal macro-particle weights."""
    p = _unequal_plasma()
    res = step_and_compare(ctx, orc, p, [0, 1, 2])
    assert res[0][0]["n_pairs"] == int(np.minimum(np.diff(p.off_e), np.diff(p.off_g)).sum())


def test_invalid_inputs_and_clipping(ctx, orc):
    p = plasma.grid(seed=4, nx=3, ny=3, per_cell=256, dtype=np.float64)
    p.dt = 40.0  # many P > 1
    p.e["x"][5] = np.nan
    p.e["w"][600] = -1.0
    p.g["z"][1000] = np.inf
    res = step_and_compare(ctx, orc, p, [0])
    st, ost, _ = res[0]
    assert st["n_clipped"] > 0 and st["n_invalid"] >= 2


def test_bad_layout_touches_nothing(ctx):
    import torch

    from paper_2206_02937_amd import compton

    p = plasma.grid(seed=5, nx=4, ny=1, per_cell=64)
    e_dev, g_dev, oe, og = compton.to_device(p)
    bad = oe.clone()
    bad[2] = bad[3] + 1  # decreasing
    before = compton.to_host(e_dev)
    stats = ctx.stats_buffer()
    ctx.step(e_dev, g_dev, bad, og, p.dt, p.density_norm, 0, 0, stats=stats)
    torch.cuda.synchronize()
    st = compton.decode_stats(stats)
    assert st["layout_error"] == 1 and st["n_pairs"] == 0 and st["n_collided"] == 0
    after = compton.to_host(e_dev)
    for k in "xyz":
        assert np.array_equal(before[k], after[k])
    assert ctx.check_layout(oe, p.e["x"].size)
    assert not ctx.check_layout(bad, p.e["x"].size)
    short = oe.clone()
    short[-1] -= 1  # does not end at the particle count
    assert not ctx.check_layout(short, p.e["x"].size)


def test_empty_problem(ctx):
    import torch

    from paper_2206_02937_amd import compton

    z = torch.zeros(0, dtype=torch.float32, device="cuda:0")
    e = {"x": z, "y": z, "z": z, "w": z}
    off = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    stats = ctx.stats_buffer()
    ctx.step(e, e, off, off, 0.1, 1.0, 0, 0, stats=stats)
    torch.cuda.synchronize()
    assert compton.decode_stats(stats)["n_pairs"] == 0
    off4 = torch.zeros(4, dtype=torch.int64, device="cuda:0")
    ctx.step(e, e, off4, off4, 0.1, 1.0, 0, 0, stats=stats)
    torch.cuda.synchronize()
    st = compton.decode_stats(stats)
    assert st["n_pairs"] == 0 and st["layout_error"] == 0


def test_argument_validation(ctx):
    import torch

    from paper_2206_02937_amd import compton

    p = plasma.grid(seed=6, nx=2, ny=1, per_cell=16)
    e_dev, g_dev, oe, og = compton.to_device(p)
    for kwargs, code in [({"dt": 0.0}, compton.CS_ERR_INVALID_ARG), ({"dt": float("nan")}, compton.CS_ERR_INVALID_ARG),
                         ({"density_norm": -1.0}, compton.CS_ERR_INVALID_ARG),
                         ({"sampler": "mlp_bf16"}, compton.CS_ERR_NOT_READY)]:
        args = dict(dt=0.1, density_norm=1.0, sampler="plain")
        args.update(kwargs)
        with pytest.raises(compton.CSError) as ei:
            ctx.step(e_dev, g_dev, oe, og, args["dt"], args["density_norm"], 0, 0, sampler=args["sampler"])
        assert ei.value.code == code
    with pytest.raises(compton.CSError) as ei:
        ctx.step(e_dev, g_dev, oe[:1], og[:1], 0.1, 1.0, 0, 0)
    assert ei.value.code == compton.CS_ERR_INVALID_ARG  # particles given but no cells


def test_deterministic_and_repeatable(ctx):
    """Two runs of the same steps from the same state are bitwise equal,
    including the stats."""
    import torch

    from paper_2206_02937_amd import compton

    p = plasma.grid(seed=7, nx=16, ny=16, per_cell=256)
    results = []
    for _ in range(2):
        e_dev, g_dev, oe, og = compton.to_device(p)
        stats = ctx.stats_buffer()
        for s in range(4):
            ctx.step(e_dev, g_dev, oe, og, p.dt, p.density_norm, p.seed, s, stats=stats)
        torch.cuda.synchronize()
        results.append((compton.to_host(e_dev), compton.to_host(g_dev), stats.cpu().numpy().copy()))
    (e1, g1, s1), (e2, g2, s2) = results
    for k in "xyzw":
        assert np.array_equal(e1[k], e2[k]) and np.array_equal(g1[k], g2[k])
    assert np.array_equal(s1, s2)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_sample_plain_parity(ctx, orc, dtype):
    """The conventional sampler alone, against the oracle's inverse CDF:
    per element 1e-12 in FP64 (absolute in mu, relative in eps'/eps)."""
    import torch

    n = 4096
    x, u = plasma.sampler_inputs(n, seed=3, x_min=1e-8, x_max=1e3)
    x = np.concatenate([x, [0.0, 1e-12, 0.19999999, 0.2, 0.2000001, 100.0, 5.0, 1e-3]])
    u = np.concatenate([u, [0.3, 0.0, 1 - 2**-53, 0.5, 0.5, 1e-12, 0.999999, 0.5]])
    x = x.astype(dtype)
    u = u.astype(dtype)
    xd = torch.from_numpy(x).cuda()
    ud = torch.from_numpy(u).cuda()
    mu, r = ctx.sample_plain(xd, ud)
    torch.cuda.synchronize()
    mu = mu.cpu().numpy().astype(np.float64)
    r = r.cpu().numpy().astype(np.float64)
    mu_ref, r_ref = orc.sample_plain(x.astype(np.float64), u.astype(np.float64))
    tol = parity.tolerance(dtype)
    if dtype == np.float32:
        mu_ref = mu_ref.astype(np.float32).astype(np.float64)
        r_ref = r_ref.astype(np.float32).astype(np.float64)
        tol = 1e-6
    assert np.max(np.abs(mu - mu_ref)) <= tol
    assert np.max(np.abs(r - r_ref) / r_ref) <= tol


def test_compact_list_modes_identical(ctx):
    """The compact strategy lists its accepted pairs in one of two ways: one
    segment per pair workgroup whose prefix sums the collide kernel forms
    (up to 4096 pair workgroups), or a dense list ordered by the pair
    kernel's look-back (more workgroups).  A 68x68-cell grid (4624 chunks)
    with one chunk per pair workgroup takes the look-back, with 16 the
    segments; both match the fused strategy bitwise, and so does the pair
    kernel forced to 64-bit particle indexing (it otherwise reads with
    32-bit byte offsets)."""
    import torch

    from paper_2206_02937_amd import compton

    p = plasma.grid(seed=21, nx=68, ny=68, per_cell=256)
    n_chunks = int(np.minimum(np.diff(p.off_e), np.diff(p.off_g)).sum()) // 256
    assert n_chunks > 4096
    results = []
    for strategy, g, wide in (("fused", 0, 0), ("compact", 1, 0), ("compact", 16, 0), ("compact", 16, 1),
                              ("compact", 1, 1)):
        ctx.set_strategy(strategy)
        ctx.set_chunks_per_block(g)
        ctx.set_pairs_per_lane(1 if strategy == "compact" else 0)
        ctx.set_wide_index(wide)
        e_dev, g_dev, oe, og = compton.to_device(p)
        stats = ctx.stats_buffer()
        for s in range(2):
            ctx.step(e_dev, g_dev, oe, og, p.dt, p.density_norm, p.seed, s, stats=stats)
        torch.cuda.synchronize()
        results.append((compton.to_host(e_dev), compton.to_host(g_dev), stats.cpu().numpy().copy()))
    ctx.set_strategy("fused")
    ctx.set_chunks_per_block(0)
    ctx.set_pairs_per_lane(0)
    ctx.set_wide_index(0)
    assert ctx.get_option(compton.OPT_WIDE_INDEX) == 0
    e0, g0, s0 = results[0]
    assert s0[1] > 0  # collisions happened
    for e1, g1, s1 in results[1:]:
        for k in "xyzw":
            assert np.array_equal(e0[k], e1[k]), k
            assert np.array_equal(g0[k], g1[k]), k
        assert np.array_equal(s0[:8], s1[:8])
        assert np.allclose(s0.view(np.float64)[8:11], s1.view(np.float64)[8:11], rtol=1e-13, atol=0)


@pytest.mark.parametrize("workload", ["grid_small", "uneven_small", "unequal"])
def test_strategies_bitwise_identical(ctx, workload):
    """Every kernel strategy (compact with 1, 2, 4 pairs per lane and several
    chunks per pair workgroup, fused with several chunks per workgroup, the
    multi-kernel and per-cell baselines)
    gives bitwise-identical particles and counters; the
    FP64 sums of the stats differ only by summation order."""
    import torch

    from paper_2206_02937_amd import compton

    if workload == "grid_small":
        p = plasma.grid(seed=8, nx=12, ny=10, per_cell=256)
    elif workload == "uneven_small":
        p = plasma.uneven(seed=8, side=40, mean=20, peak=20.0, area_frac=0.05)
    else:
        p = _unequal_plasma(np.float32)
    # (strategy, pairs per lane, chunks per workgroup)
    variants = [("compact", 4, 0), ("compact", 1, 0), ("compact", 2, 0), ("compact", 1, 16), ("compact", 2, 5),
               ("compact", 4, 8), ("fused", 0, 0), ("fused", 0, 1), ("fused", 0, 3), ("fused", 0, 64),
               ("multi_kernel", 0, 0), ("per_cell", 0, 0)]
    results = []
    for strategy, ppl, g in variants:
        ctx.set_strategy(strategy)
        ctx.set_chunks_per_block(g)
        ctx.set_pairs_per_lane(ppl)
        e_dev, g_dev, oe, og = compton.to_device(p)
        stats = ctx.stats_buffer()
        for s in range(3):
            ctx.step(e_dev, g_dev, oe, og, p.dt, p.density_norm, p.seed, s, stats=stats)
        torch.cuda.synchronize()
        results.append((compton.to_host(e_dev), compton.to_host(g_dev), stats.cpu().numpy().copy()))
    ctx.set_strategy("fused")
    ctx.set_chunks_per_block(0)
    ctx.set_pairs_per_lane(0)
    ctx.set_wide_index(0)
    assert ctx.get_option(compton.OPT_WIDE_INDEX) == 0
    e0, g0, s0 = results[0]
    for (strategy, _, g), (e1, g1, s1) in zip(variants[1:], results[1:]):
        for k in "xyzw":
            assert np.array_equal(e0[k], e1[k]), (strategy, g, k)
            assert np.array_equal(g0[k], g1[k]), (strategy, g, k)
        assert np.array_equal(s0[:8], s1[:8]), (strategy, g)
        d0, d1 = s0.view(np.float64)[8:11], s1.view(np.float64)[8:11]
        assert np.allclose(d0, d1, rtol=1e-13, atol=0), (strategy, g, d0, d1)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_pair_x_matches_oracle(ctx, orc, dtype):
    """cs_pair_x (the rest-frame photon energy of pairs) against the oracle's
    invariant, relative 1e-13, on power-law electrons (gamma up to 1e4) with
    blackbody photons, plus a photon at rest (x = 0) and a head-on pair."""
    import torch

    p = plasma.power_law(seed=4, n_cells=8, per_cell=256).astype(dtype)
    n = p.e["x"].size
    e = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in p.e.items()}
    g = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in p.g.items()}
    g["x"][0] = g["y"][0] = g["z"][0] = 0.0
    e["x"][1], e["y"][1], e["z"][1] = 0.0, 0.0, 3.0
    g["x"][1], g["y"][1], g["z"][1] = 0.0, 0.0, -0.5
    x = ctx.pair_x(e, g).cpu().numpy()
    assert x.shape == (n,) and x.dtype == np.float64
    pe = np.stack([e[c].cpu().numpy() for c in "xyz"], axis=1).astype(np.float64)
    k = np.stack([g[c].cpu().numpy() for c in "xyz"], axis=1).astype(np.float64)
    ref = np.array([orc.pair_invariants(pe[i], k[i])[0] for i in range(n)])
    assert x[0] == 0.0 and ref[0] == 0.0
    assert abs(x[1] - 0.5 * (np.sqrt(10.0) + 3.0)) <= 1e-15 * x[1]  # x = eps (gamma + p) head-on
    rel = np.abs(x - ref) / np.maximum(ref, 1e-300)
    assert np.max(rel[1:]) <= 1e-13, np.max(rel[1:])
    assert x.max() > 1e-3 * x.min() and np.all(x[1:] > 0)
    with pytest.raises(Exception):
        ctx.pair_x(e, g, n=n + 1)
