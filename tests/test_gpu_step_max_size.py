"""The step at the largest species sizes of the pair kernel's two indexing
forms.  The compact pair kernel forms particle byte offsets as unsigned 32-bit
values while every species has at most 2^32 / sizeof(T) elements (2^29 for
FP64 storage) and switches to 64-bit indexing beyond.  The seeded 64x64x256
FP64 grid (2^20 particles per species) tiled 512 times on the device puts each
species exactly at that limit, 513 times just past it (2,101,248 cells, about
5.4e8 pairs).  In both, the compact step's particles equal the fused
strategy's bit for bit (its counts too, its sums to rounding), and the last
cells -- whose particles lie beyond element 2^29 in the larger case -- and a
few others match the FP64 oracle per event.  Needs about 130 GB of device
memory and 20 GB of host memory; skipped when the device has less free."""
import numpy as np
import pytest

from paper_2206_02937_amd import plasma

from . import parity

pytestmark = pytest.mark.gpu

BASE_CELLS = 64 * 64
PER_CELL = 256


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2206_02937_amd import compton

    c = compton.Context(0)
    yield c
    c.set_strategy("fused")
    c.set_chunks_per_block(0)
    c.set_pairs_per_lane(0)
    c.close()


def _log(msg):
    print(msg, flush=True)


def _subset(d, ranges):
    return {k: np.concatenate([v[a:b] for a, b in ranges]) for k, v in d.items()}


@pytest.mark.parametrize("reps", [512, 513])
def test_largest_species_both_indexings(ctx, orc, reps):
    import torch

    from paper_2206_02937_amd import compton

    n = reps * BASE_CELLS * PER_CELL  # particles per species
    need = 4 * 8 * n * 2 * 2 + 96 * n  # two copies of both species, the compact workspace
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 2**30:.0f} GiB of free device memory, {free / 2**30:.0f} GiB free")
    assert (n > 1 << 29) == (reps == 513)
    base = plasma.grid(seed=5, nx=64, ny=64, per_cell=PER_CELL, dtype=np.float64)
    n_cells = reps * BASE_CELLS
    off_host = np.arange(n_cells + 1, dtype=np.int64) * PER_CELL
    off = torch.from_numpy(off_host).cuda()
    e0 = {k: torch.from_numpy(base.e[k]).cuda().repeat(reps) for k in "xyzw"}
    g0 = {k: torch.from_numpy(base.g[k]).cuda().repeat(reps) for k in "xyzw"}
    step = 3
    # the oracle's cells: the last four (the highest particle indices) and
    # four spread over the rest; their pre-step state on the host
    rng = np.random.default_rng(reps)
    cells = np.unique(np.concatenate([np.arange(n_cells - 4, n_cells),
                                      rng.choice(n_cells - 4, 4, replace=False)])).astype(np.int64)
    ranges = [(int(off_host[c]), int(off_host[c + 1])) for c in cells]
    e_host = {k: np.empty(n, np.float64) for k in "xyzw"}  # committed only where written
    g_host = {k: np.empty(n, np.float64) for k in "xyzw"}
    for a, b in ranges:
        for k in "xyzw":
            e_host[k][a:b] = e0[k][a:b].cpu().numpy()
            g_host[k][a:b] = g0[k][a:b].cpu().numpy()
    before_e, before_g = _subset(e_host, ranges), _subset(g_host, ranges)

    _log(f"  {reps} tiles, {n} particles per species: compact step")
    ctx.set_strategy("compact")
    ctx.set_chunks_per_block(0)
    ctx.set_pairs_per_lane(1)
    e1 = {k: v.clone() for k, v in e0.items()}
    g1 = {k: v.clone() for k, v in g0.items()}
    s1 = ctx.stats_buffer()
    ctx.step(e1, g1, off, off, base.dt, base.density_norm, base.seed, step, stats=s1)
    torch.cuda.synchronize()
    st1 = compton.decode_stats(s1)
    gpu_e = {k: np.concatenate([e1[k][a:b].cpu().numpy() for a, b in ranges]) for k in "xyzw"}
    gpu_g = {k: np.concatenate([g1[k][a:b].cpu().numpy() for a, b in ranges]) for k in "xyzw"}

    _log("  fused step on the same state")
    ctx.set_strategy("fused")
    ctx.set_chunks_per_block(0)
    ctx.set_pairs_per_lane(0)
    s0 = ctx.stats_buffer()
    ctx.step(e0, g0, off, off, base.dt, base.density_norm, base.seed, step, stats=s0)
    torch.cuda.synchronize()
    st0 = compton.decode_stats(s0)
    assert st1["layout_error"] == 0 and st1["n_pairs"] == n and st1["n_collided"] > 0
    for k in ("n_pairs", "n_collided", "n_clipped", "n_invalid"):
        assert st0[k] == st1[k], (k, st0[k], st1[k])
    # the sums are reduced over each strategy's own workgroups: the same
    # terms, another order
    for k in ("sum_prob", "energy_before", "energy_after"):
        assert abs(st0[k] - st1[k]) <= 1e-12 * abs(st0[k]), (k, st0[k], st1[k])
    for k in "xyzw":
        assert torch.equal(e0[k], e1[k]), k
        assert torch.equal(g0[k], g1[k]), k
    del e1, g1
    torch.cuda.empty_cache()

    _log(f"  oracle on cells {cells.tolist()}")
    st, diag = orc.compton_step(e_host, g_host, off_host, off_host, base.dt, base.density_norm, base.seed, step,
                                cells=cells, diagnostics=True)
    ref_e, ref_g = _subset(e_host, ranges), _subset(g_host, ranges)
    # the diagnostics of the listed electrons, partners renumbered into the
    # subset (electrons and photons share the offsets here)
    starts = np.cumsum([0] + [b - a for a, b in ranges])
    sub_diag = {k: np.concatenate([diag[k][a:b] for a, b in ranges]) for k in ("P", "u", "x")}
    partner = []
    for (a, b), s in zip(ranges, starts[:-1]):
        q = diag["partner"][a:b]
        partner.append(np.where(q >= 0, q - a + s, -1))
    sub_diag["partner"] = np.concatenate(partner)
    del diag
    res = parity.compare(before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, sub_diag, np.float64)
    _log(f"  {res}; collided oracle {st['n_collided']} of {st['n_pairs']} pairs")
    assert st["n_pairs"] == len(cells) * PER_CELL and st["n_collided"] > 0
    parity.assert_parity(res, np.float64, f"{reps} tiles")
    del e0, g0, off
    torch.cuda.empty_cache()
