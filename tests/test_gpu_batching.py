"""Batching of the step over uneven cells: the one-workgroup-per-cell baseline
gives the same bits as the batched strategies; a captured step replayed as a
HIP graph (step index in device memory) equals the eager steps, replay after
replay, with eager work and synchronisations in between; the autotuner leaves
the caller's particles untouched and picks a strategy whose results are the
same bits."""
import sys

import numpy as np
import pytest

from paper_2206_02937_amd import plasma

pytestmark = pytest.mark.gpu

WEIGHTS_SAMPLERS = ["plain", "mlp_bf16"]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2206_02937_amd import compton

    c = compton.Context(0)
    yield c
    c.set_strategy("fused")
    c.set_chunks_per_block(0)
    c.close()


@pytest.fixture(scope="module")
def net(ctx):
    import os

    from paper_2206_02937_amd import compton

    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2206_02937_amd",
                        "weights", "sampler_2x64x4.csnet")
    n = compton.MLP.load(ctx, path)
    n.quantize("mlp_bf16")
    yield n
    n.close()


def _uneven():
    return plasma.uneven(seed=5, side=40, mean=40, peak=20.0, area_frac=0.05)


def _same(a, b):
    return all(np.array_equal(a[c], b[c]) for c in "xyzw")


def test_per_cell_baseline_matches_fused(ctx):
    import torch

    from paper_2206_02937_amd import compton

    p = _uneven()
    outs = []
    for strategy in ("fused", "per_cell"):
        ctx.set_strategy(strategy)
        e, g, oe, og = compton.to_device(p)
        stats = ctx.stats_buffer()
        for s in range(3):
            ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, s, stats=stats)
        torch.cuda.synchronize()
        outs.append((compton.to_host(e), compton.to_host(g), compton.decode_stats(stats)))
    ctx.set_strategy("fused")
    (e0, g0, s0), (e1, g1, s1) = outs
    assert _same(e0, e1) and _same(g0, g1)
    for k in ("n_pairs", "n_collided", "n_clipped", "n_invalid", "n_fallback", "layout_error"):
        assert s0[k] == s1[k], k
    assert abs(s0["sum_prob"] - s1["sum_prob"]) <= 1e-13 * s0["sum_prob"]


@pytest.mark.parametrize("strategy", ["fused", "compact"])
@pytest.mark.parametrize("sampler", WEIGHTS_SAMPLERS)
def test_graph_replays_match_eager_steps(ctx, net, strategy, sampler):
    import torch

    from paper_2206_02937_amd import compton

    p = _uneven()
    mlp = None if sampler == "plain" else net
    ctx.set_strategy(strategy)
    ea, ga, oea, oga = compton.to_device(p)
    eb, gb, oeb, ogb = compton.to_device(p)
    sa, sb = ctx.stats_buffer(), ctx.stats_buffer()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        graph = ctx.graph(eb, gb, oeb, ogb, p.dt, p.density_norm, p.seed, sampler=sampler, mlp=mlp, stats=sb)
        graph.set_step(7)
        for k in range(4):
            _log(f"  {strategy} {sampler}: replay {k}")
            graph.launch()
            stream.synchronize()
            ctx.step(ea, ga, oea, oga, p.dt, p.density_norm, p.seed, 7 + k, sampler=sampler, mlp=mlp, stats=sa)
            stream.synchronize()
            hea, hga, heb, hgb = (compton.to_host(t) for t in (ea, ga, eb, gb))
            assert _same(hea, heb) and _same(hga, hgb), k
            st_a, st_b = compton.decode_stats(sa), compton.decode_stats(sb)
            assert st_a == st_b, (k, st_a, st_b)
            assert st_a["n_collided"] > 0
    graph.close()
    ctx.set_strategy("fused")


def test_graph_argument_errors(ctx):
    import torch

    from paper_2206_02937_amd import compton

    p = _uneven()
    e, g, oe, og = compton.to_device(p)
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    ctx.set_strategy("multi_kernel")
    with torch.cuda.stream(stream):
        with pytest.raises(compton.CSError) as ei:
            ctx.graph(e, g, oe, og, p.dt, p.density_norm, p.seed)
        assert ei.value.code == compton.CS_ERR_UNSUPPORTED
    ctx.set_strategy("fused")
    null_stream = torch.cuda.default_stream()
    if null_stream.cuda_stream == 0:
        with pytest.raises(compton.CSError) as ei:
            compton.Graph(ctx, e, g, oe, og, p.dt, p.density_norm, p.seed, "plain", None, None, null_stream)
        assert ei.value.code == compton.CS_ERR_INVALID_ARG


@pytest.mark.parametrize("sampler", WEIGHTS_SAMPLERS)
def test_autotune_keeps_particles_and_bits(ctx, net, sampler):
    import torch

    from paper_2206_02937_amd import compton

    p = _uneven()
    mlp = None if sampler == "plain" else net
    e, g, oe, og = compton.to_device(p)
    before_e, before_g = compton.to_host(e), compton.to_host(g)
    res = ctx.autotune(e, g, oe, og, p.dt, p.density_norm, p.seed, 3, sampler=sampler, mlp=mlp, reps=3)
    _log(f"  autotune {sampler}: {res}")
    torch.cuda.synchronize()
    assert _same(compton.to_host(e), before_e) and _same(compton.to_host(g), before_g)
    # fused 4..32, compact (1, 4/8/16), (2, 8/16), and the resident-fit chunks
    # for one and two pairs per lane unless one of those already has them
    assert 9 <= len(res["candidates"]) <= 11 and all(c[3] > 0 for c in res["candidates"])
    best = res["best"]
    assert ctx.get_option(compton.OPT_STRATEGY) == compton.STRATEGIES[best[0]]
    assert ctx.get_option(compton.OPT_CHUNKS_PER_BLOCK) == best[1]
    assert ctx.get_option(compton.OPT_PAIRS_PER_LANE) == best[2]
    # the tuned configuration and the default one give the same bits
    ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, 3, sampler=sampler, mlp=mlp)
    ctx.set_strategy("fused")
    ctx.set_chunks_per_block(0)
    ctx.set_pairs_per_lane(0)
    e2, g2, oe2, og2 = compton.to_device(p)
    ctx.step(e2, g2, oe2, og2, p.dt, p.density_norm, p.seed, 3, sampler=sampler, mlp=mlp)
    torch.cuda.synchronize()
    assert _same(compton.to_host(e), compton.to_host(e2)) and _same(compton.to_host(g), compton.to_host(g2))
