"""The benchmark's own configuration against the FP64 oracle: the 128x128-cell
grid with 256 electrons and 256 photons per cell in FP32 storage (2^22 pairs
per step), the compact strategy with 16 chunks per pair workgroup and one
pair per lane, one captured step replayed as a HIP graph, with the plain
sampler and with the shipped network in BF16.  The oracle checks 256 sampled
cells element by element after each of two replays (each from the GPU's
state before that replay); the network events are bounded as in the step
tests: the step against the oracle fed the library network's cos(theta), and
that cos(theta) within one BF16 rounding step of the oracle's emulation."""
import os
import sys

import numpy as np
import pytest

from paper_2206_02937_amd import plasma

from . import parity
from .test_gpu_step_net import ROUNDING_STEP, network_parity

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2206_02937_amd",
                       "weights", "sampler_2x64x4.csnet")


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2206_02937_amd import compton

    c = compton.Context(0)
    c.set_strategy("compact")
    c.set_chunks_per_block(16)
    c.set_pairs_per_lane(1)
    yield c
    c.set_strategy("fused")
    c.set_chunks_per_block(0)
    c.set_pairs_per_lane(0)
    c.close()


@pytest.fixture(scope="module")
def workload():
    return plasma.make("grid_large", seed=0)


@pytest.mark.parametrize("sampler", ["plain", "mlp_bf16"])
def test_headline_configuration_matches_oracle(ctx, orc, workload, sampler):
    import torch

    from oracle import mlp_oracle as mo
    from paper_2206_02937_amd import compton

    p = workload
    assert p.n_cells == 16384 and p.n_pairs == 1 << 22 and p.e["x"].dtype == np.float32
    net = None
    if sampler != "plain":
        net = compton.MLP.load(ctx, WEIGHTS)
        net.quantize(sampler)
        params64 = net.get_params().astype(np.float64)
    rng = np.random.default_rng(17)
    cells = np.sort(rng.choice(p.n_cells, 256, replace=False))
    e, g, oe, og = compton.to_device(p)
    stats = ctx.stats_buffer()
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        gr = ctx.graph(e, g, oe, og, p.dt, p.density_norm, p.seed, sampler=sampler, mlp=net, stats=stats)
        try:
            for step in (0, 1):
                gr.set_step(step)
                stream.synchronize()
                before_e, before_g = compton.to_host(e), compton.to_host(g)
                _log(f"  {sampler} replay of step {step}")
                gr.launch()
                stream.synchronize()
                gpu_e, gpu_g = compton.to_host(e), compton.to_host(g)
                st = compton.decode_stats(stats)
                assert st["n_pairs"] == p.n_pairs and st["layout_error"] == 0
                assert st["n_collided"] > 150000
                _log(f"  oracle on {cells.size} cells")
                if net is None:
                    ref_e, ref_g, _, diag = parity.run_oracle(orc, p, before_e, before_g, step, cells=cells)
                    me, mg = parity.cell_masks(p, cells)
                    res = parity.compare(before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, diag, np.float32, me, mg)
                    _log(f"  {res}")
                    parity.assert_parity(res, np.float32, f"step {step}")
                else:
                    emu = lambda x, u: mo.forward_quantized(params64, x, u, "bf16", domain=net.domain)  # noqa: E731
                    res, dev, n_ev = network_parity(orc, p, net, sampler, before_e, before_g, gpu_e, gpu_g, step,
                                                    cells=cells, emu=emu)
                    _log(f"  {n_ev} network events; {res}; |mu - emu| max {dev.max():.3e}")
                    parity.assert_parity(res, np.float32, f"step {step}")
                    assert n_ev > 1000
                    assert dev.max() <= ROUNDING_STEP[sampler]
                assert res["n_expected_e"] == int(np.diff(p.off_e)[cells].sum()) - res["n_ambiguous"]
        finally:
            gr.close()
    if net is not None:
        net.close()
