"""GPU parity of the Compton step with the sampler network in place of the
inverse-CDF sampler (through the C ABI), against the FP64 oracle step fed the
angle the network oracle gives for the same (x, u): FP32 network per event,
BF16 / FP8 networks per event within their rounding, the domain fallback
count, the strategies' agreement and the error paths."""
import sys

import numpy as np
import pytest

from paper_2206_02937_amd import plasma

from . import parity

pytestmark = pytest.mark.gpu


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
    c.close()


@pytest.fixture(scope="module")
def mo():
    from oracle import mlp_oracle

    return mlp_oracle


def _net_params(mo, seed=21):
    """Glorot weights, small biases; the cos(theta) output is widened so that
    it spans [-1, 1] and part of it is clamped."""
    rng = np.random.default_rng([seed, 5])
    p = mo.glorot_uniform(rng)
    for _, b in mo.unpack(p):
        b[:] = rng.uniform(-0.1, 0.1, size=b.shape)
    W5, b5 = mo.unpack(p)[-1]
    W5[0] *= 40.0
    b5[0] = 2.3
    return p.astype(np.float32)


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _quantized_forward(mo, params64, xf, uf, precision, calib):
    if precision == "mlp_f32":
        return mo.forward(params64, xf, uf)
    if precision == "mlp_bf16":
        return mo.forward_quantized(params64, xf, uf, "bf16")
    cx, cu = calib
    _, hs, _ = mo.forward(params64, cx.astype(np.float64), cu.astype(np.float64), keep=True)
    amax = {li: float(np.max(np.abs(hs[li]))) for li in (1, 2, 3)}
    return mo.forward_quantized(params64, xf, uf, "e4m3", act_scales=amax)


def oracle_net_step(orc, mo, p, state_e, state_g, step, params, precision, calib=None, cells=None):
    """The oracle step with cos(theta) from the network oracle: x from the
    oracle's own pair diagnostics, u from the oracle's Philox stream, both
    rounded to FP32 as the network takes them; outside the network's x
    domain the plain sampler answers."""
    _, _, _, diag = parity.run_oracle(orc, p, state_e, state_g, step, cells=cells)
    ne = state_e["x"].size
    u_mu, _ = orc.scatter_uniforms(np.arange(ne), p.seed, step)
    x = diag["x"]
    xf = x.astype(np.float32)
    uf = u_mu.astype(np.float32)
    valid = (diag["P"] >= 0) & (x > 0)
    inside = valid & (xf >= np.float32(mo.X_MIN)) & (xf <= np.float32(mo.X_MAX))
    mu = np.full(ne, np.nan)
    y = _quantized_forward(mo, params.astype(np.float64), xf[inside].astype(np.float64),
                           uf[inside].astype(np.float64), precision, calib)
    mu[inside] = 1.0 - mo.reading_v(y, xf[inside].astype(np.float64))
    mu_raw = np.full(ne, np.nan)
    mu_raw[inside] = y[:, 0]
    e = {k: v.copy() for k, v in state_e.items()}
    g = {k: v.copy() for k, v in state_g.items()}
    st = orc.compton_step(e, g, p.off_e, p.off_g, p.dt, p.density_norm, p.seed, step, cells=cells, mu_given=mu)
    collided = valid & (diag["u"] < diag["P"])
    return e, g, st, diag, mu_raw, collided, inside


def per_event_errors(before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, diag):
    """Per-particle error (parity metric) of the particles of collided pairs
    and a check that every other particle is bitwise unchanged."""

    def arr(d):
        return np.stack([d["x"], d["y"], d["z"]], axis=1).astype(np.float64)

    pr, pg, p0 = arr(ref_e), arr(gpu_e), arr(before_e)
    kr, kg, k0 = arr(ref_g), arr(gpu_g), arr(before_g)
    err_e = np.linalg.norm(pg - pr, axis=1) / np.sqrt(1.0 + (pr * pr).sum(1))
    eps = np.sqrt((kr * kr).sum(1))
    err_g = np.linalg.norm(kg - kr, axis=1) / np.where(eps > 0, eps, 1.0)
    untouched_e = np.all(pr == p0, axis=1)
    untouched_g = np.all(kr == k0, axis=1)
    return err_e, err_g, untouched_e, untouched_g


def _plasma(dtype, seed=4):
    p = plasma.grid(seed=seed, nx=8, ny=8, per_cell=256, dtype=dtype)
    p.dt *= 4.0  # about 20 % of the pairs collide
    return p


def run_case(ctx, orc, mo, p, precision, strategy="fused", step=1, cells=None):
    from paper_2206_02937_amd import compton

    params = _net_params(mo)
    net = compton.MLP(ctx, params)
    calib = None
    if precision == "mlp_bf16":
        net.quantize("mlp_bf16")
    elif precision == "mlp_fp8":
        cx, cu = plasma.sampler_inputs(65536, seed=7)
        calib = (cx.astype(np.float32), cu.astype(np.float32))
        net.quantize("mlp_fp8", _dev(calib[0]), _dev(calib[1]))
    ctx.set_strategy(strategy)
    e_dev, g_dev, oe, og = compton.to_device(p)
    before_e, before_g = compton.to_host(e_dev), compton.to_host(g_dev)
    stats = ctx.stats_buffer()
    _log(f"  {precision} {strategy} {p.e['x'].dtype}: gpu step")
    ctx.step(e_dev, g_dev, oe, og, p.dt, p.density_norm, p.seed, step, sampler=precision, mlp=net, stats=stats)
    st = compton.decode_stats(stats)
    gpu_e, gpu_g = compton.to_host(e_dev), compton.to_host(g_dev)
    _log("  oracle step")
    ref_e, ref_g, ost, diag, mu, collided, inside = oracle_net_step(orc, mo, p, before_e, before_g, step, params,
                                                                    precision, calib, cells)
    ctx.set_strategy("fused")
    net.close()
    return before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, st, ost, diag, mu, collided, inside


def _ambiguous(diag):
    P, u = diag["P"], diag["u"]
    return (P >= 0) & (np.abs(u - P) <= 1e-12 * np.maximum(P, 0))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("strategy", ["fused", "compact"])
def test_step_f32_network_matches_oracle(ctx, orc, mo, dtype, strategy):
    p = _plasma(dtype)
    (before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, st, ost, diag, mu, collided,
     inside) = run_case(ctx, orc, mo, p, "mlp_f32", strategy)
    amb = _ambiguous(diag)
    assert amb.sum() <= 3
    err_e, err_g, ue, ug = per_event_errors(before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, diag)
    ok_e = ~amb
    ok_g = np.ones(err_g.size, bool)
    ok_g[diag["partner"][amb]] = False
    # untouched particles stay bitwise unchanged
    assert np.array_equal(np.stack([gpu_e[c] for c in "xyz"])[:, ue & ok_e],
                          np.stack([before_e[c] for c in "xyz"])[:, ue & ok_e])
    assert np.array_equal(np.stack([gpu_g[c] for c in "xyz"])[:, ug & ok_g],
                          np.stack([before_g[c] for c in "xyz"])[:, ug & ok_g])
    # The FP32 network's cos(theta) differs from the FP64 network oracle by a
    # few 1e-7; the scattered momenta inherit it (times 1/sin(theta) for the
    # direction).  Bound: the FP32 per-event tolerance 1e-5, except pairs whose
    # network output lies within 1e-4 of +-1 (at or near the clamp), bounded
    # by 1e-3.
    near_pole = collided & inside & (np.abs(np.abs(np.nan_to_num(mu, nan=0.0)) - 1.0) < 1e-4)
    pole_g = np.zeros(err_g.size, bool)
    pole_g[diag["partner"][near_pole]] = True
    te = ok_e & ~near_pole
    tg = ok_g & ~pole_g
    _log(f"  max err e {err_e[te].max():.2e} g {err_g[tg].max():.2e}; near-pole {near_pole.sum()}; "
         f"collided {collided.sum()} fallback {(collided & ~inside).sum()}")
    assert err_e[te].max() <= 1e-5 and err_g[tg].max() <= 1e-5
    assert near_pole.sum() <= 5
    if near_pole.any():
        assert err_e[near_pole].max() <= 1e-3 and err_g[pole_g].max() <= 1e-3
    assert st["n_collided"] == ost["n_collided"] == int(collided.sum()) or amb.any()
    assert abs(st["n_collided"] - int(collided.sum())) <= amb.sum()
    assert abs(st["n_fallback"] - int((collided & ~inside).sum())) <= amb.sum()
    assert (collided & inside).sum() > 1000
    assert abs(st["energy_after"] - st["energy_before"]) <= 1e-12 * st["energy_before"]


# One rounding step of each reduced format at unit magnitude (the spacing of
# the format's values in [1, 2)): the largest change one rounding decision of
# a unit-sized quantity can make.
ROUNDING_STEP = {"mlp_bf16": 2.0 ** -7, "mlp_fp8": 2.0 ** -3}


def gpu_network_mu(net, precision, diag, u_mu, sel):
    """cos(theta) the library's network gives at the FP32 rounding of the
    oracle's (x, u) of the electrons in sel (its raw outputs, cs_mlp_forward,
    read by the oracle's reading of the two outputs, in FP64 as the step
    reads them); NaN elsewhere."""
    from oracle import mlp_oracle as mo

    mu = np.full(diag["x"].size, np.nan)
    if not sel.any():
        return mu
    xf = diag["x"][sel].astype(np.float32)
    uf = u_mu[sel].astype(np.float32)
    y = net.forward(_dev(xf), _dev(uf), precision).cpu().numpy().astype(np.float64)
    mu[sel] = 1.0 - mo.reading_v(y, xf.astype(np.float64))
    return mu


def network_parity(orc, p, net, precision, before_e, before_g, gpu_e, gpu_g, step, cells=None, emu=None):
    """Per-event parity of a GPU step with the network sampler, in two parts
    that bound every event:
      (1) the oracle step fed, for each collided pair inside the network's
          domain, the cos(theta) the library's network gives at that pair's
          (x, u) must match the GPU step per event to the storage tolerance
          (everything but the network evaluation is checked in full);
      (2) that cos(theta) must lie within one rounding step of the format
          (ROUNDING_STEP) of the network oracle's emulation, for every event
          (emu: callable (x, u) -> raw outputs y[n, 2] of the network's
          oracle with the network's x range).
    Returns (parity result, mu deviations |mu_gpu - mu_emu|, event count)."""
    from oracle import mlp_oracle as mo

    _, _, _, diag = parity.run_oracle(orc, p, before_e, before_g, step, cells=cells)
    ne = before_e["x"].size
    u_mu, _ = orc.scatter_uniforms(np.arange(ne), p.seed, step)
    x = diag["x"]
    xf = x.astype(np.float32)
    lo, hi = net.domain
    valid = (diag["P"] >= 0) & (x > 0)
    inside = valid & (xf >= np.float32(lo)) & (xf <= np.float32(hi))
    collided = valid & (diag["u"] < diag["P"])
    # the network is asked for every pair that could collide (ambiguous
    # decisions included), so the oracle step never falls back by accident
    mu_gpu = gpu_network_mu(net, precision, diag, u_mu, inside)
    e = {k: v.copy() for k, v in before_e.items()}
    g = {k: v.copy() for k, v in before_g.items()}
    orc.compton_step(e, g, p.off_e, p.off_g, p.dt, p.density_norm, p.seed, step, cells=cells, mu_given=mu_gpu)
    me = mg = None
    if cells is not None:
        me, mg = parity.cell_masks(p, cells)
    res = parity.compare(before_e, before_g, gpu_e, gpu_g, e, g, diag, before_e["x"].dtype, me, mg)
    dev = np.zeros(0)
    sel = collided & inside
    if emu is not None and sel.any():
        xs = xf[sel].astype(np.float64)
        y = emu(xs, u_mu[sel].astype(np.float32).astype(np.float64))
        dev = np.abs((1.0 - mo.reading_v(y, xs)) - mu_gpu[sel])
    return res, dev, int(sel.sum())


@pytest.mark.parametrize("precision", ["mlp_bf16", "mlp_fp8"])
def test_step_quantized_network_matches_emulation(ctx, orc, mo, precision):
    """Reduced-precision networks inside the step, every event bounded: the
    step matches the FP64 oracle fed the library network's cos(theta) to
    1e-12 per event (FP64 storage), and that cos(theta) lies within one
    rounding step of the format of the oracle's rounding emulation.  (The
    kernel's SiLU and accumulation order differ from the emulation by ~1e-6
    relative, which moves a few layer inputs across a rounding boundary.)"""
    from paper_2206_02937_amd import compton

    p = _plasma(np.float64)
    params = _net_params(mo)
    net = compton.MLP(ctx, params)
    calib = None
    if precision == "mlp_bf16":
        net.quantize("mlp_bf16")
    else:
        cx, cu = plasma.sampler_inputs(65536, seed=7)
        calib = (cx.astype(np.float32), cu.astype(np.float32))
        net.quantize("mlp_fp8", _dev(calib[0]), _dev(calib[1]))
    e_dev, g_dev, oe, og = compton.to_device(p)
    before_e, before_g = compton.to_host(e_dev), compton.to_host(g_dev)
    stats = ctx.stats_buffer()
    ctx.step(e_dev, g_dev, oe, og, p.dt, p.density_norm, p.seed, 1, sampler=precision, mlp=net, stats=stats)
    st = compton.decode_stats(stats)
    gpu_e, gpu_g = compton.to_host(e_dev), compton.to_host(g_dev)
    emu = lambda x, u: _quantized_forward(mo, params.astype(np.float64), x, u, precision, calib)  # noqa: E731
    res, dev, n_ev = network_parity(orc, p, net, precision, before_e, before_g, gpu_e, gpu_g, 1, emu=emu)
    _log(f"  {precision}: {n_ev} network events; {res}; |mu - emu| max {dev.max():.3e}, "
         f"p99 {np.percentile(dev, 99):.3e}, exact to 1e-6: {np.mean(dev <= 1e-6):.4f}")
    parity.assert_parity(res, np.float64, precision)
    assert n_ev > 1000
    assert dev.max() <= ROUNDING_STEP[precision], dev.max()
    # the oracle emulation reproduces most events to FP32 accuracy
    assert np.mean(dev <= 1e-5) >= (0.8 if precision == "mlp_bf16" else 0.5)
    assert abs(st["energy_after"] - st["energy_before"]) <= 1e-12 * st["energy_before"]
    net.close()


def test_step_network_fallback_heavy(ctx, orc, mo):
    """Power-law electrons with blackbody photons: most rest-frame energies
    fall below the network's domain, so the plain sampler answers those."""
    p = plasma.power_law(seed=1, n_cells=16, per_cell=256)
    p.dt *= 50.0
    (before_e, before_g, gpu_e, gpu_g, ref_e, ref_g, st, ost, diag, mu, collided,
     inside) = run_case(ctx, orc, mo, p, "mlp_f32")
    n_fb = int((collided & ~inside).sum())
    _log(f"  collided {collided.sum()} fallback {n_fb}")
    assert n_fb > 0.5 * collided.sum() and (collided & inside).sum() > 0
    assert st["n_fallback"] == n_fb


@pytest.mark.parametrize("precision", ["mlp_f32", "mlp_bf16", "mlp_fp8"])
def test_strategies_agree_with_network(ctx, mo, precision):
    import torch

    from paper_2206_02937_amd import compton

    p = _plasma(np.float32, seed=6)
    net = compton.MLP(ctx, _net_params(mo))
    if precision == "mlp_bf16":
        net.quantize(precision)
    elif precision == "mlp_fp8":
        cx, cu = plasma.sampler_inputs(4096, seed=7)
        net.quantize(precision, _dev(cx.astype(np.float32)), _dev(cu.astype(np.float32)))
    outs = []
    for strategy in ("fused", "compact"):
        ctx.set_strategy(strategy)
        e, g, oe, og = compton.to_device(p)
        stats = ctx.stats_buffer()
        for s in range(3):
            ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, s, sampler=precision, mlp=net, stats=stats)
        torch.cuda.synchronize()
        outs.append((compton.to_host(e), compton.to_host(g), compton.decode_stats(stats)))
    ctx.set_strategy("fused")
    (e0, g0, s0), (e1, g1, s1) = outs
    for c in "xyzw":
        assert np.array_equal(e0[c], e1[c]) and np.array_equal(g0[c], g1[c])
    for k in ("n_pairs", "n_collided", "n_clipped", "n_invalid", "n_fallback"):
        assert s0[k] == s1[k]
    net.close()


@pytest.mark.parametrize("precision", ["mlp_bf16", "mlp_fp8"])
def test_network_list_modes_identical(ctx, mo, precision):
    """The compact strategy's collide kernel with a network sampler, in both
    of its accepted-pair list layouts: one pair chunk per pair workgroup on
    a 68x68-cell grid (4624 workgroups, more than the 4096 whose segment
    counts a collide workgroup scans: the look-back list) and 16 chunks per
    workgroup (the segments).  Both give the fused strategy's bits."""
    import torch

    from paper_2206_02937_amd import compton

    p = plasma.grid(seed=23, nx=68, ny=68, per_cell=256)
    p.dt *= 4.0
    assert int(np.minimum(np.diff(p.off_e), np.diff(p.off_g)).sum()) // 256 > 4096
    net = compton.MLP(ctx, _net_params(mo))
    if precision == "mlp_bf16":
        net.quantize(precision)
    else:
        cx, cu = plasma.sampler_inputs(4096, seed=7)
        net.quantize(precision, _dev(cx.astype(np.float32)), _dev(cu.astype(np.float32)))
    outs = []
    try:
        for strategy, chunks in (("fused", 0), ("compact", 1), ("compact", 16)):
            _log(f"  {precision} {strategy} chunks per workgroup {chunks}")
            ctx.set_strategy(strategy)
            ctx.set_chunks_per_block(chunks)
            ctx.set_pairs_per_lane(1 if strategy == "compact" else 0)
            e, g, oe, og = compton.to_device(p)
            stats = ctx.stats_buffer()
            for s in range(2):
                ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, s, sampler=precision, mlp=net, stats=stats)
            torch.cuda.synchronize()
            outs.append((compton.to_host(e), compton.to_host(g), compton.decode_stats(stats)))
    finally:
        ctx.set_strategy("fused")
        ctx.set_chunks_per_block(0)
        ctx.set_pairs_per_lane(0)
    e0, g0, s0 = outs[0]
    assert s0["n_collided"] > 0
    for e1, g1, s1 in outs[1:]:
        for c in "xyzw":
            assert np.array_equal(e0[c], e1[c]) and np.array_equal(g0[c], g1[c])
        for k in ("n_pairs", "n_collided", "n_clipped", "n_invalid", "n_fallback"):
            assert s0[k] == s1[k]
    net.close()


def test_network_sampler_errors(ctx, mo):
    import torch

    from paper_2206_02937_amd import compton

    p = _plasma(np.float32)
    e, g, oe, og = compton.to_device(p)
    net = compton.MLP(ctx, _net_params(mo))
    with pytest.raises(compton.CSError) as ei:
        ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, 0, sampler="mlp_bf16", mlp=net)
    assert ei.value.code == compton.CS_ERR_NOT_READY
    with pytest.raises(compton.CSError) as ei:
        ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, 0, sampler="mlp_f32", mlp=None)
    assert ei.value.code == compton.CS_ERR_NOT_READY
    with pytest.raises(compton.CSError) as ei:
        ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, 0, sampler="plain", mlp=net)
    assert ei.value.code == compton.CS_ERR_INVALID_ARG
    ctx.set_strategy("multi_kernel")
    with pytest.raises(compton.CSError) as ei:
        ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, 0, sampler="mlp_f32", mlp=net)
    assert ei.value.code == compton.CS_ERR_UNSUPPORTED
    ctx.set_strategy("fused")
    torch.cuda.synchronize()
    net.close()
