"""GPU parity of the sampler network (through the C ABI) against the FP64
network oracle: FP32 forward, gradients (MSE and MAE), Adam, the BF16 and
FP8 MFMA forward against the oracle's rounding emulation, the sampler
reading of the outputs with its domain fallback, save / load, and the
not-prepared error paths."""
import os
import sys

import numpy as np
import pytest

from paper_2206_02937_amd import plasma

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
    c.close()


@pytest.fixture(scope="module")
def mlp_oracle():
    from oracle import mlp_oracle

    return mlp_oracle


def _params(mo, seed, bias_scale=0.1):
    """Glorot weights with small random biases (so every bias term is tested),
    rounded to float32 (the GPU's parameter format)."""
    rng = np.random.default_rng([seed, 77])
    p = mo.glorot_uniform(rng)
    layers = mo.unpack(p)
    for _, b in layers:
        b[:] = rng.uniform(-bias_scale, bias_scale, size=b.shape)
    return p.astype(np.float32)


def _inputs(n, seed=0, x_min=1e-4, x_max=1e2):
    x, u = plasma.sampler_inputs(n, seed=seed, x_min=x_min, x_max=x_max)
    return x.astype(np.float32), u.astype(np.float32)


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _host(t):
    return t.detach().cpu().numpy()


def _targets(mo, params, x, u, rng):
    """Targets near the network output (so MSE / MAE terms are O(0.1))."""
    y = mo.forward(params.astype(np.float64), x.astype(np.float64), u.astype(np.float64))
    return (y + rng.normal(0.0, 0.1, size=y.shape)).astype(np.float32)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 70001])
def test_forward_f32_matches_oracle(ctx, mlp_oracle, n):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 1)
    x, u = _inputs(n, seed=n)
    net = compton.MLP(ctx, params)
    _log(f"  forward f32 n={n}")
    y = _host(net.forward(_dev(x), _dev(u), "mlp_f32"))
    ref = mo.forward(params.astype(np.float64), x.astype(np.float64), u.astype(np.float64))
    err = np.abs(y - ref)
    # FP32 arithmetic through five layers of at most 64-term dot products
    # with O(1) activations: a few 1e-7 absolute; bound at the FP32 per-event
    # tolerance 1e-5.
    assert err.max() <= 1e-5, err.max()
    net.close()


def _layer_normwise(mo, g_gpu, g_ref):
    out = []
    o = 0
    for i in range(len(mo.WIDTHS) - 1):
        n = mo.WIDTHS[i] * mo.WIDTHS[i + 1] + mo.WIDTHS[i + 1]
        a, b = g_gpu[o:o + n], g_ref[o:o + n]
        out.append(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))
        o += n
    return out


@pytest.mark.parametrize("loss", ["mse", "mae"])
@pytest.mark.parametrize("n", [1, 100, 4096, 200003])
def test_grad_matches_oracle(ctx, mlp_oracle, loss, n):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 2)
    x, u = _inputs(n, seed=10 + n)
    t = _targets(mo, params, x, u, np.random.default_rng(n))
    net = compton.MLP(ctx, params)
    _log(f"  grad {loss} n={n}")
    l_gpu, g_gpu = net.grad(_dev(x), _dev(u), _dev(np.ascontiguousarray(t[:, 0])),
                            _dev(np.ascontiguousarray(t[:, 1])), loss=loss)
    l_ref, g_ref = mo.grad(params.astype(np.float64), x.astype(np.float64), u.astype(np.float64),
                           t.astype(np.float64), kind=loss)
    rel = _layer_normwise(mo, _host(g_gpu).astype(np.float64), g_ref)
    assert max(rel) <= 1e-5, rel
    assert abs(float(_host(l_gpu)) - l_ref) <= 1e-5 * abs(l_ref), (float(_host(l_gpu)), l_ref)
    net.close()


def test_grad_is_deterministic(ctx, mlp_oracle):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 3)
    x, u = _inputs(300000, seed=5)
    t = _targets(mo, params, x, u, np.random.default_rng(5))
    net = compton.MLP(ctx, params)
    args = (_dev(x), _dev(u), _dev(np.ascontiguousarray(t[:, 0])), _dev(np.ascontiguousarray(t[:, 1])))
    g1 = _host(net.grad(*args)[1])
    g2 = _host(net.grad(*args)[1])
    assert np.array_equal(g1, g2)
    net.close()


def test_adam_matches_oracle_and_train_step(ctx, mlp_oracle):
    """Three Adam steps on GPU gradients against the oracle's Adam fed the same
    gradients; train_step (fused gradient + update) gives the same bits as
    grad followed by adam_step."""
    import torch

    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 4)
    x, u = _inputs(4096, seed=6)
    t = _targets(mo, params, x, u, np.random.default_rng(6))
    args = (_dev(x), _dev(u), _dev(np.ascontiguousarray(t[:, 0])), _dev(np.ascontiguousarray(t[:, 1])))
    a = compton.MLP(ctx, params)
    b = compton.MLP(ctx, params)
    opt = mo.Adam(params.size, lr=1e-3)
    ref = params.astype(np.float64)
    for k in range(3):
        _, g = a.grad(*args)
        g_host = _host(g).astype(np.float64)
        a.adam_step(g, lr=1e-3)
        ref = opt.step(ref, g_host)
        got = a.get_params().astype(np.float64)
        # each update is lr * mhat / (sqrt(vhat) + eps) computed in FP32;
        # the difference is the FP32 rounding of the update and of the stored
        # parameter, well under 1e-7 absolute for |params| < 1.
        assert np.max(np.abs(got - ref)) <= 2e-7, (k, np.max(np.abs(got - ref)))
        # keep the oracle state on the GPU's FP32 parameters
        ref = got
        loss_t = torch.empty((), dtype=torch.float32, device="cuda:0")
        b.train_step(*args, lr=1e-3, loss="mse", loss_out=loss_t)
        assert np.array_equal(a.get_params(), b.get_params()), k
    a.close()
    b.close()


def test_first_adam_step_closed_form(ctx, mlp_oracle):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 8)
    x, u = _inputs(2048, seed=8)
    t = _targets(mo, params, x, u, np.random.default_rng(8))
    net = compton.MLP(ctx, params)
    args = (_dev(x), _dev(u), _dev(np.ascontiguousarray(t[:, 0])), _dev(np.ascontiguousarray(t[:, 1])))
    _, g = net.grad(*args)
    g = _host(g).astype(np.float64)
    net.adam_step(_dev(g.astype(np.float32)), lr=1e-3)
    got = net.get_params().astype(np.float64)
    expect = params.astype(np.float64) - 1e-3 * g / (np.abs(g) + 1e-8)
    assert np.max(np.abs(got - expect)) <= 2e-7
    net.close()


def test_loss_decreases(ctx, mlp_oracle):
    """Training on plain-sampler targets lowers the loss."""
    import torch

    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    rng = np.random.default_rng(9)
    params = mo.glorot_uniform(rng).astype(np.float32)
    x, u = _inputs(8192, seed=9)
    xd, ud = _dev(x), _dev(u)
    mu, r = ctx.sample_plain(xd, ud)
    net = compton.MLP(ctx, params)
    loss_t = torch.empty((), dtype=torch.float32, device="cuda:0")
    losses = []
    for k in range(300):
        net.train_step(xd, ud, mu, r, lr=1e-3, loss="mse", loss_out=loss_t)
        if k % 50 == 0 or k == 299:
            losses.append(float(loss_t.item()))
    _log(f"  losses {losses}")
    assert losses[-1] < 0.2 * losses[0], losses
    net.close()


def _act_amax(mo, params, x, u):
    """amax of the inputs of hidden layers 2..4 over the calibration set,
    indexed by layer (1..3) as forward_quantized expects."""
    _, hs, _ = mo.forward(params.astype(np.float64), x.astype(np.float64), u.astype(np.float64), keep=True)
    return {li: float(np.max(np.abs(hs[li]))) for li in (1, 2, 3)}


def _quant_errors(y_gpu, y_emu, y_ref):
    return (float(np.sqrt(np.mean((y_gpu - y_emu) ** 2))), float(np.max(np.abs(y_gpu - y_emu))),
            float(np.sqrt(np.mean((y_emu - y_ref) ** 2))))


@pytest.mark.parametrize("n", [1, 1000, 300001])
def test_forward_bf16_matches_emulation(ctx, mlp_oracle, n):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 11)
    x, u = _inputs(n, seed=20 + n)
    net = compton.MLP(ctx, params)
    net.quantize("mlp_bf16")
    y = _host(net.forward(_dev(x), _dev(u), "mlp_bf16")).astype(np.float64)
    p64, x64, u64 = params.astype(np.float64), x.astype(np.float64), u.astype(np.float64)
    emu = mo.forward_quantized(p64, x64, u64, "bf16")
    ref = mo.forward(p64, x64, u64)
    rms, mx, rms_q = _quant_errors(y, emu, ref)
    _log(f"  bf16 n={n}: rms(gpu-emu)={rms:.3e} max={mx:.3e} rms(emu-f64)={rms_q:.3e}")
    assert rms <= 2e-3 and mx <= 2e-2, (rms, mx)
    if n >= 1000:
        # the kernel reproduces the stated rounding: its distance to the
        # emulation is well under the rounding error itself
        assert rms <= 0.25 * rms_q, (rms, rms_q)
    net.close()


@pytest.mark.parametrize("n", [1, 1000, 300001])
def test_forward_fp8_matches_emulation(ctx, mlp_oracle, n):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 12)
    cx, cu = _inputs(65536, seed=99)
    x, u = _inputs(n, seed=30 + n)
    net = compton.MLP(ctx, params)
    net.quantize("mlp_fp8", _dev(cx), _dev(cu))
    y = _host(net.forward(_dev(x), _dev(u), "mlp_fp8")).astype(np.float64)
    p64, x64, u64 = params.astype(np.float64), x.astype(np.float64), u.astype(np.float64)
    amax = _act_amax(mo, params, cx, cu)
    emu = mo.forward_quantized(p64, x64, u64, "e4m3", act_scales=amax)
    ref = mo.forward(p64, x64, u64)
    rms, mx, rms_q = _quant_errors(y, emu, ref)
    _log(f"  fp8 n={n}: rms(gpu-emu)={rms:.3e} max={mx:.3e} rms(emu-f64)={rms_q:.3e}")
    assert rms <= 2e-2 and mx <= 2e-1, (rms, mx)
    if n >= 1000:
        assert rms <= 0.25 * rms_q, (rms, rms_q)
    net.close()


@pytest.mark.parametrize("precision", ["mlp_f32", "mlp_bf16", "mlp_fp8"])
def test_sample_reading_and_fallback(ctx, mlp_oracle, orc, precision):
    """mu = clamp(mu_hat, -1, 1), r = 1 / (1 + x (1 - mu)); outside the
    network's x domain the plain sampler answers and the mask says so."""
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 13)
    params[-2] = 0.962  # output bias of mu_hat: most outputs exceed 1
    params[-1] = 0.9  # output bias of the energy ratio: part of it inside (0, 1), where x > 1 reads it
    x, u = _inputs(5000, seed=40, x_min=1e-6, x_max=1e4)
    x[:3] = np.float32([1e-4, 1e2, 0.5])  # domain edges are inside
    net = compton.MLP(ctx, params)
    if precision == "mlp_fp8":
        cx, cu = _inputs(4096, seed=41)
        net.quantize(precision, _dev(cx), _dev(cu))
    elif precision == "mlp_bf16":
        net.quantize(precision)
    xd, ud = _dev(x), _dev(u)
    y = _host(net.forward(xd, ud, precision)).astype(np.float64)
    mu, r, mask = (_host(t) for t in net.sample(xd, ud, precision))
    inside = (x >= np.float32(1e-4)) & (x <= np.float32(1e2))
    assert np.array_equal(mask.astype(bool), ~inside)
    assert inside[:3].all()
    # the reading of the two outputs (the oracle's, in FP64; stored as FP32)
    mu_exp, r_exp = mo.sample_from_outputs(y[inside], x[inside].astype(np.float64))
    assert np.max(np.abs(mu[inside] - mu_exp)) <= 1e-7
    assert (np.abs(y[inside, 0]) > 1.0).any(), "test needs clamped outputs"
    xi = x[inside].astype(np.float64)
    assert ((xi > 1.0) & (np.abs(mu_exp - np.clip(y[inside, 0], -1, 1)) > 1e-3)).any(), "test needs ratio reads"
    assert np.max(np.abs(r[inside] - r_exp) / r_exp) <= 1e-6
    mu_o, r_o = orc.sample_plain(x[~inside].astype(np.float64), u[~inside].astype(np.float64))
    assert np.max(np.abs(mu[~inside] - mu_o)) <= 1e-6
    assert np.max(np.abs(r[~inside] - r_o) / r_o) <= 1e-6
    net.close()


def test_not_ready_and_invalidation(ctx, mlp_oracle):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 14)
    x, u = _inputs(100, seed=14)
    xd, ud = _dev(x), _dev(u)
    net = compton.MLP(ctx, params)
    for prec in ("mlp_bf16", "mlp_fp8"):
        with pytest.raises(compton.CSError) as ei:
            net.sample(xd, ud, prec)
        assert ei.value.code == compton.CS_ERR_NOT_READY
    net.quantize("mlp_bf16")
    net.sample(xd, ud, "mlp_bf16")
    with pytest.raises(compton.CSError) as ei:
        net.quantize("mlp_fp8")  # needs calibration inputs
    assert ei.value.code == compton.CS_ERR_INVALID_ARG
    net.set_params(params * 0.5)
    with pytest.raises(compton.CSError) as ei:
        net.sample(xd, ud, "mlp_bf16")
    assert ei.value.code == compton.CS_ERR_NOT_READY
    net.close()


def test_unsupported_widths(ctx):
    import ctypes as C

    from paper_2206_02937_amd import compton

    w = (C.c_int32 * 4)(2, 9, 12, 1)
    h = C.c_void_p()
    rc = compton.lib().cs_mlp_create(ctx.handle, w, 4, None, C.byref(h))
    assert rc == compton.CS_ERR_UNSUPPORTED and not h.value


def test_save_load_roundtrip(ctx, mlp_oracle, tmp_path):
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    params = _params(mo, 15)
    x, u = _inputs(4096, seed=15)
    t = _targets(mo, params, x, u, np.random.default_rng(15))
    args = (_dev(x), _dev(u), _dev(np.ascontiguousarray(t[:, 0])), _dev(np.ascontiguousarray(t[:, 1])))
    a = compton.MLP(ctx, params)
    for _ in range(3):
        a.train_step(*args, lr=1e-3)
    path = str(tmp_path / "net.bin")
    a.save(path)
    b = compton.MLP.load(ctx, path)
    assert np.array_equal(a.get_params(), b.get_params())
    # the Adam state and step count travel too: the next step agrees bitwise
    a.train_step(*args, lr=1e-3)
    b.train_step(*args, lr=1e-3)
    assert np.array_equal(a.get_params(), b.get_params())
    raw = bytearray(open(path, "rb").read())
    raw[100] ^= 0x01
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    with pytest.raises(compton.CSError) as ei:
        compton.MLP.load(ctx, bad)
    assert ei.value.code == compton.CS_ERR_IO
    short = str(tmp_path / "short.bin")
    open(short, "wb").write(bytes(raw[:-9]))
    with pytest.raises(compton.CSError) as ei:
        compton.MLP.load(ctx, short)
    assert ei.value.code == compton.CS_ERR_IO
    with pytest.raises(compton.CSError):
        compton.MLP.load(ctx, str(tmp_path / "missing.bin"))
    a.close()
    b.close()


def test_custom_x_range(ctx, mlp_oracle, tmp_path):
    """A network trained for another x range: the features map that range onto
    [-1, 1] (FP32 forward against the oracle with the same range), samples
    outside it go to the plain sampler, the range travels with save / load,
    and a file without a range loads with the default one."""
    from paper_2206_02937_amd import compton

    mo = mlp_oracle
    lo, hi = 1e-8, 1e3
    params = _params(mo, 16)
    net = compton.MLP(ctx, params)
    assert net.domain == (compton.X_MIN, compton.X_MAX)
    net.set_domain(lo, hi)
    assert net.domain == (lo, hi)
    x, u = _inputs(5000, seed=50, x_min=1e-9, x_max=1e4)
    x[:2] = np.float32([lo, hi])
    y = _host(net.forward(_dev(x), _dev(u), "mlp_f32")).astype(np.float64)
    ref = mo.forward(params.astype(np.float64), x.astype(np.float64), u.astype(np.float64), domain=(lo, hi))
    assert np.max(np.abs(y - ref)) <= 1e-5
    net.quantize("mlp_bf16")
    yb = _host(net.forward(_dev(x), _dev(u), "mlp_bf16")).astype(np.float64)
    emu = mo.forward_quantized(params.astype(np.float64), x.astype(np.float64), u.astype(np.float64), "bf16",
                               domain=(lo, hi))
    assert np.sqrt(np.mean((yb - emu) ** 2)) <= 2e-3
    _, _, mask = (_host(t) for t in net.sample(_dev(x), _dev(u), "mlp_bf16"))
    inside = (x >= np.float32(lo)) & (x <= np.float32(hi))
    assert np.array_equal(mask.astype(bool), ~inside) and (~inside).any() and inside[:2].all()
    path = str(tmp_path / "ranged.csnet")
    net.save(path)
    back = compton.MLP.load(ctx, path)
    assert back.domain == (lo, hi) and np.array_equal(back.get_params(), net.get_params())
    shipped = compton.MLP.load(ctx, os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                                 "paper_2206_02937_amd", "weights", "sampler_2x64x4.csnet"))
    assert shipped.domain[0] > 0
    for bad in ((0.0, 1.0), (1.0, 1.0), (2.0, 1.0), (1e-3, float("inf"))):
        with pytest.raises(compton.CSError):
            net.set_domain(*bad)
    assert net.domain == (lo, hi)
    # the FP8 copy is recalibrated after a range change
    cx, cu = _inputs(4096, seed=51)
    net.quantize("mlp_fp8", _dev(cx), _dev(cu))
    net.set_domain(1e-6, 1e2)
    with pytest.raises(compton.CSError) as ei:
        net.sample(_dev(x), _dev(u), "mlp_fp8")
    assert ei.value.code == compton.CS_ERR_NOT_READY
    for n_ in (net, back, shipped):
        n_.close()
