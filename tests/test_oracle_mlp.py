"""Pins of the MLP oracle: gradients against central finite differences,
Adam's first step against its closed form, loss decrease on a toy problem,
a hand-computed one-unit network, and the reduced-precision rounding
emulation against PyTorch's own bfloat16 / float8_e4m3fn conversions."""
import numpy as np
import pytest
import torch

from oracle import mlp_oracle as M


def small_widths():
    return (2, 5, 4, 2)


def test_param_count():
    assert M.n_params() == 12802
    assert M.n_params(small_widths()) == 2 * 5 + 5 + 5 * 4 + 4 + 4 * 2 + 2


def test_one_unit_network_by_hand():
    widths = (2, 1, 1)
    # W1 = [a, b], b1 = c; W2 = [d], b2 = e
    a, b, c, d, e = 0.7, -1.3, 0.2, 2.5, -0.4
    params = np.array([a, b, c, d, e])
    x, u = np.array([10.0]), np.array([0.25])
    f1, f2 = (1.0 + 1.0) / 3.0, -0.5
    z = a * f1 + b * f2 + c
    h = z / (1.0 + np.exp(-z))
    y = M.forward(params, x, u, widths)
    assert y.shape == (1, 1)
    assert abs(y[0, 0] - (d * h + e)) < 1e-15


def test_feature_map_over_an_x_range():
    """log10 x maps linearly from the network's x range onto [-1, 1]: the
    range's ends go to -1 and +1, its log-midpoint to 0; the default range
    [1e-4, 1e2] gives (log10 x + 1) / 3 (x = 10 -> 2/3, as by hand above)."""
    for lo, hi in ((1e-4, 1e2), (1e-8, 1e3), (0.5, 2.0)):
        mid = np.sqrt(lo * hi)
        f = M.features(np.array([lo, mid, hi]), np.array([0.0, 0.5, 0.75]), domain=(lo, hi))
        assert np.allclose(f[:, 0], [-1.0, 0.0, 1.0], rtol=0, atol=1e-15)
        assert np.array_equal(f[:, 1], [-1.0, 0.0, 0.5])
    x = np.array([1e-4, 3e-2, 10.0, 1e2])
    assert np.allclose(M.features(x, np.zeros(4))[:, 0], (np.log10(x) + 1.0) / 3.0, rtol=0, atol=1e-15)
    # the range enters only through the features
    p = M.glorot_uniform(np.random.default_rng(3))
    xs = np.array([1e-7, 1e-3, 5e2])
    us = np.array([0.1, 0.5, 0.9])
    lo, hi = 1e-8, 1e3
    f1 = (np.log10(xs) + 2.5) / 5.5
    x_equiv = 10.0 ** (3.0 * f1 - 1.0)  # the x with the same f1 under the default range
    assert np.allclose(M.forward(p, xs, us, domain=(lo, hi)), M.forward(p, x_equiv, us), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("kind", ["mse", "mae"])
def test_gradient_vs_central_differences(kind):
    rng = np.random.default_rng(0)
    widths = small_widths()
    params = M.glorot_uniform(rng, widths) + 0.05 * rng.normal(size=M.n_params(widths))
    x = np.exp(rng.uniform(np.log(1e-4), np.log(1e2), 37))
    u = rng.random(37)
    t = rng.normal(size=(37, 2))
    L, g = M.grad(params, x, u, t, kind, widths)
    h = 1e-6
    for i in range(params.size):
        pp = params.copy()
        pm = params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss(M.forward(pp, x, u, widths), t, kind) - M.loss(M.forward(pm, x, u, widths), t, kind)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + (1e-6 if kind == "mae" else 0), i
    assert abs(L - M.loss(M.forward(params, x, u, widths), t, kind)) < 1e-15


def test_gradient_full_size_spot_check():
    rng = np.random.default_rng(1)
    params = M.glorot_uniform(rng)
    x = np.exp(rng.uniform(np.log(1e-4), np.log(1e2), 64))
    u = rng.random(64)
    t = rng.normal(size=(64, 2))
    _, g = M.grad(params, x, u, t)
    for i in rng.choice(params.size, 40, replace=False):
        h = 1e-6
        pp = params.copy()
        pm = params.copy()
        pp[i] += h
        pm[i] -= h
        fd = (M.loss(M.forward(pp, x, u), t) - M.loss(M.forward(pm, x, u), t)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i]))


def test_adam_first_step_closed_form():
    """With m = v = 0, the first bias-corrected step is -lr g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    g = rng.normal(size=100) * np.logspace(-9, 1, 100)
    p = rng.normal(size=100)
    opt = M.Adam(100, lr=1e-3)
    p1 = opt.step(p, g)
    assert np.allclose(p1 - p, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_second_step_closed_form():
    g1, g2 = np.array([0.3, -2.0]), np.array([0.1, 1.0])
    opt = M.Adam(2, lr=0.01)
    p = opt.step(np.zeros(2), g1)
    p = opt.step(p, g2)
    m = 0.1 * (0.9 * g1 + g2) / (1 - 0.81)
    v = 0.001 * (0.999 * g1**2 + g2**2) / (1 - 0.999**2)
    step1 = -0.01 * g1 / (np.abs(g1) + 1e-8)
    assert np.allclose(p, step1 - 0.01 * m / (np.sqrt(v) + 1e-8), rtol=1e-12)


def test_training_reduces_loss_on_toy_problem():
    rng = np.random.default_rng(4)
    widths = (2, 16, 16, 2)
    params = M.glorot_uniform(rng, widths)
    x = np.exp(rng.uniform(np.log(1e-4), np.log(1e2), 512))
    u = rng.random(512)
    t = np.stack([np.sin(2 * u), np.log10(x) / 10], axis=1)
    opt = M.Adam(params.size, lr=1e-2)
    L0 = M.loss(M.forward(params, x, u, widths), t)
    for _ in range(300):
        _, g = M.grad(params, x, u, t, "mse", widths)
        params = opt.step(params, g)
    L1 = M.loss(M.forward(params, x, u, widths), t)
    assert L1 < 0.05 * L0


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.normal(size=20000) * np.exp(rng.uniform(-20, 20, 20000)),
                        [0.0, -0.0, 1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-9, 3.0e38, -1e-40]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.round_bf16(a), ref)


def test_e4m3_rounding_matches_torch():
    rng = np.random.default_rng(6)
    a = np.concatenate([rng.normal(size=20000) * np.exp(rng.uniform(-12, 6, 20000)),
                        M._E4M3, -M._E4M3, (M._E4M3[1:] + M._E4M3[:-1]) / 2])
    a = a[np.abs(a) <= 448.0]
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = M.round_e4m3(a.astype(np.float32).astype(np.float64))
    assert np.array_equal(got, ref)
    # saturation (the saturating conversion mode) and the format's extremes
    assert M.round_e4m3(np.array([1000.0, -500.0]))[0] == 448.0
    assert M.round_e4m3(np.array([1000.0, -500.0]))[1] == -448.0
    assert M._E4M3.max() == 448.0 and M._E4M3[1] == 2.0**-9


def test_sample_reading_of_outputs():
    """x <= 1: the cosine output, clamped; x > 1: the energy-ratio output where
    it fixes v = 1 - cos theta better (v_r < (sqrt x - 1) / x), else the
    cosine; the ratio is always recomputed from v (Compton relation)."""
    y = np.array([[1.3, 0.5], [-0.2, 0.9], [-4.0, 0.1], [0.3, 0.02], [0.3, 0.95], [0.1, 1.2]])
    x = np.array([0.5, 2.0, 1e-3, 100.0, 100.0, 50.0])
    mu, r = M.sample_from_outputs(y, x)
    v_r = lambda rr, xx: (1.0 / rr - 1.0) / xx  # noqa: E731
    expect = np.array([1.0, 1.0 - v_r(0.9, 2.0), -1.0, 0.3, 1.0 - v_r(0.95, 100.0), 1.0])
    assert np.allclose(mu, expect, rtol=0, atol=1e-15)
    assert np.allclose(r, 1 / (1 + x * (1 - mu)), rtol=1e-15)


def test_sample_reading_takes_the_better_conditioned_output():
    """Outputs off the exact event by at most e each: the reading's error in
    v is at most the larger of the two outputs' propagated errors at the
    crossover (both equal e there), and where x v is small against sqrt(x)
    it is far below e (the ratio carries the forward scatters of large x)."""
    rng = np.random.default_rng(8)
    e = 1e-3
    for x in (0.3, 2.0, 30.0, 1e3):
        v = rng.uniform(0.0, 2.0, 20000) ** 3 / 4.0  # many small angles
        mu_t, r_t = 1.0 - v, 1.0 / (1.0 + x * v)
        y = np.stack([mu_t + rng.uniform(-e, e, v.size), r_t + rng.uniform(-e, e, v.size)], axis=1)
        err = np.abs(M.reading_v(y, np.full(v.size, x)) - v)
        assert err.max() <= 1.02 * e, (x, err.max())
        if x > 100:
            small = v < 0.01 / np.sqrt(x)
            assert small.any() and err[small].max() <= 2e-5 * e * x, (x, err[small].max())


def test_bf16_emulation_by_hand():
    """One unit per layer: the BF16 network rounds the hidden layer's weight
    and its input -log2(e) SiLU(z) to bfloat16 (the scale undone after), the
    first and last layers stay in float64."""
    widths = (2, 1, 1, 1)
    params = np.array([0.7, -1.3, 0.2, 1.2345678, -0.1, 2.5, -0.4])  # W1[2], b1, W2, b2, W3, b3
    x, u = np.array([10.0]), np.array([0.25])
    f1, f2 = 2.0 / 3.0, -0.5
    z1 = 0.7 * f1 - 1.3 * f2 + 0.2
    h1 = z1 / (1.0 + np.exp(-z1))
    c = -np.log2(np.e)
    q = M.round_bf16(c * h1)[()] / c
    z2 = q * M.round_bf16(1.2345678)[()] - 0.1
    h2 = z2 / (1.0 + np.exp(-z2))
    y = M.forward_quantized(params, x, u, "bf16", widths=widths)
    assert abs(y[0, 0] - (2.5 * h2 - 0.4)) < 1e-15
    assert q != M.round_bf16(h1)[()]  # the scale changes the rounding here
