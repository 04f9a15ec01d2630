"""Pins of the probability-network oracle: gradients against central finite
differences (MSE, and MAE away from its kinks), a network with all
parameters zero (output sigmoid(0) = 1/2 and its gradient by hand), Adam's
first step against its closed form, the parameter count of the 9-9-12-9-1
network, and the target y = P / P_max in limits the physics fixes."""
import numpy as np
import pytest

import oracle
from oracle import pnet_oracle as N


def _data(rng, n=16):
    k = rng.standard_normal((n, 3)) * 0.3
    p = rng.standard_normal((n, 3)) * 2.0
    X = N.inputs(k, p, rng.uniform(0.01, 0.5, n), rng.uniform(0.5, 2, n), rng.uniform(0.5, 2, n))
    return X


def test_param_count():
    assert N.n_params() == 9 * 9 + 9 + 9 * 12 + 12 + 12 * 9 + 9 + 9 + 1 == 337


@pytest.mark.parametrize("kind", ["mse", "mae"])
def test_grad_matches_finite_differences(kind):
    rng = np.random.default_rng(1)
    params = N.glorot_uniform(rng) + rng.normal(0, 0.05, N.n_params())
    X = _data(rng)
    t = rng.uniform(0.0, 1.0, X.shape[0])
    if kind == "mae":
        # keep |y - t| away from zero so the loss is smooth around params
        t = np.where(N.forward(params, X) > 0.5, 0.0, 1.0)
    g, _ = N.grad(params, X, t, kind)
    h = 1e-6
    for j in rng.choice(N.n_params(), size=60, replace=False):
        e = np.zeros_like(params)
        e[j] = h
        num = (N.loss(N.forward(params + e, X), t, kind) - N.loss(N.forward(params - e, X), t, kind)) / (2 * h)
        assert abs(num - g[j]) <= 1e-6 * max(1.0, abs(num)), (j, num, g[j])


def test_zero_network_by_hand():
    params = np.zeros(N.n_params())
    X = _data(np.random.default_rng(2), 5)
    t = np.array([0.0, 1.0, 0.25, 0.5, 0.75])
    y = N.forward(params, X)
    assert np.all(y == 0.5)
    g, l = N.grad(params, X, t, "mse")
    assert l == pytest.approx(0.5 * np.mean((0.5 - t) ** 2))
    # only the output bias sees a gradient: mean(y - t) * sigmoid'(0), sigmoid'(0) = 1/4
    assert g[-1] == pytest.approx(np.mean(0.5 - t) * 0.25)
    assert np.all(g[:-1] == 0.0)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(3)
    p0 = rng.standard_normal(10)
    g = rng.standard_normal(10)
    p1, m, v = N.adam_step(p0, g, np.zeros(10), np.zeros(10), 1, lr=1e-3)
    # bias-corrected m / sqrt(v) = g / |g| on the first step
    assert np.allclose(p1, p0 - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_target_limits():
    # lepton at rest, low-energy photon: x = eps, flux = 1, s -> 1: y -> 1/2
    y = N.target_ratio([[1e-6, 0, 0]], [[0, 0, 0]])
    assert y[0] == pytest.approx(0.5, rel=1e-5)
    # lepton at rest: y = s(eps) / 2 exactly
    eps = np.array([0.01, 0.3, 2.0, 40.0])
    k = np.stack([eps, 0 * eps, 0 * eps], axis=1)
    y = N.target_ratio(k, np.zeros_like(k))
    assert np.allclose(y, [0.5 * oracle.sigma_ratio(e) for e in eps], rtol=1e-15)
    # photon moving along a fast lepton (p . k > 0, head-away): flux = 1 - beta < 1/(2 gamma^2)
    p = np.array([[0.0, 0.0, 50.0]])
    y_par = N.target_ratio([[0, 0, 0.01]], p)
    gam = np.sqrt(1 + 50.0 ** 2)
    assert 0 < y_par[0] <= 0.5 / (2 * gam * gam) * 1.0001
    # head-on: flux = 1 + beta, so y is larger than at rest for the same rest-frame x
    y_ho = N.target_ratio([[0, 0, -1e-4]], p)
    assert y_ho[0] > 0.5 * 0.99 * oracle.sigma_ratio(gam * 1e-4 * 2)
    assert y_ho[0] <= 1.0


def test_outputs_in_unit_interval():
    rng = np.random.default_rng(4)
    params = N.glorot_uniform(rng)
    y = N.forward(params, _data(rng, 200))
    assert np.all((y > 0) & (y < 1))
