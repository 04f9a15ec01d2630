"""FP64 oracle of the paper's own learned component, the probability network
(Sec. 3.2) -- TEST INFRASTRUCTURE ONLY, like the rest of this package.

The paper trains a small dense network to predict, for a candidate
lepton-photon pair, the probability of interaction in place of the analytic
Klein-Nishina evaluation.  Readings (the text leaves them open):

* inputs, nine per pair, in code units: the photon momentum k (3), the
  lepton momentum p (3), the majorant P_max of the pair's cell, and the two
  macro-particle weights w_e, w_g -- the union of the lists the paper gives
  for the network and for its data;
* output: y' = P / P_max in [0, 1], the acceptance ratio against the
  majorant, which the sigmoid output fits;
* widths 9 -> 9 -> 12 -> 9 -> 1: three hidden ReLU layers, a sigmoid output;
  ReLU'(0) taken as 0;
* loss MAE (the paper's) or MSE, Adam with the paper's learning rate 1e-3.

With P = tau w_max s(x) (1 - beta . k_hat) and P_max = 2 tau w_max (the
pair probability of the step and its bound), the target is
y = s(x) flux / 2, flux = x / (gamma eps), whatever the weights and tau.

Parameter layout (flat vector, the GPU library's): per layer the weight
matrix W[n_out, n_in] row-major, then the bias b[n_out].  Plain numpy
float64; every layer a matrix product written out.
"""
import numpy as np

import oracle as _orc

WIDTHS = (9, 9, 12, 9, 1)


def n_params(widths=WIDTHS):
    return sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))


def unpack(params, widths=WIDTHS):
    params = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        W = params[o:o + n_in * n_out].reshape(n_out, n_in)
        o += n_in * n_out
        b = params[o:o + n_out]
        o += n_out
        out.append((W, b))
    assert o == params.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def inputs(k, p, p_max, w_e, w_g):
    """Rows of the nine inputs: k (3), p (3), P_max, w_e, w_g."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
    n = k.shape[0]
    col = lambda v: np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)).reshape(n, 1)
    return np.concatenate([k, p, col(p_max), col(w_e), col(w_g)], axis=1)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, X, keep=False):
    """y' for each row of X; with keep, also the pre-activations and
    activations of every layer (for the backward pass)."""
    layers = unpack(params)
    a = np.asarray(X, dtype=np.float64)
    acts, pres = [a], []
    for i, (W, b) in enumerate(layers):
        z = a @ W.T + b
        pres.append(z)
        a = np.maximum(z, 0.0) if i < len(layers) - 1 else sigmoid(z)
        acts.append(a)
    y = a[:, 0]
    return (y, pres, acts) if keep else y


def loss(y, t, kind="mae"):
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    return float(np.mean(np.abs(d))) if kind == "mae" else float(0.5 * np.mean(d * d))


def grad(params, X, t, kind="mae"):
    """(gradient of the mean loss over the rows, loss), by the chain rule
    through each layer; d|e|/de taken as sign(e) (0 at 0)."""
    y, pres, acts = forward(params, X, keep=True)
    n = y.size
    e = y - np.asarray(t, dtype=np.float64)
    dy = (np.sign(e) if kind == "mae" else e) / n
    layers = unpack(params)
    # output: y = sigmoid(z), dy/dz = y (1 - y)
    delta = (dy * y * (1.0 - y))[:, None]
    grads = []
    for i in range(len(layers) - 1, -1, -1):
        W, _ = layers[i]
        a_prev = acts[i]
        grads.append((delta.T @ a_prev, delta.sum(axis=0)))
        if i > 0:
            delta = (delta @ W) * (pres[i - 1] > 0.0)
    grads.reverse()
    return pack(grads), loss(y, t, kind)


def adam_step(params, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), step number t >= 1, bias-corrected."""
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return np.asarray(params, dtype=np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def target_ratio(k, p):
    """y = P / P_max = s(x) flux / 2 of each pair, from the oracle's
    rest-frame invariants and cross-section."""
    k = np.asarray(k, dtype=np.float64).reshape(-1, 3)
    p = np.asarray(p, dtype=np.float64).reshape(-1, 3)
    out = np.empty(k.shape[0])
    for i in range(k.shape[0]):
        x, flux = _orc.pair_invariants(p[i], k[i])
        out[i] = 0.5 * _orc.sigma_ratio(x) * flux if x > 0.0 else 0.0
    return out


def glorot_uniform(rng, widths=WIDTHS):
    layers = []
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        lim = np.sqrt(6.0 / (n_in + n_out))
        layers.append((rng.uniform(-lim, lim, size=(n_out, n_in)), np.zeros(n_out)))
    return pack(layers)
