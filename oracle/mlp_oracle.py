"""FP64 oracle of the sampler MLP -- TEST INFRASTRUCTURE ONLY.

The learned part stands in for the inverse-CDF angle/energy sampling: a fully
connected network (the paper's Sec. 3.2 uses dense layers, Adam, and trains on
data the conventional method produced) maps (x, u) to (cos theta, eps'/eps).

Plain numpy float64; every layer is a matrix product written out, no fusion.

Parameter layout (flat vector, the same order the GPU library uses at its
boundary): for each layer l with fan-in n_in and fan-out n_out, the weight
matrix W_l[n_out, n_in] row-major, then the bias b_l[n_out].

Features (a reading: the paper gives none for this network):
    f1 = (log10 x - c) / h      maps log10 x linearly from the network's x
                                range [x_min, x_max] onto [-1, 1]:
                                c, h = midpoint and half-width of
                                [log10 x_min, log10 x_max]; the default range
                                [1e-4, 1e2] gives f1 = (log10 x + 1) / 3
    f2 = 2 u - 1
Hidden layers: SiLU z * sigmoid(z); output layer linear.
Loss: MSE = 1/(2n) sum (y - t)^2 over the n samples and both outputs, or
MAE = 1/(2n) sum |y - t| (the paper's choice, Sec. 3.2).
Adam (Kingma & Ba): beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; the
paper's learning rate 1e-3 is the default.
"""
import numpy as np

X_MIN = 1e-4
X_MAX = 1e2
WIDTHS = (2, 64, 64, 64, 64, 2)


def n_params(widths=WIDTHS):
    return sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(len(widths) - 1))


def unpack(params, widths=WIDTHS):
    """Flat vector -> list of (W, b) views."""
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


def features(x, u, domain=(X_MIN, X_MAX)):
    x = np.asarray(x, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    lo, hi = np.log10(domain[0]), np.log10(domain[1])
    c, h = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return np.stack([(np.log10(x) - c) / h, 2.0 * u - 1.0], axis=1)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, u, widths=WIDTHS, keep=False, domain=(X_MIN, X_MAX)):
    """Network outputs y[n, 2] (raw: mu_hat, r_hat).  With keep=True also the
    per-layer inputs and pre-activations needed by the backward pass."""
    layers = unpack(params, widths)
    h = features(x, u, domain)
    hs, zs = [h], []
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        zs.append(z)
        h = silu(z) if li < len(layers) - 1 else z
        hs.append(h)
    if keep:
        return h, hs, zs
    return h


def loss(y, t, kind="mse"):
    n = y.shape[0]
    d = y - t
    if kind == "mse":
        return float(np.sum(d * d) / (2.0 * n))
    if kind == "mae":
        return float(np.sum(np.abs(d)) / (2.0 * n))
    raise ValueError(kind)


def grad(params, x, u, t, kind="mse", widths=WIDTHS, domain=(X_MIN, X_MAX)):
    """Loss and its gradient with respect to the flat parameter vector."""
    y, hs, zs = forward(params, x, u, widths, keep=True, domain=domain)
    n = y.shape[0]
    d = y - t
    if kind == "mse":
        dy = d / n
    elif kind == "mae":
        dy = np.sign(d) / (2.0 * n)
    else:
        raise ValueError(kind)
    layers = unpack(params, widths)
    grads = [None] * len(layers)
    delta = dy
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        if li < len(layers) - 1:
            delta = delta * silu_grad(zs[li])
        gW = delta.T @ hs[li]
        gb = delta.sum(axis=0)
        grads[li] = (gW, gb)
        delta = delta @ W
    return loss(y, t, kind), pack(grads)


class Adam:
    """Adam with bias correction; state m, v and step count t."""

    def __init__(self, n, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, params, g, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return params - lr * mhat / (np.sqrt(vhat) + self.eps)


def glorot_uniform(rng, widths=WIDTHS):
    """Glorot-uniform weights, zero biases (the Keras defaults)."""
    layers = []
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        lim = np.sqrt(6.0 / (n_in + n_out))
        layers.append((rng.uniform(-lim, lim, size=(n_out, n_in)), np.zeros(n_out)))
    return pack(layers)


def reading_v(y, x):
    """The sampler's reading of the two outputs (cos theta, eps'/eps) as
    v = 1 - cos theta (a reading: both outputs are trained, the configuration
    lists both).  With the same absolute error e in either output, cos theta
    fixes v to e, while eps'/eps = r = 1 / (1 + x v) fixes it to
    e (1 + x v)^2 / x; so v comes from the ratio (clamped to its range
    [1 / (1 + 2x), 1]) where that is smaller -- x > 1 and
    v_r < (sqrt(x) - 1) / x, i.e. r > 1 / sqrt(x) -- and from the cosine
    (clamped to [-1, 1]) elsewhere.  x: the network's FP32 input, as
    float64."""
    y = np.asarray(y, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    v_mu = 1.0 - np.clip(y[:, 0], -1.0, 1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.clip(y[:, 1], 1.0 / (1.0 + 2.0 * x), 1.0)
        v_r = (1.0 - r) / (r * x)
        # v_r < (sqrt(x) - 1) / x  <=>  1 + x v_r < sqrt(x)  <=>  r > 1 / sqrt(x)
        use_r = (x > 1.0) & (r * r * x > 1.0)
    return np.where(use_r, v_r, v_mu)


def sample_from_outputs(y, x):
    """Sampler reading of the network output: v from reading_v, mu = 1 - v,
    and the energy ratio recomputed from v so that the Compton relation
    holds."""
    v = reading_v(y, x)
    return 1.0 - v, 1.0 / (1.0 + np.asarray(x, dtype=np.float64) * v)


# ----------------------------------------------------------------------------
# Reduced-precision emulation (for stating BF16 / FP8 error separately from
# the approximation error).  Rounding is to nearest, ties to even.
# ----------------------------------------------------------------------------
def round_bf16(a):
    """Round to bfloat16 (8 exponent bits, 7 stored mantissa bits), RNE.
    Values are first rounded to float32 (exact for float32 input)."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    out[nan] = np.nan
    return out.reshape(np.shape(a))


def _e4m3_table():
    """All non-negative finite OCP FP8 E4M3 values (bias 7, max 448), by code."""
    vals = []
    for code in range(0x7F):  # 0x7F is NaN
        e = code >> 3
        m = code & 7
        if e == 0:
            v = (m / 8.0) * 2.0 ** (-6)
        else:
            v = (1.0 + m / 8.0) * 2.0 ** (e - 7)
        vals.append(v)
    return np.array(vals)


_E4M3 = _e4m3_table()
E4M3_MAX = 448.0


def round_e4m3(a):
    """Round to OCP FP8 E4M3, nearest with ties to the even code, saturating
    at +-448 (the saturating conversion mode)."""
    a = np.asarray(a, dtype=np.float64)
    mag = np.minimum(np.abs(a), E4M3_MAX)
    idx = np.searchsorted(_E4M3, mag)  # first table value >= mag
    idx = np.clip(idx, 1, _E4M3.size - 1)
    lo = _E4M3[idx - 1]
    hi = _E4M3[idx]
    pick_hi = (hi - mag < mag - lo) | ((hi - mag == mag - lo) & ((idx % 2) == 0))
    q = np.where(pick_hi, hi, lo)
    q = np.where(mag == 0.0, 0.0, q)
    return np.copysign(q, a)


# The BF16 network rounds its hidden-layer inputs scaled by -log2(e) (a
# reading of the reduced-precision scheme: the kernel carries SiLU's
# exponential argument t = -log2(e) z, so the value it rounds is -log2(e)
# SiLU(z)); the factor is undone exactly in the next layer.
SILU_SCALE = -np.log2(np.e)


def forward_quantized(params, x, u, fmt, act_scales=None, widths=WIDTHS, domain=(X_MIN, X_MAX)):
    """Forward pass with the hidden-layer contractions in reduced precision:
    'bf16' rounds the weights and the layer inputs (scaled by SILU_SCALE,
    then unscaled) to bfloat16; 'e4m3' divides them by per-layer scales
    (weights: amax/448; inputs: the given calibrated amax/448) and rounds to
    FP8 E4M3.  Products and sums in float64, bias and activation in float64.
    The first (2 -> 64) and last (64 -> 2) layers stay in full precision, as
    in the GPU kernel."""
    layers = unpack(params, widths)
    h = features(x, u, domain)
    nl = len(layers)
    for li, (W, b) in enumerate(layers):
        if 0 < li < nl - 1:
            if fmt == "bf16":
                z = (round_bf16(SILU_SCALE * h) / SILU_SCALE) @ round_bf16(W).T + b
            elif fmt == "e4m3":
                sw = np.max(np.abs(W)) / E4M3_MAX
                sh = act_scales[li] / E4M3_MAX
                z = (round_e4m3(h / sh) @ round_e4m3(W / sw).T) * (sw * sh) + b
            else:
                raise ValueError(fmt)
        else:
            z = h @ W.T + b
        h = silu(z) if li < nl - 1 else z
    return h
