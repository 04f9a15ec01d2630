"""Train the sampler network on the GPU with the library's own kernels.

    python -m paper_2206_02937_amd.train_sampler [--out PATH] [--samples N]
        [--batch B] [--epochs E] [--lr LR] [--loss mse|mae] [--seed S]
        [--x-min X0 --x-max X1]

Data: N inputs (x log-uniform on the network's x range [X0, X1], by default
[1e-8, 1e3]; u uniform on [0, 1)) with targets (cos theta, eps'/eps) from the
plain inverse-CDF sampler on the GPU (FP64 arithmetic, stored as FP32); the
network's first feature maps that range onto [-1, 1] and outside it the plain
sampler answers.  The first 80 % train, the last 20 %
validate (the paper's split, Sec. 3.2).  Optimiser: Adam (the paper's
learning rate 1e-3 as the peak), cosine decay to 1 % of it; Glorot-uniform
initial weights, zero biases.  Each epoch visits the training batches in a
new random order.  The result is written with cs_mlp_save; a JSON summary
(loss curve, validation error, KS distances) goes to stdout.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "weights", "sampler_2x64x4.csnet")
X_RANGE = (1e-8, 1e3)  # rest-frame photon energies of the workloads, power-law and beam plasmas included


def glorot_params(seed, widths=(2, 64, 64, 64, 64, 2)):
    """Flat parameter vector: per layer W[n_out, n_in] (Glorot uniform), then
    zero biases."""
    rng = np.random.default_rng([seed, 101])
    parts = []
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        lim = math.sqrt(6.0 / (n_in + n_out))
        parts.append(rng.uniform(-lim, lim, size=n_out * n_in))
        parts.append(np.zeros(n_out))
    return np.concatenate(parts).astype(np.float32)


def make_data(ctx, n, seed, x_range=X_RANGE):
    import torch

    from . import plasma

    x, u = plasma.sampler_inputs(n, seed=seed, x_min=x_range[0], x_max=x_range[1])
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    mu, r = ctx.sample_plain(xd, ud)
    torch.cuda.synchronize()
    return xd, ud, mu, r


def evaluate(net, xd, ud, mu, r, precision="mlp_f32"):
    """Validation MAE of both outputs and KS distances of the sampled
    cos(theta) and energy ratio against the plain sampler's."""
    from .sampler_quality import ks_distance

    y = net.forward(xd, ud, precision).cpu().numpy().astype(np.float64)
    m_hat, r_hat, _ = net.sample(xd, ud, precision)
    mu_h, r_h = mu.cpu().numpy().astype(np.float64), r.cpu().numpy().astype(np.float64)
    return {
        "mae_mu": float(np.mean(np.abs(y[:, 0] - mu_h))),
        "mae_r": float(np.mean(np.abs(y[:, 1] - r_h))),
        "ks_mu": ks_distance(m_hat.cpu().numpy(), mu_h),
        "ks_r": ks_distance(r_hat.cpu().numpy(), r_h),
    }


def train(ctx, n=1 << 24, batch=4096, epochs=60, lr=1e-3, loss="mse", seed=0, log=print, init=None,
          x_range=X_RANGE, eval_every=10):
    """Returns (network, summary dict)."""
    import torch

    from . import compton

    xd, ud, mu, r = make_data(ctx, n, seed, x_range)
    n_train = int(0.8 * n)
    n_batches = (n_train - batch) // batch + 1
    net = compton.MLP(ctx, glorot_params(seed) if init is None else init)
    net.set_domain(*x_range)
    losses = torch.zeros(n_batches, dtype=torch.float32, device=xd.device)
    rng = np.random.default_rng([seed, 202])
    hist = []
    t0 = time.time()
    val = slice(n_train, n)
    for ep in range(epochs):
        lr_ep = lr * (0.01 + 0.99 * 0.5 * (1.0 + math.cos(math.pi * ep / max(1, epochs - 1))))
        start = int(rng.integers(0, n_train - n_batches * batch + 1))
        for i, b in enumerate(rng.permutation(n_batches)):
            s = slice(start + b * batch, start + (b + 1) * batch)
            net.train_step(xd[s], ud[s], mu[s], r[s], lr=lr_ep, loss=loss, loss_out=losses[i])
        mean_loss = float(losses.mean().item())
        rec = {"epoch": ep, "lr": lr_ep, "train_loss": mean_loss, "seconds": round(time.time() - t0, 2)}
        if ep % eval_every == eval_every - 1 or ep == epochs - 1:
            rec.update(evaluate(net, xd[val], ud[val], mu[val], r[val]))
        hist.append(rec)
        log(json.dumps(rec))
    torch.cuda.synchronize()
    summary = {"samples": n, "train": n_train, "batch": batch, "epochs": epochs, "lr": lr, "loss": loss,
               "seed": seed, "x_range": list(x_range), "seconds": round(time.time() - t0, 2), "final": hist[-1]}
    return net, summary


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--samples", type=int, default=1 << 24)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--loss", default="mse", choices=["mse", "mae"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--x-min", type=float, default=X_RANGE[0])
    ap.add_argument("--x-max", type=float, default=X_RANGE[1])
    a = ap.parse_args(argv)
    from . import compton

    ctx = compton.Context(0)
    net, summary = train(ctx, a.samples, a.batch, a.epochs, a.lr, a.loss, a.seed,
                         log=lambda s: print(s, flush=True), x_range=(a.x_min, a.x_max))
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    net.save(a.out)
    summary["out"] = a.out
    print(json.dumps(summary), flush=True)
    net.close()
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
