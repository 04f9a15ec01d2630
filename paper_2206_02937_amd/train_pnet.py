"""Train the paper's probability network (Sec. 3.2) on the GPU with the
library's own kernels, in cumulative transfer-learning stages over the
photon energy range, and evaluate it on head-on collisions.

    python -m paper_2206_02937_amd.train_pnet [--steps N] [--out params.npy]

Data: candidate pairs with isotropic photons of energy eps log-uniform in the
stage's range [1e-3, eps_max] (stages: eps_max = 0.1, 1, 10 m_e c^2, each
stage keeping the earlier ranges, as the paper trains on cumulative ranges)
and isotropic leptons with |p| uniform in [0, 60] m_e c; P_max and the two
weights uniform (the target does not depend on them).  Targets y = P / P_max
from cs_pnet_target (FP64).  A fresh seeded batch of 4096 pairs per Adam step
(lr 1e-3, MAE, the paper's choices).

The network trains on inputs divided by fixed scales (photon momentum by 10,
lepton momentum by 60: inputs of order one); the exported parameters take
the inputs in code units, the scales folded into the first layer's weights
(W1[:, q] / scale[q]).

Evaluation (the paper's head-on check): lepton p = (0, 0, p_e) with p_e = 5,
25, 50, photon k = (0, 0, -eps) for 61 energies log-spaced over
[1e-3, 10]; the relative error of y' against y after each stage, and for a
network trained on the whole range from the start for the same number of
steps (the ablation of the stages).
"""
import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2206_02937_amd import compton  # noqa: E402

STAGES = (0.1, 1.0, 10.0)
EPS_MIN = 1e-3
P_MAX_LEPTON = 60.0
BATCH = 4096
SCALE = np.array([10.0, 10.0, 10.0, 60.0, 60.0, 60.0, 1.0, 1.0, 1.0], dtype=np.float32)


def glorot_uniform(rng):
    widths = (9, 9, 12, 9, 1)
    out = []
    for i in range(len(widths) - 1):
        n_in, n_out = widths[i], widths[i + 1]
        lim = np.sqrt(6.0 / (n_in + n_out))
        out.append(rng.uniform(-lim, lim, size=n_out * n_in))
        out.append(np.zeros(n_out))
    return np.concatenate(out).astype(np.float32)


def batch(rng, n, eps_max):
    def iso(m):
        v = rng.standard_normal((m, 3))
        return v / np.linalg.norm(v, axis=1, keepdims=True)

    k = iso(n) * np.exp(rng.uniform(np.log(EPS_MIN), np.log(eps_max), (n, 1)))
    p = iso(n) * rng.uniform(0.0, P_MAX_LEPTON, (n, 1))
    rest = np.stack([rng.uniform(0.01, 1.0, n), rng.uniform(0.5, 2.0, n), rng.uniform(0.5, 2.0, n)], axis=1)
    return np.concatenate([k, p, rest], axis=1).astype(np.float32)


def head_on_inputs():
    eps = np.logspace(-3, 1, 61)
    rows = []
    for pe in (5.0, 25.0, 50.0):
        for e in eps:
            rows.append([0.0, 0.0, -e, 0.0, 0.0, pe, 0.5, 1.0, 1.0])
    return np.array(rows, dtype=np.float32)


def unscaled(params):
    """Parameters for inputs in code units: W1 (the first 81 entries, [9][9]
    row-major) divided column-wise by the input scales."""
    out = np.array(params, dtype=np.float32, copy=True)
    out[:81] = (out[:81].reshape(9, 9) / SCALE[None, :]).ravel()
    return out


def evaluate(ctx, params, X_eval, y_eval):
    y = ctx.pnet_forward(params, X_eval).cpu().numpy().astype(np.float64)
    rel = np.abs(y - y_eval) / np.maximum(y_eval, 1e-12)
    out = {}
    for i, pe in enumerate((5, 25, 50)):
        r = rel[61 * i:61 * (i + 1)]
        out[f"p_e={pe}"] = {"median_rel_err": float(np.median(r)), "max_rel_err": float(np.max(r))}
    return out


def train(ctx, params, stages, steps_per_stage, seed, X_eval, y_eval, log):
    import torch

    rng = np.random.default_rng(seed)
    p = torch.from_numpy(params.copy()).cuda()
    m = torch.zeros_like(p)
    v = torch.zeros_like(p)
    t = 0
    report = []
    for si, eps_max in enumerate(stages):
        ranges = stages[:si + 1]
        for _ in range(steps_per_stage):
            # cumulative: each batch draws its energy range from the stages so far
            X = np.concatenate([batch(rng, BATCH // len(ranges), e) for e in ranges])
            Xd = torch.from_numpy(X).cuda()
            yd = ctx.pnet_target(Xd)
            g, loss = ctx.pnet_grad(p, torch.from_numpy(X / SCALE).cuda(), yd, "mae")
            t += 1
            ctx.pnet_adam(p, g, m, v, t, lr=1e-3)
        ev = evaluate(ctx, torch.from_numpy(unscaled(p.cpu().numpy())).cuda(), X_eval, y_eval)
        entry = {"stage": si + 1, "eps_max": eps_max, "steps": t, "train_mae": float(loss.cpu().numpy()[0]),
                 "head_on": ev}
        report.append(entry)
        log(entry)
    return unscaled(p.cpu().numpy()), report


def main():
    import torch

    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=10000, help="Adam steps per stage")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--out", default=None, help="write the trained parameters (.npy)")
    args = ap.parse_args()
    ctx = compton.Context(0)
    X_eval = torch.from_numpy(head_on_inputs()).cuda()
    y_eval = ctx.pnet_target(X_eval).cpu().numpy().astype(np.float64)
    init = glorot_uniform(np.random.default_rng(args.seed))
    log = lambda e: print(json.dumps(e), flush=True)
    params, staged = train(ctx, init, STAGES, args.steps, args.seed + 1, X_eval, y_eval, log)
    # ablation: the whole range from the start, the same number of steps
    _, flat = train(ctx, init, (STAGES[-1],) * len(STAGES), args.steps, args.seed + 1, X_eval, y_eval,
                    lambda e: print(json.dumps({"no_stages": e}), flush=True))
    if args.out:
        np.save(args.out, params)
    print(json.dumps({"summary": {"staged": staged[-1]["head_on"], "no_stages": flat[-1]["head_on"]}}),
          flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
