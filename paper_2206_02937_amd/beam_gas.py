"""Inverse-Compton beam in a monoenergetic photon gas (the paper's spectrum
benchmark, Sec. 3.3, Fig. 4a): electron beams of momentum p_e = 25, 50, 100
m_e c along z in a gas of isotropic photons of energy 2.5 m_e c^2, stepped by
the library with the plain inverse-CDF sampler and with the sampler network;
the scattered photons' momentum spectra are compared.

    python -m paper_2206_02937_amd.beam_gas [--steps N] [--cells C] [--sampler mlp_bf16]

Per beam: photons whose momentum changed over the run (each counted once, in
its final state), their |k| relative to p_e (median, mode of a log-binned
histogram, the fraction below p_e / 2), the two-sample Kolmogorov-Smirnov
distance between the plain and the network spectra, and the fraction of
network samples outside the network's x range that the plain sampler
answered (for p_e = 100 most rest-frame energies x exceed the range).
"""
import argparse
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from paper_2206_02937_amd import compton, plasma  # noqa: E402

WEIGHTS = os.path.join(HERE, "weights", "sampler_2x64x4.csnet")
BEAMS = (25.0, 50.0, 100.0)
EPS = 2.5


def run(ctx, p, sampler="plain", mlp=None, steps=20):
    """Step the plasma `steps` times on the GPU; returns the final |k| of
    every photon whose momentum changed, and the summed step counters."""
    import torch

    e, g, oe, og = compton.to_device(p)
    buf = ctx.stats_buffer()
    coll = fb = pairs = 0
    for s in range(steps):
        ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, s, sampler=sampler, mlp=mlp, stats=buf)
        st = buf.cpu().numpy()
        pairs += int(st[0])
        coll += int(st[1])
        fb += int(st[4])
    torch.cuda.synchronize()
    gh = compton.to_host(g)
    k = np.stack([gh["x"], gh["y"], gh["z"]], axis=1).astype(np.float64)
    k0 = np.stack([p.g["x"], p.g["y"], p.g["z"]], axis=1).astype(np.float64)
    moved = np.any(k != k0, axis=1)
    return {"k": np.linalg.norm(k[moved], axis=1), "pairs": pairs, "collisions": coll, "fallback": fb}


def ks_distance(a, b):
    """Two-sample Kolmogorov-Smirnov statistic sup |F_a - F_b|."""
    a, b = np.sort(a), np.sort(b)
    x = np.concatenate([a, b])
    return float(np.max(np.abs(np.searchsorted(a, x, side="right") / a.size
                               - np.searchsorted(b, x, side="right") / b.size)))


def spectrum(k, p_e, bins=48):
    """Counts of |k| / p_e in log bins over [1e-3, 2]; returns (edges, counts)."""
    edges = np.logspace(-3, np.log10(2.0), bins + 1)
    counts, _ = np.histogram(np.asarray(k) / p_e, bins=edges)
    return edges, counts


def describe(k, p_e):
    edges, counts = spectrum(k, p_e)
    i = int(np.argmax(counts))
    return {"scattered": int(k.size), "median_over_pe": float(np.median(k) / p_e),
            "mode_over_pe": float(np.sqrt(edges[i] * edges[i + 1])),
            "below_half_pe": float(np.mean(k < 0.5 * p_e))}


def compare_beam(ctx, p_e, mlp, sampler, steps, n_cells, per_cell=256, seed=3):
    p = plasma.beam_gas(seed=seed, p_e=p_e, eps=EPS, n_cells=n_cells, per_cell=per_cell)
    a = run(ctx, p, "plain", None, steps)
    b = run(ctx, p, sampler, mlp, steps)
    return {"p_e": p_e, "plain": {**describe(a["k"], p_e), "collisions": a["collisions"]},
            sampler: {**describe(b["k"], p_e), "collisions": b["collisions"],
                      "fallback_fraction": b["fallback"] / max(b["collisions"], 1)},
            "ks": ks_distance(a["k"], b["k"])}


def load_sampler(ctx, sampler):
    net = compton.MLP.load(ctx, WEIGHTS)
    if sampler == "mlp_bf16":
        net.quantize("mlp_bf16")
    elif sampler != "mlp_f32":
        raise ValueError("sampler must be mlp_f32 or mlp_bf16")
    return net


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--cells", type=int, default=1024)
    ap.add_argument("--sampler", default="mlp_bf16", choices=["mlp_f32", "mlp_bf16"])
    args = ap.parse_args()
    ctx = compton.Context(0)
    ctx.set_strategy("compact")
    net = load_sampler(ctx, args.sampler)
    for pe in BEAMS:
        print(json.dumps(compare_beam(ctx, pe, net, args.sampler, args.steps, args.cells)), flush=True)
    net.close()
    ctx.close()


if __name__ == "__main__":
    main()
