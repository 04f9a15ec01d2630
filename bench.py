"""Benchmark: scattering pairs/s of the Compton step on one MI355X, the
network sampler (BF16 on MFMA by default) against the plain inverse-CDF
sampler, with the KS distance of their outputs.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload grid_large]
                    [--sampler mlp_bf16] [--no-autotune --strategy fused] [--no-graph]

A step is one cs_compton_step call over the whole plasma (pairing, boost,
cross-section, probability, accept/compaction, sampling, scattering,
write-back, stats).  The default workload is the 128x128-cell FP32 grid with
256 electrons and 256 photons per cell (2^22 pairs per step; Maxwell-Juttner
kT = 0.5 electrons, photons log-uniform in [1e-4, 1e-1]); the particles are
resident in device memory before the timed region starts.  The sampler
network is the trained one shipped in the package.  By default the library's
autotuner picks the kernel strategy and tile shape first (on a private copy of
the particles), and the timed steps replay one captured step as a HIP graph
(the step index advances in device memory).  Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WEIGHTS = os.path.join(ROOT, "paper_2206_02937_amd", "weights", "sampler_2x64x4.csnet")
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"mlp_bf16": 2500.0, "mlp_fp8": 5000.0}
PEAK_FP32_TFLOPS = 157.3
SIMD_COUNT = 256 * 4
CLOCK_HZ = 2.4e9
# the network's SiLU issues two transcendental instructions (exp2, reciprocal)
# per activation, 256 activations per sample; one wavefront transcendental
# instruction takes ~11.7 cycles on this part (measured), so at most
# SIMD_COUNT x CLOCK_HZ x 64 / (512 x 11.7) samples/s
TRANS_CYCLES = 11.7
SILU_CEILING = SIMD_COUNT * CLOCK_HZ * 64 / (512 * TRANS_CYCLES)
MLP_MFMA_FLOPS = 3 * 64 * 64 * 2  # hidden 64x64 layers per sample
WORKLOADS = ["grid_large", "grid", "single_cell", "uneven", "power_law"]
METRIC = "scattering pairs/s, MLP vs plain sampler, 1 MI355X at KS≤2e-3 vs FP64 oracle"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="grid_large", choices=WORKLOADS)
    ap.add_argument("--sampler", default="mlp_bf16", choices=["plain", "mlp_f32", "mlp_bf16", "mlp_fp8"])
    ap.add_argument("--strategy", default="fused", choices=["fused", "compact", "multi_kernel", "per_cell"])
    ap.add_argument("--chunks-per-block", type=int, default=0, help="fused strategy; 0 = automatic")
    ap.add_argument("--sweep", action="store_true", help="time every strategy / chunks-per-block candidate")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-sampler comparison run")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-autotune", dest="autotune", action="store_false",
                    help="keep --strategy / --chunks-per-block instead of choosing with cs_autotune")
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="time eager cs_compton_step calls instead of replaying one captured step (HIP graph)")
    ap.add_argument("--baseline", default=None, choices=["per_cell", "multi_kernel", "fused", "compact"],
                    help="also time this strategy with the plain sampler (eager)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip the uneven-cell and power-law workloads")
    ap.add_argument("--traffic-calibration", action="store_true",
                    help="end with one plain 256 MiB device-to-device copy (scale for the HBM byte counters)")
    return ap.parse_args()


def source_digest():
    """16 hex digits of SHA-1 over the kernel sources (csrc/*.hip and *.h in
    name order, each file's name then its bytes): identifies the kernels a
    counter record was taken with."""
    import glob
    import hashlib

    h = hashlib.sha1()
    csrc = os.path.join(ROOT, "paper_2206_02937_amd", "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.h"))):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def counter_record(tag, kernel, workload, launch=None):
    """The fields of the `tag` line ("traffic-record:", "valu-record:") for
    `kernel` on `workload` (and, when given, the launch configuration
    `launch`, e.g. "ppl1_g16": pairs per lane and chunks per pair block) in
    the counter summaries under profiles/; None when no record matches or the
    kernel sources changed since the counters were taken."""
    import glob

    digest = source_digest()
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "counters_*.md"))):
        with open(f) as fh:
            for line in fh:
                if not line.startswith(tag):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("kernel") == kernel and kv.get("workload") == workload and kv.get("source_sha") == digest
                        and (launch is None or kv.get("launch") == launch)):
                    return kv
    return None


def traffic_record(kernel, workload, launch=None):
    """HBM bytes per launch of `kernel` on `workload` from the FETCH_SIZE /
    WRITE_SIZE counters, each scaled by what it reads for a plain device copy
    of known size (the calibration recorded with them); None as above."""
    kv = counter_record("traffic-record:", kernel, workload, launch)
    return int(kv["bytes_per_launch"]) if kv else None


def launch_tag(ctx):
    """The pair kernel's launch configuration as the counter records name it:
    pairs per lane and chunks per pair block, as the context holds them."""
    from paper_2206_02937_amd import compton

    return (f"ppl{ctx.get_option(compton.OPT_PAIRS_PER_LANE)}"
            f"_g{ctx.get_option(compton.OPT_CHUNKS_PER_BLOCK)}")


def valu_roofline(kernel, workload, avg_ms, units, launch=None):
    """VALU-issue roofline of `kernel` on `workload`: the SIMD cycles spent
    issuing VALU instructions per launch (4 x SQ_ACTIVE_INST_VALU, summed
    over the chip, from the counter summaries) against every SIMD's cycles
    over the launch's live average duration (1024 SIMDs at 2.4 GHz); with
    the VALU instructions per unit of work.  None without a current record."""
    kv = counter_record("valu-record:", kernel, workload, launch)
    if kv is None:
        return None
    busy = float(kv["valu_busy_cycles"])
    avail = avg_ms * 1e-3 * SIMD_COUNT * CLOCK_HZ
    return {"kernel": kernel, "bound": "valu", "achieved": busy / avail, "peak": 1.0,
            "unit": "fraction of SIMD cycles issuing VALU", "frac": busy / avail,
            "valu_busy_cycles_per_launch": busy, "wave_valu_insts_per_launch": float(kv["valu_insts"]),
            "valu_insts_per_unit": float(kv["valu_insts"]) * 64 / units, "unit_of_work": "pair (per lane)",
            "avg_ms": avg_ms}


def hbm_copy_stage(mib=512, reps=20):
    """The HBM bandwidth a plain device-to-device copy reaches on this machine: a
    512 MiB buffer (twice the Infinity Cache) copied `reps` times, timed with
    HIP events; bytes moved = read + written.  Context for the HBM rooflines,
    whose peak stays the published 8 TB/s."""
    import torch

    src = torch.ones((mib << 20) // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        dst.copy_(src)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    moved = 2 * src.numel() * 4
    del src, dst
    torch.cuda.empty_cache()
    gbs = moved / (ms * 1e-3) / 1e9
    return {"gbs": gbs, "bytes_per_copy": moved, "ms_per_copy": ms, "frac_of_peak": gbs / PEAK_HBM_GBS}


def storage_bytes(dtype):
    return 8 if str(dtype).endswith("64") else 4


def cpu_baseline(p, seconds):
    """The FP64 oracle timed on this host's cores over a bounded sample of
    the same workload: whole cells of the initial state, growing the number of
    cells (and then of steps) until about `seconds` of CPU work."""
    import numpy as np

    import oracle

    threads = oracle.num_threads()
    counts = np.minimum(np.diff(p.off_e), np.diff(p.off_g))
    rng = np.random.default_rng(123)
    order = rng.permutation(p.n_cells)
    n_sel, n_steps = max(1, min(p.n_cells, 8)), 1
    while True:
        cells = np.sort(order[:n_sel])
        q = p.copy()
        t0 = time.perf_counter()
        for s in range(n_steps):
            oracle.compton_step(q.e, q.g, q.off_e, q.off_g, q.dt, q.density_norm, q.seed, s, cells=cells)
        elapsed = time.perf_counter() - t0
        pairs = int(counts[cells].sum()) * n_steps
        if elapsed >= seconds:
            break
        grow = max(1.5, min(8.0, 1.2 * seconds / max(elapsed, 1e-3)))
        if n_sel < p.n_cells:
            n_sel = min(p.n_cells, int(n_sel * grow) + 1)
        else:
            n_steps = int(n_steps * grow) + 1
    return {"value": pairs / elapsed, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"{n_steps} step(s) over {n_sel} of {p.n_cells} cells ({pairs} pair-steps) of the same "
                      f"plasma, plain sampler, {elapsed:.1f} s"}


def binning_stage(ctx, p, reps=20):
    """Cell binning (cs_bin_particles) of the workload's electrons after a
    seeded shuffle: particles/s and the HBM roofline of the whole call, whose
    algorithmic bytes per particle are its cell id and four values read and
    the four values written (plus 8 B per cell offset)."""
    import numpy as np
    import torch

    rng = np.random.default_rng(1)
    n = p.e["x"].size
    cell = np.repeat(np.arange(p.n_cells, dtype=np.int32), np.diff(p.off_e))
    perm = rng.permutation(n)
    sp = {k: torch.from_numpy(np.ascontiguousarray(p.e[k][perm])).cuda() for k in "xyzw"}
    cell_d = torch.from_numpy(cell[perm]).cuda()
    out = {k: torch.empty_like(sp[k]) for k in "xyzw"}
    off = torch.empty(p.n_cells + 1, dtype=torch.int64, device="cuda")
    n_inv = torch.zeros(1, dtype=torch.int64, device="cuda")
    for _ in range(3):
        ctx.bin_particles(cell_d, sp, p.n_cells, out, off, n_inv)
    torch.cuda.synchronize()
    assert np.array_equal(off.cpu().numpy(), p.off_e), "binning offsets differ from the workload's"
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        ctx.bin_particles(cell_d, sp, p.n_cells, out, off, n_inv)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    sb = sp["x"].element_size()
    bytes_call = n * (4 + 8 * sb) + 8 * (p.n_cells + 1)
    gbs = bytes_call / (ms * 1e-3) / 1e9
    return {"particles_per_s": n / (ms * 1e-3), "ms_per_call": ms, "particles": n, "cells": p.n_cells,
            "roofline": {"kernel": "cs_bin_particles (all passes)", "bound": "hbm", "achieved": gbs,
                         "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": None,
                         "bytes_per_launch": bytes_call, "avg_ms": ms}}


def ntc_stage(ctx, p, steps=50, warmup=5):
    """The step with no-time-counter candidate selection on the same plasma:
    eager cs_ntc_step calls (milliseconds per step by wall clock around the
    calls; each call waits for the device's candidate count) and replays of
    a captured step (cs_ntc_graph_create, sized 1.5x the eager count;
    milliseconds per replay by HIP events on the replay stream), candidates
    and collisions per step, and the workload's 1:1-pairing pair count per
    second for comparison with the headline (both advance the same plasma
    by one step)."""
    import time

    import torch

    from paper_2206_02937_amd import compton

    e, g, oe, og = compton.to_device(p)
    stats = ctx.stats_buffer()
    for s in range(warmup):
        ctx.ntc_step(e, g, oe, og, p.dt, p.density_norm, p.seed, s, stats=stats)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(warmup, warmup + steps):
        ctx.ntc_step(e, g, oe, og, p.dt, p.density_norm, p.seed, s, stats=stats)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    st = compton.decode_stats(stats)
    out = {"ms_per_step": ms, "candidates_per_step": st["n_pairs"], "collisions_per_step": st["n_collided"],
           "candidates_per_s": st["n_pairs"] / (ms * 1e-3), "pairs_equivalent_per_s": p.n_pairs / (ms * 1e-3),
           "expected_collisions": st["sum_prob"]}
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        gr = ctx.ntc_graph(e, g, oe, og, p.dt, p.density_norm, p.seed, (3 * st["n_pairs"]) // 2, stats=stats)
        try:
            gr.set_step(warmup + steps)
            for _ in range(warmup):
                gr.launch()
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(steps):
                gr.launch()
            t1.record(stream)
            stream.synchronize()
            gms = t0.elapsed_time(t1) / steps
        finally:
            gr.close()
    gst = compton.decode_stats(stats)
    out["graph"] = {"ms_per_step": gms, "candidates_per_step": gst["n_pairs"], "overflow": gst["overflow"],
                    "pairs_equivalent_per_s": p.n_pairs / (gms * 1e-3)}
    return out


def training_stage(ctx, batch=4096, steps=200, more_batches=(16384, 65536)):
    """One optimiser step of the sampler network (cs_mlp_train_step: forward,
    backward, fixed-order gradient sum, Adam) at the training driver's batch
    of 4096 samples, on a separate copy of the network: samples/s and the
    FP32 rate at 75 k flops per sample (forward 25 k, backward 50 k); the
    same at larger batches, which fill more of the chip (the driver keeps
    4096: its optimisation is tuned at that batch)."""
    import numpy as np
    import torch

    from paper_2206_02937_amd import compton, plasma

    net = compton.MLP.load(ctx, WEIGHTS)

    def timed(b, n_steps):
        x, u = plasma.sampler_inputs(b, seed=11)
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        ud = torch.from_numpy(u.astype(np.float32)).cuda()
        mu, r = ctx.sample_plain(xd, ud)
        loss = torch.zeros((), dtype=torch.float32, device="cuda")
        for _ in range(10):
            net.train_step(xd, ud, mu, r, lr=1e-4, loss_out=loss)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(n_steps):
            net.train_step(xd, ud, mu, r, lr=1e-4, loss_out=loss)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / n_steps
        tfs = 75e3 * b / (ms * 1e-3) / 1e12
        return {"batch": b, "ms_per_step": ms, "samples_per_s": b / (ms * 1e-3), "fp32_tflops": tfs,
                "fp32_frac": tfs / PEAK_FP32_TFLOPS}

    out = timed(batch, steps)
    out["larger_batches"] = [timed(b, max(20, steps // 4)) for b in more_batches]
    net.close()
    return out


def beam_gas_stage(ctx, net, sampler, steps=10, n_cells=4096):
    """The paper's inverse-Compton benchmark at p_e = 100 m_e c (photon gas of
    2.5 m_e c^2): scattered-photon spectra with the plain sampler and with
    the network after `steps` steps (peak position, KS distance between the
    two, the network's fallback fraction)."""
    from paper_2206_02937_amd import beam_gas as B

    if sampler not in ("mlp_f32", "mlp_bf16"):
        return None
    return B.compare_beam(ctx, 100.0, net, sampler, steps, n_cells)


def pnet_stage(ctx, p, reps=20):
    """The paper's probability network against the analytic ratio it
    replaces, on the workload's 2^22 candidate pairs (photon, lepton, P_max and
    weights per pair: nine FP32 inputs, 36 B in and 4 B out per pair).  The
    network's parameters are Glorot-uniform: the timing does not depend on
    them.  Roofline: HBM (40 B per pair) and FP32 vector arithmetic (612
    multiply-adds counted as 2 flops: 2 (81 + 108 + 108 + 9))."""
    import numpy as np
    import torch

    from paper_2206_02937_amd import train_pnet

    n = min(p.e["x"].size, p.g["x"].size)
    rows = np.stack([p.g["x"][:n], p.g["y"][:n], p.g["z"][:n], p.e["x"][:n], p.e["y"][:n], p.e["z"][:n],
                     np.full(n, 0.5), p.e["w"][:n], p.g["w"][:n]], axis=1).astype(np.float32)
    X = torch.from_numpy(rows).cuda()
    params = torch.from_numpy(train_pnet.glorot_uniform(np.random.default_rng(0))).cuda()
    y = torch.empty(n, dtype=torch.float32, device="cuda")

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    ms_net = timed(lambda: ctx.pnet_forward(params, X, y))
    ms_ana = timed(lambda: ctx.pnet_target(X, y))
    gbs = n * 40 / (ms_net * 1e-3) / 1e9
    tfs = n * 612 / (ms_net * 1e-3) / 1e12
    return {"pairs": n, "network_pairs_per_s": n / (ms_net * 1e-3), "analytic_pairs_per_s": n / (ms_ana * 1e-3),
            "network_ms": ms_net, "analytic_ms": ms_ana,
            "roofline": {"kernel": "k_pnet_fwd", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS, "traffic": None,
                         "bytes_per_launch": n * 40, "avg_ms": ms_net,
                         "fp32_tflops": tfs, "fp32_frac": tfs / 157.3}}


def load_network(ctx, sampler):
    """The shipped sampler network, prepared for BF16 and for FP8 (calibrated
    on 2^16 inputs log-uniform over the network's x range)."""
    import numpy as np
    import torch

    from paper_2206_02937_amd import compton, plasma

    if sampler == "plain":
        return None
    net = compton.MLP.load(ctx, WEIGHTS)
    lo, hi = net.domain
    net.quantize("mlp_bf16")
    cx, cu = plasma.sampler_inputs(65536, seed=7, x_min=lo, x_max=hi)
    net.quantize("mlp_fp8", torch.from_numpy(cx.astype(np.float32)).cuda(),
                 torch.from_numpy(cu.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return net


def run_steps(ctx, p, sampler, net, steps, warmup, step0=0, graph=False):
    """Warm up, then time `steps` steps (wall clock between two device
    synchronisations, plus the library's per-stage HIP events recorded on the
    launch stream during the same steps).  graph=True replays one captured
    step instead (no per-stage events then)."""
    import torch

    from paper_2206_02937_amd import compton

    e, g, oe, og = compton.to_device(p)
    stats = ctx.stats_buffer()
    torch.cuda.synchronize()
    stream = torch.cuda.Stream() if graph else torch.cuda.current_stream()
    with torch.cuda.stream(stream):
        gr = None
        if graph:
            gr = ctx.graph(e, g, oe, og, p.dt, p.density_norm, p.seed, sampler=sampler, mlp=net, stats=stats)
            gr.set_step(step0)
        step = step0

        def one():
            nonlocal step
            if gr is not None:
                gr.launch()
            else:
                ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, step, sampler=sampler, mlp=net, stats=stats)
            step += 1

        for _ in range(warmup):
            one()
        torch.cuda.synchronize()
        if gr is None:
            ctx.set_stage_timing(True)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(steps):
            one()
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stage_ms = None
        if gr is None:
            stage_ms = ctx.stage_times()
            ctx.set_stage_timing(False)
        else:
            gr.close()
    st = compton.decode_stats(stats)
    return {"pairs_per_s": p.n_pairs * steps / wall, "ms_per_step": wall * 1e3 / steps,
            "gpu_ms_per_step": ev0.elapsed_time(ev1) / steps, "stage_ms": stage_ms, "last_stats": st}


def sampler_stage(ctx, p, net, sampler, n=1 << 22):
    """Sampler-stage throughput on the same n (x, u) inputs drawn from the
    plasma's pairs: the plain FP64 inverse-CDF sampler and the network, plus
    the KS distance of the network's outputs from the plain sampler's."""
    import numpy as np
    import torch

    from paper_2206_02937_amd import sampler_quality as sq

    x, u = sq.plasma_inputs(ctx, p, n, seed=0)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    ud = torch.from_numpy(u.astype(np.float32)).cuda()
    mu = torch.empty_like(xd)
    r = torch.empty_like(xd)

    def timed(fn, reps=20):
        fn()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps * 1e-3

    out = {"n": n, "inputs": "x of the plasma's electron-photon pairs, u uniform"}
    out["plain"] = n / timed(lambda: ctx.sample_plain(xd, ud, mu, r))
    mu_p, r_p = mu.cpu().numpy(), r.cpu().numpy()
    res = {}
    if net is not None:
        mask = torch.empty(n, dtype=torch.uint8, device=xd.device)
        from paper_2206_02937_amd import compton

        lib = compton.lib()

        def net_sample(prec):
            ctx._check(lib.cs_mlp_sample(ctx.handle, net.handle, compton.SAMPLERS[prec], compton._ptr(xd),
                                         compton._ptr(ud), n, compton._ptr(mu), compton._ptr(r),
                                         compton._ptr(mask), compton._stream(None)))

        for prec in ("mlp_f32", "mlp_bf16", "mlp_fp8"):
            t = timed(lambda: net_sample(prec))
            out[prec] = n / t
            ks_mu = sq.ks_distance(mu.cpu().numpy(), mu_p)
            ks_r = sq.ks_distance(r.cpu().numpy(), r_p)
            res[prec] = {"mu": ks_mu, "r": ks_r, "fallback_frac": float(mask.float().mean().item()), "t": t}
    return out, res


def mfma_roofline(prec, stage, ks):
    """MFMA rate of the network kernel (k_mlp_mfma) from its sampler-stage
    time: 3 x 64 x 64 x 2 flops per sample in the hidden layers."""
    if prec not in ks:
        return None
    t = ks[prec]["t"]
    tf = stage["n"] * MLP_MFMA_FLOPS / t / 1e12
    rate = stage["n"] / t
    return {"kernel": f"k_mlp_mfma<{prec[4:]}>", "bound": "mfma", "achieved": tf, "peak": PEAK_MFMA_TFLOPS[prec],
            "unit": "TFLOP/s", "frac": tf / PEAK_MFMA_TFLOPS[prec], "traffic": None,
            "flops_per_launch": stage["n"] * MLP_MFMA_FLOPS, "avg_ms": t * 1e3,
            "silu_ceiling_samples_per_s": SILU_CEILING, "samples_per_s": rate, "silu_frac": rate / SILU_CEILING}


def pair_roofline(p, run, strategy, launch=None):
    """HBM roofline of the pair kernel from a stage-timed (eager) run:
    algorithmic bytes = every pair's 8 particle values read + per collision
    its stash entry (8 values, 2 indices) and list slot written."""
    sb = storage_bytes(p.e["x"].dtype)
    st = run["last_stats"]
    stage_ms = run["stage_ms"]
    if strategy != "compact" or not stage_ms:
        return None
    ms = stage_ms["pair"] - stage_ms["compact"]
    b = p.n_pairs * 8 * sb + st["n_collided"] * (8 * sb + 12)
    gbs = b / (ms * 1e-3) / 1e9
    return {"kernel": "k_pair_compact", "bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": gbs / PEAK_HBM_GBS, "traffic": traffic_record("k_pair_compact", p.name, launch),
            "bytes_per_launch": b, "avg_ms": ms, "units_per_launch": f"{p.n_pairs} pairs, {st['n_collided']} collisions",
            "launch": launch, "working_set_mib": p.nbytes() / 2**20,
            "valu": valu_roofline("k_pair_compact", p.name, ms, p.n_pairs, launch)}


def workload_stage(ctx, p, net, samplers, steps, warmup, autotune_sampler="mlp_bf16", baseline=None,
                   baseline_steps=5):
    """One more workload, measured like the headline: the autotuner's pick,
    graph-replayed steps for each sampler, a stage-timed eager run (the pair
    kernel's HBM roofline), optionally the plain sampler under a baseline
    strategy, and the network's KS distance on 2^20 of the plasma's pair
    inputs.  The context's options are restored afterwards."""
    import numpy as np
    import torch

    from paper_2206_02937_amd import compton, sampler_quality as sq

    saved = [ctx.get_option(o) for o in (compton.OPT_STRATEGY, compton.OPT_CHUNKS_PER_BLOCK,
                                         compton.OPT_PAIRS_PER_LANE)]
    e, g, oe, og = compton.to_device(p)
    tuned = ctx.autotune(e, g, oe, og, p.dt, p.density_norm, p.seed, 0, sampler=autotune_sampler,
                         mlp=net if autotune_sampler != "plain" else None, reps=3)
    del e, g, oe, og
    strategy = compton.STRATEGY_NAMES[ctx.get_option(compton.OPT_STRATEGY)]
    out = {"workload": f"{p.name}: {p.n_cells} cells, {p.n_pairs} pairs per step", "pairs_per_step": p.n_pairs,
           "autotune_best": tuned["best"], "steps": steps}
    for sampler in samplers:
        r = run_steps(ctx, p, sampler, net if sampler != "plain" else None, steps, warmup, graph=True)
        out[sampler] = {"pairs_per_s": r["pairs_per_s"], "ms_per_step": r["ms_per_step"],
                        "collisions_per_step": r["last_stats"]["n_collided"],
                        "fallback_per_step": r["last_stats"]["n_fallback"]}
    eager = run_steps(ctx, p, "plain", None, steps, warmup)
    out["roofline"] = pair_roofline(p, eager, strategy, launch_tag(ctx))
    if baseline:
        ctx.set_strategy(baseline)
        ctx.set_chunks_per_block(0)
        r = run_steps(ctx, p, "plain", None, baseline_steps, 1)
        out["baseline"] = {"strategy": baseline, "sampler": "plain", "pairs_per_s": r["pairs_per_s"],
                           "ms_per_step": r["ms_per_step"]}
    for o, v in zip((compton.OPT_STRATEGY, compton.OPT_CHUNKS_PER_BLOCK, compton.OPT_PAIRS_PER_LANE), saved):
        ctx.set_option(o, v)
    if net is not None:
        n = 1 << 20
        x, u = sq.plasma_inputs(ctx, p, n, seed=0)
        xd = torch.from_numpy(x.astype(np.float32)).cuda()
        ud = torch.from_numpy(u.astype(np.float32)).cuda()
        mu_p, r_p = ctx.sample_plain(xd, ud)
        mu_p, r_p = mu_p.cpu().numpy(), r_p.cpu().numpy()
        out["ks"] = {}
        for prec in samplers:
            if prec == "plain":
                continue
            m, rr, fb = net.sample(xd, ud, prec)
            out["ks"][prec] = {"mu": sq.ks_distance(m.cpu().numpy(), mu_p), "r": sq.ks_distance(rr.cpu().numpy(), r_p),
                               "fallback_frac": float(fb.float().mean().item())}
    return out


def gpu_step_cells(ctx, p, sampler, net, cells, step=0):
    """One eager step of the whole plasma from its initial state with the
    context's strategy; returns the sampled cells' particles (host)."""
    import numpy as np
    import torch

    from paper_2206_02937_amd import compton

    e, g, oe, og = compton.to_device(p)
    ctx.step(e, g, oe, og, p.dt, p.density_norm, p.seed, step, sampler=sampler,
             mlp=net if sampler != "plain" else None)
    ie = np.concatenate([np.arange(p.off_e[c], p.off_e[c + 1]) for c in cells])
    ig = np.concatenate([np.arange(p.off_g[c], p.off_g[c + 1]) for c in cells])
    tie, tig = torch.from_numpy(ie).cuda(), torch.from_numpy(ig).cuda()
    out = ({k: v.index_select(0, tie).cpu().numpy() for k, v in e.items()},
           {k: v.index_select(0, tig).cpu().numpy() for k, v in g.items()}, ie, ig)
    torch.cuda.synchronize()
    return out


def oracle_leg(ctx, p, net, samplers, seconds, n_cells_err=128):
    """The oracle's leg: the FP64 oracle timed on this host's cores over a
    bounded sample of the workload (cpu_baseline), and, from the same initial
    state, the per-event error of the GPU step against it on n_cells_err
    sampled cells (photon |k - k_ref| / eps_ref, electron |p - p_ref| /
    gamma_ref over the particles the step moved): the plain sampler must
    match to the storage tolerance; for the network samplers this is their
    error against the exact method."""
    import numpy as np

    import oracle

    cpu = cpu_baseline(p, seconds) if seconds > 0 else None
    rng = np.random.default_rng(5)
    cells = np.sort(rng.choice(p.n_cells, min(n_cells_err, p.n_cells), replace=False))
    ref = p.copy()
    oracle.compton_step(ref.e, ref.g, ref.off_e, ref.off_g, ref.dt, ref.density_norm, ref.seed, 0, cells=cells)
    errs = {}
    for sampler in samplers:
        ge, gg, ie, ig = gpu_step_cells(ctx, p, sampler, net, cells)

        def vec(d, idx=None):
            return np.stack([d[c] if idx is None else d[c][idx] for c in "xyz"], axis=1).astype(np.float64)

        pr, kr = vec(ref.e, ie), vec(ref.g, ig)
        p0, k0 = vec(p.e, ie), vec(p.g, ig)
        moved_e = np.any(pr != p0, axis=1) | np.any(vec(ge) != p0, axis=1)
        moved_g = np.any(kr != k0, axis=1) | np.any(vec(gg) != k0, axis=1)
        ee = np.linalg.norm(vec(ge) - pr, axis=1)[moved_e] / np.sqrt(1.0 + (pr * pr).sum(1))[moved_e]
        eg = np.linalg.norm(vec(gg) - kr, axis=1)[moved_g] / np.linalg.norm(kr, axis=1)[moved_g]
        unmoved_same = bool(np.array_equal(vec(ge)[~moved_e], p0[~moved_e]) and
                            np.array_equal(vec(gg)[~moved_g], k0[~moved_g]))
        q = lambda a, f: float(f(a)) if a.size else 0.0  # noqa: E731
        errs[sampler] = {"events": int(moved_g.sum()),
                         "photon_rel_err": {"median": q(eg, np.median), "p99": q(eg, lambda a: np.percentile(a, 99)),
                                            "max": q(eg, np.max)},
                         "electron_rel_err": {"median": q(ee, np.median),
                                              "p99": q(ee, lambda a: np.percentile(a, 99)), "max": q(ee, np.max)},
                         "untouched_bitwise": unmoved_same}
    return cpu, {"cells": int(cells.size), "step": 0, "metric": "|k - k_ref| / eps_ref, |p - p_ref| / gamma_ref "
                 "per moved particle against the FP64 oracle's plain-sampler step", **errs}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; multi-GPU sharding is a design note, "
                                   "not an implemented path", "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    from paper_2206_02937_amd import compton, plasma

    copy_bw = hbm_copy_stage()
    print(json.dumps({"progress": "hbm copy", **copy_bw}), flush=True)
    p = plasma.make(args.workload, seed=0)
    n_pairs = p.n_pairs
    ctx = compton.Context(0)
    ctx.set_strategy(args.strategy)
    ctx.set_chunks_per_block(args.chunks_per_block)
    net = load_network(ctx, args.sampler)
    if args.sweep:
        sweep(ctx, p, args, net)
    tuned = None
    if args.autotune:
        e, g, oe, og = compton.to_device(p)
        tuned = ctx.autotune(e, g, oe, og, p.dt, p.density_norm, p.seed, 0, sampler=args.sampler, mlp=net, reps=5)
        print(json.dumps({"progress": "autotune", **tuned}), flush=True)
        del e, g, oe, og
    if compton.STRATEGY_NAMES[ctx.get_option(compton.OPT_STRATEGY)] not in ("fused", "compact"):
        args.graph = False  # graphs capture the fused or compact strategy only
    launch = launch_tag(ctx)  # the pair kernel's configuration, for the counter records
    print(json.dumps({"progress": "timing", "sampler": args.sampler}), flush=True)
    # per-stage timing (eager) for the roofline, then the measured run
    eager = run_steps(ctx, p, args.sampler, net, args.steps, args.warmup)
    main_run = run_steps(ctx, p, args.sampler, net, args.steps, args.warmup, graph=True) if args.graph else eager
    plain_run = None
    if args.sampler != "plain" and not args.no_plain:
        print(json.dumps({"progress": "timing", "sampler": "plain"}), flush=True)
        plain_run = run_steps(ctx, p, "plain", None, args.steps, args.warmup, graph=args.graph)
    base_run = None
    if args.baseline:
        print(json.dumps({"progress": "timing", "baseline": args.baseline}), flush=True)
        saved = (ctx.get_option(compton.OPT_STRATEGY), ctx.get_option(compton.OPT_CHUNKS_PER_BLOCK))
        ctx.set_strategy(args.baseline)
        ctx.set_chunks_per_block(0)
        base_run = run_steps(ctx, p, "plain", None, args.steps, args.warmup)
        ctx.set_option(compton.OPT_STRATEGY, saved[0])
        ctx.set_option(compton.OPT_CHUNKS_PER_BLOCK, saved[1])
    fp8_run = None
    if net is not None and args.sampler != "mlp_fp8":
        print(json.dumps({"progress": "timing", "sampler": "mlp_fp8"}), flush=True)
        fp8_run = run_steps(ctx, p, "mlp_fp8", net, args.steps, args.warmup, graph=args.graph)
    print(json.dumps({"progress": "sampler stage"}), flush=True)
    stage, ks = sampler_stage(ctx, p, net, args.sampler)

    sb = storage_bytes(p.e["x"].dtype)
    st = main_run["last_stats"]
    acc_per_step = st["n_collided"]
    stage_ms = eager["stage_ms"]
    # algorithmic bytes of the dominant kernel (k_step, fused strategy: every
    # pair reads both particles, 8 values; every collision writes 6 values
    # back); for the other strategies the pair and collide kernels separately
    # (compact: the pair kernel stashes each accepted pair's 8 values and two
    # indices and writes its 4-byte list slot, which the collide kernel reads
    # back; multi-kernel: an 8-byte index pair per accepted pair, and the
    # collide kernel gathers the 8 values)
    strategy_used = compton.STRATEGY_NAMES[ctx.get_option(compton.OPT_STRATEGY)]
    if strategy_used == "fused":
        kern, ms = "k_step", stage_ms["pair"]
        bytes_launch = n_pairs * 8 * sb + acc_per_step * 6 * sb
    else:
        kern = "k_pair_compact" if strategy_used == "compact" else "k_pair"
        ms = stage_ms["pair"]
        per_acc = 8 * sb + 8 + 4 if strategy_used == "compact" else 8
        bytes_launch = n_pairs * 8 * sb + acc_per_step * per_acc
        if stage_ms["collide"] > ms:
            kern = "k_collide_dense" if strategy_used == "compact" else "k_collide"
            ms = stage_ms["collide"]
            bytes_launch = acc_per_step * (per_acc + 8 * sb + 6 * sb if strategy_used != "compact"
                                           else per_acc + 6 * sb)
    # the library's stage events bracket each kernel; with the compact
    # strategy the "compact" stage is an empty bracket (two events back to
    # back), i.e. the events' own cost, which is taken off the kernel's time
    overhead = stage_ms["compact"] if strategy_used == "compact" else 0.0
    ms_events = ms
    ms = ms_events - overhead
    achieved = bytes_launch / (ms * 1e-3) / 1e9
    roof = {"kernel": kern, "bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": traffic_record(kern, p.name, launch),
            "bytes_per_launch": bytes_launch, "avg_ms": ms, "avg_ms_events": ms_events,
            "event_overhead_ms": overhead,
            "units_per_launch": f"{n_pairs} pairs, {acc_per_step} collisions", "launch": launch,
            "valu": valu_roofline(kern, p.name, ms, n_pairs, launch) if kern == "k_pair_compact" else None}
    roof_mlp = mfma_roofline("mlp_bf16", stage, ks)
    roof_mlp_fp8 = mfma_roofline("mlp_fp8", stage, ks)
    uneven = power = None
    if not args.no_workloads:
        from paper_2206_02937_amd import plasma as plasma_mod

        print(json.dumps({"progress": "uneven workload"}), flush=True)
        pu = plasma_mod.make("uneven", seed=0)
        uneven = workload_stage(ctx, pu, net, ["plain", "mlp_bf16"], args.steps, args.warmup, baseline="per_cell")
        del pu
        print(json.dumps({"progress": "power-law workload"}), flush=True)
        pw = plasma_mod.make("power_law", seed=0)
        power = workload_stage(ctx, pw, net, ["plain", "mlp_bf16", "mlp_fp8"], args.steps, args.warmup)
    print(json.dumps({"progress": "binning"}), flush=True)
    binned = binning_stage(ctx, p)
    print(json.dumps({"progress": "probability network"}), flush=True)
    pnet = pnet_stage(ctx, p)
    print(json.dumps({"progress": "ntc"}), flush=True)
    ntc = ntc_stage(ctx, p)
    print(json.dumps({"progress": "beam_gas"}), flush=True)
    beam = beam_gas_stage(ctx, net, args.sampler)
    print(json.dumps({"progress": "training"}), flush=True)
    training = training_stage(ctx)
    cpu = parity = None
    if not args.no_cpu:
        print(json.dumps({"progress": "cpu baseline"}), flush=True)
        samplers = ["plain"] + ([] if net is None else ["mlp_bf16", "mlp_fp8"])
        cpu, parity = oracle_leg(ctx, p, net, samplers, args.cpu_seconds)
        if power is not None:
            _, power["error_vs_oracle"] = oracle_leg(ctx, pw, net, samplers, 0.0, n_cells_err=64)

    dtype = {"plain": "f64", "mlp_f32": "f64/f32", "mlp_bf16": "f64/bf16", "mlp_fp8": "f64/fp8"}[args.sampler]
    line = {
        "metric": METRIC,
        "value": main_run["pairs_per_s"],
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{p.name}: {p.n_cells} cells, {n_pairs} pairs per step, "
                               f"{'fp32' if sb == 4 else 'fp64'} particles",
                   "cells": p.n_cells, "pairs_per_step": n_pairs, "sampler": args.sampler,
                   "strategy": strategy_used,
                   "chunks_per_block": ctx.get_option(compton.OPT_CHUNKS_PER_BLOCK),
                   "pairs_per_lane": ctx.get_option(compton.OPT_PAIRS_PER_LANE),
                   "autotuned": tuned is not None, "graph": args.graph,
                   "collisions_per_step": acc_per_step},
        "gpu_ms_per_step": main_run["gpu_ms_per_step"],
        "stage_ms": stage_ms,
        "eager_pairs_per_s": eager["pairs_per_s"],
        "plain": None if plain_run is None else {k: plain_run[k] for k in
                                                 ("pairs_per_s", "ms_per_step", "gpu_ms_per_step", "stage_ms")},
        "baseline": None if base_run is None else {"strategy": args.baseline, "sampler": "plain",
                                                   "pairs_per_s": base_run["pairs_per_s"],
                                                   "ms_per_step": base_run["ms_per_step"]},
        "autotune": tuned,
        "mlp_vs_plain": None if plain_run is None else main_run["pairs_per_s"] / plain_run["pairs_per_s"],
        "ks": {k: {"mu": v["mu"], "r": v["r"], "fallback_frac": v["fallback_frac"]} for k, v in ks.items()},
        "sampler_stage_samples_per_s": {k: v for k, v in stage.items() if k not in ("n", "inputs")},
        "fp8": None if fp8_run is None else {"pairs_per_s": fp8_run["pairs_per_s"],
                                             "ms_per_step": fp8_run["ms_per_step"],
                                             "vs_plain": None if plain_run is None else
                                             fp8_run["pairs_per_s"] / plain_run["pairs_per_s"]},
        "roofline": roof,
        "hbm_copy": copy_bw,
        "roofline_mlp": roof_mlp,
        "roofline_mlp_fp8": roof_mlp_fp8,
        "error_vs_oracle": parity,
        "uneven": uneven,
        "power_law": power,
        "binning": binned,
        "pnet": pnet,
        "ntc": ntc,
        "beam_gas": beam,
        "training": training,
        "cpu_baseline": cpu,
        "last_stats": st,
    }
    for r in (roof, (uneven or {}).get("roofline"), (power or {}).get("roofline"), (binned or {}).get("roofline"),
              (pnet or {}).get("roofline")):
        if r and r.get("bound") == "hbm":
            r["frac_of_copy"] = r["achieved"] / copy_bw["gbs"]
    print(json.dumps(line), flush=True)
    if args.traffic_calibration:
        # a plain copy kernel of known size: its FETCH_SIZE / WRITE_SIZE
        # readings give the counters' scale against bytes actually moved
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"traffic_calibration_bytes": src.numel() * 4}), flush=True)
    if net is not None:
        net.close()
    ctx.close()


def sweep(ctx, p, args, net):
    """Time each kernel strategy on the same initial state (printed as JSON
    lines tagged "sweep"); the measured run that follows uses the options
    given on the command line."""
    cands = [("compact", 0)] + [("fused", g) for g in (2, 4, 8, 16, 32)]
    if args.sampler == "plain":
        cands.append(("multi_kernel", 0))
    for strategy, gpb in cands:
        ctx.set_strategy(strategy)
        ctx.set_chunks_per_block(gpb)
        r = run_steps(ctx, p, args.sampler, net, 50, 3)
        print(json.dumps({"sweep": True, "strategy": strategy, "chunks_per_block": gpb,
                          "ms_per_step": r["ms_per_step"], "pairs_per_s": r["pairs_per_s"],
                          "stage_ms": r["stage_ms"]}), flush=True)
    ctx.set_strategy(args.strategy)
    ctx.set_chunks_per_block(args.chunks_per_block)


if __name__ == "__main__":
    main()
