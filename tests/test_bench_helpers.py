"""CPU checks of the benchmark's own arithmetic and bookkeeping: the counter
records it reads from profiles/ (matched to the kernel sources they were
taken with), the VALU-issue and MFMA rooflines built from them, the pair
kernel's algorithmic bytes, and the refusal of more than one GPU."""
import os
import re
import subprocess
import sys
from types import SimpleNamespace

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_committed_records_are_well_formed():
    """Every record line of the committed counter summaries names a kernel,
    a workload, an integer figure and a 16-hex-digit source digest."""
    pat = {
        "traffic-record:": ("bytes_per_launch",),
        "valu-record:": ("valu_busy_cycles", "valu_insts", "waves"),
    }
    n = 0
    prof = os.path.join(ROOT, "profiles")
    for f in sorted(os.listdir(prof)):
        if not (f.startswith("counters_") and f.endswith(".md")):
            continue
        for line in open(os.path.join(prof, f)):
            for tag, keys in pat.items():
                if not line.startswith(tag):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                assert kv["kernel"] and kv["workload"]
                assert re.fullmatch(r"[0-9a-f]{16}", kv["source_sha"])
                for k in keys:
                    assert int(kv[k]) > 0
                n += 1
    assert n >= 2


def _fake_tree(tmp_path, body):
    """A repository root with one kernel source and one counter summary."""
    (tmp_path / "paper_2206_02937_amd" / "csrc").mkdir(parents=True)
    (tmp_path / "paper_2206_02937_amd" / "csrc" / "k.hip").write_text("// kernel\n")
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "counters_x.md").write_text(body)


def test_records_are_matched_to_the_kernel_sources(tmp_path, monkeypatch):
    """A record counts only when its digest is that of the current sources:
    after a source change the benchmark reports null instead of a stale
    figure."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_tree(tmp_path, "")
    digest = bench.source_digest()
    assert re.fullmatch(r"[0-9a-f]{16}", digest)
    (tmp_path / "profiles" / "counters_x.md").write_text(
        f"traffic-record: kernel=k_a workload=w1 bytes_per_launch=1234 source_sha={digest}\n"
        f"traffic-record: kernel=k_a workload=w2 bytes_per_launch=99 source_sha=0000000000000000\n")
    assert bench.traffic_record("k_a", "w1") == 1234
    assert bench.traffic_record("k_a", "w2") is None  # another digest
    assert bench.traffic_record("k_b", "w1") is None  # another kernel
    (tmp_path / "paper_2206_02937_amd" / "csrc" / "k.hip").write_text("// kernel, changed\n")
    assert bench.source_digest() != digest
    assert bench.traffic_record("k_a", "w1") is None


def test_records_are_matched_to_the_launch_configuration(tmp_path, monkeypatch):
    """A record that names a launch configuration (pairs per lane, chunks
    per pair block) counts only for that configuration: the autotuner may
    pick another one, whose traffic the record does not describe."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_tree(tmp_path, "")
    d = bench.source_digest()
    (tmp_path / "profiles" / "counters_x.md").write_text(
        f"traffic-record: kernel=k_a launch=ppl1_g16 workload=w bytes_per_launch=111 source_sha={d}\n"
        f"traffic-record: kernel=k_a launch=ppl2_g16 workload=w bytes_per_launch=222 source_sha={d}\n"
        f"valu-record: kernel=k_a launch=ppl2_g16 workload=w valu_busy_cycles=10 valu_insts=5 waves=1 "
        f"source_sha={d}\n")
    assert bench.traffic_record("k_a", "w", "ppl1_g16") == 111
    assert bench.traffic_record("k_a", "w", "ppl2_g16") == 222
    assert bench.traffic_record("k_a", "w", "ppl1_g32") is None
    assert bench.valu_roofline("k_a", "w", 1.0, 1, "ppl1_g16") is None
    assert bench.valu_roofline("k_a", "w", 1.0, 1, "ppl2_g16")["valu_busy_cycles_per_launch"] == 10
    ctx = SimpleNamespace(get_option=lambda o: {bench_opt("OPT_PAIRS_PER_LANE"): 2,
                                                bench_opt("OPT_CHUNKS_PER_BLOCK"): 16}[o])
    assert bench.launch_tag(ctx) == "ppl2_g16"


def bench_opt(name):
    from paper_2206_02937_amd import compton

    return getattr(compton, name)


def test_valu_roofline_arithmetic(tmp_path, monkeypatch):
    """Busy SIMD cycles per launch against 1024 SIMDs x 2.4 GHz x the live
    duration; instructions per unit = wavefront instructions x 64 / units."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _fake_tree(tmp_path, "")
    d = bench.source_digest()
    (tmp_path / "profiles" / "counters_x.md").write_text(
        f"valu-record: kernel=k_a workload=w valu_busy_cycles=49152000 valu_insts=1000000 waves=4096 "
        f"source_sha={d}\n")
    r = bench.valu_roofline("k_a", "w", 0.04, 2**22)
    avail = 0.04e-3 * 1024 * 2.4e9
    assert r["frac"] == pytest.approx(49152000 / avail, rel=1e-12)
    assert r["frac"] == pytest.approx(0.5, rel=1e-12)
    assert r["valu_insts_per_unit"] == pytest.approx(1000000 * 64 / 2**22, rel=1e-12)
    assert bench.valu_roofline("k_a", "other", 0.04, 1) is None


def test_mfma_roofline_and_silu_ceiling():
    """Three 64x64 hidden layers, 2 flops per multiply-add, per sample; the
    SiLU ceiling is two transcendental instructions per activation, 256
    activations per sample, over 1024 SIMDs."""
    assert bench.MLP_MFMA_FLOPS == 3 * 64 * 64 * 2
    n, t = 1 << 22, 0.3e-3
    r = bench.mfma_roofline("mlp_bf16", {"n": n}, {"mlp_bf16": {"t": t}})
    assert r["achieved"] == pytest.approx(n * 24576 / t / 1e12, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] / 2500.0, rel=1e-12)
    assert r["samples_per_s"] == pytest.approx(n / t, rel=1e-12)
    ceiling = 1024 * 2.4e9 * 64 / (2 * 256 * bench.TRANS_CYCLES)
    assert r["silu_ceiling_samples_per_s"] == pytest.approx(ceiling, rel=1e-12)
    assert r["silu_frac"] == pytest.approx(n / t / ceiling, rel=1e-12)
    r8 = bench.mfma_roofline("mlp_fp8", {"n": n}, {"mlp_fp8": {"t": t}})
    assert r8["frac"] == pytest.approx(r8["achieved"] / 5000.0, rel=1e-12)
    assert bench.mfma_roofline("mlp_bf16", {"n": n}, {}) is None


def test_pair_roofline_bytes(monkeypatch):
    """Algorithmic bytes of the pair kernel: 8 particle values per pair,
    plus per collision its stash entry's 8 values and 12 bytes of indices
    and list slot; the time is the pair stage minus an empty bracket."""
    monkeypatch.setattr(bench, "traffic_record", lambda *a: None)
    monkeypatch.setattr(bench, "valu_roofline", lambda *a: None)
    p = SimpleNamespace(e={"x": np.zeros(1, np.float32)}, n_pairs=1 << 22, name="w", nbytes=lambda: 2**27)
    run = {"last_stats": {"n_collided": 100000}, "stage_ms": {"pair": 0.046, "compact": 0.005}}
    r = bench.pair_roofline(p, run, "compact")
    b = (1 << 22) * 8 * 4 + 100000 * (8 * 4 + 12)
    assert r["bytes_per_launch"] == b
    assert r["avg_ms"] == pytest.approx(0.041, rel=1e-12)
    assert r["achieved"] == pytest.approx(b / 0.041e-3 / 1e9, rel=1e-12)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0, rel=1e-12)
    assert bench.pair_roofline(p, run, "fused") is None
    p64 = SimpleNamespace(e={"x": np.zeros(1, np.float64)}, n_pairs=1 << 22, name="w", nbytes=lambda: 2**28)
    assert bench.pair_roofline(p64, run, "compact")["bytes_per_launch"] == (1 << 22) * 64 + 100000 * 76


def test_more_than_one_gpu_is_refused():
    """bench.py --gpus 2 prints why and exits before touching a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout and '"n_gpus": 2' in r.stdout
