"""Benchmark: MLUPS and HBM-roofline fraction of the fused D3Q27 cumulant
stream-collide on a 512^3 periodic box (seeded random-phase velocity field,
spectrum k^4 exp(-2 (k/8)^2), u_rms 0.03, omega 1.9), populations stored in
FP32 (the reported value) and as FP16 / BF16 deviations (variants).

One step = one lbm_step(1): the whole per-step kernel sequence of the path
for this workload (one fused stream-collide launch; no rotor, no closure in
the base case). Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2402_13171_amd import roofline  # noqa: E402


def targets(results, base):
    """The throughput targets of the workload, each with its measured value and
    whether it is met: FP32 stream-collide at >= 80 % of the 8 TB/s HBM peak,
    and the 16-bit-stored variants (with and without the learned closure) at
    >= 1.7 times the FP32 MLUPS. Only variants that were run are listed."""
    out = {}
    if "f32" in results:
        f = results["f32"]["hbm_frac"]
        out["f32_frac_of_hbm_peak"] = {"value": round(f, 4), "target": 0.80, "met": bool(f >= 0.80)}
    for k in ("f16", "bf16", "f16+mlp"):
        if k in results and "f32" in results:
            r = results[k]["mlups"] / base["mlups"]
            out[f"{k}_vs_f32"] = {"value": round(r, 3), "target": 1.7, "met": bool(r >= 1.7)}
    return out


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_variant(n, rho, u, storage, closure, steps, warmup, blob=None):
    import torch
    from paper_2402_13171_amd.lbm import Lbm
    sim = Lbm(n, n, n, omega=1.9, storage=storage, closure=closure, cs_smag=0.1)
    if blob is not None:
        sim.set_closure_weights(blob)
    # the access pattern alone (same buffers, tiles and addressing, no
    # collision): the achievable ceiling of this kernel's memory traffic
    probe_passes = 10
    for par in (0, 1):
        sim.pattern_probe(par)
    torch.cuda.synchronize()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(sim.stream)
    for k in range(probe_passes):
        sim.pattern_probe(k % 2)
    p1.record(sim.stream)
    torch.cuda.synchronize()
    probe_ms = p0.elapsed_time(p1) / probe_passes
    sim.init_fields(rho, u)
    sim.step(warmup)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    t0 = time.perf_counter()
    sim.step(steps)
    e1.record(sim.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    m, mom, ke = sim.global_moments()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    mlups = n ** 3 * steps / (ms * 1e-3) / 1e6
    return {"mlups": mlups, "ms_per_step": ms / steps, "wall_s": wall, "mass": m, "ke": ke,
            "pattern_ms": probe_ms}


def closure_weights():
    """Trained closure weights if the training run has been committed, else a
    seeded He-initialised network (the kernel's cost does not depend on the
    weight values)."""
    import numpy as np
    path = os.path.join(ROOT, "results", "closure_weights.npy")
    if os.path.exists(path):
        return np.load(path).astype(np.float64), "results/closure_weights.npy"
    rng = np.random.default_rng(0)
    blob = np.zeros(1326)
    blob[0:192] = rng.standard_normal(192) * np.sqrt(2.0 / 6.0)
    blob[224:1248] = rng.standard_normal(1024) * np.sqrt(2.0 / 32.0)
    blob[1280:1312] = rng.standard_normal(32) * np.sqrt(1.0 / 32.0)
    blob[1319:1325] = 1e-3
    blob[1325] = 1e-3
    return blob, "seeded random network (no trained weights committed)"


def copy_bandwidth(gib=4, reps=10):
    """Achievable HBM bandwidth: the library's streaming copy kernel over two
    gib-GiB buffers (bytes read + bytes written per second), as the paper
    takes b_S from the STREAM copy kernel."""
    import torch
    from paper_2402_13171_amd.lbm import copy_probe
    nb = gib << 30
    a = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    copy_probe(a, b, s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        copy_probe(a, b, s)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(a[:1024], b[:1024]))
    del a, b
    torch.cuda.empty_cache()
    return {"GBps": 2 * nb / (ms * 1e-3) / 1e9, "ms_per_copy": ms, "bytes": nb, "verified": ok}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_stream_collide_512cube_traffic.txt")
KERNEL_SOURCES = ["lbm_lattice.hip", "lbm_access.h", "lbm_device.h", "lbm_mlp_dev.h", "lbm_internal.h"]


def measured_traffic():
    """HBM bytes per stream-collide launch from the committed FETCH_SIZE /
    WRITE_SIZE summary, or {} if the kernel sources changed since."""
    import hashlib
    if not os.path.exists(TRAFFIC_FILE):
        return {}
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2402_13171_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = (t.strip() for t in line.split("=", 1))
                vals[k] = v
    if vals.get("source_sha256_16") != h.hexdigest()[:16]:
        return {}
    return {k: float(v) for k, v in vals.items() if k != "source_sha256_16"}


def cpu_model():
    """The host CPU's model name (first entry of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample_n=128, steps=100):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    recipe (a sample_n^3 periodic box, same spectrum and omega)."""
    import oracle
    import workloads
    rho, u = workloads.random_phase_field(sample_n, seed=0)
    g = oracle.Grid(sample_n, sample_n, sample_n, omega=1.9)
    g.init_fields(rho, u)
    g.step(1)  # warm-up
    t0 = time.perf_counter()
    g.step(steps)
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": sample_n ** 3 * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
            "cpu_model": cpu_model(), "kind": "oracle",
            "sample": f"{sample_n}^3 periodic box of the same random-phase recipe, {steps} steps, "
                      f"FP64 two-array oracle ({dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--variants", default="f32,f16,bf16,f32+smag,f16+mlp")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import workloads
    n = args.n
    log(f"bench: generating {n}^3 random-phase field (seed 0)")
    t0 = time.perf_counter()
    rho, u = workloads.random_phase_field(n, seed=0)
    log(f"bench: field ready in {time.perf_counter() - t0:.1f} s")

    log("bench: copy-kernel bandwidth probe (2 x 4 GiB)")
    cbw = copy_bandwidth()
    log(f"bench: copy probe {cbw['GBps']:.0f} GB/s")

    blob, blob_src = closure_weights()
    results = {}
    for v in args.variants.split(","):
        storage, _, closure = v.partition("+")
        closure = closure or "none"
        log(f"bench: variant {v}: {args.warmup} warm-up + {args.steps} timed steps")
        r = time_variant(n, rho, u, storage, closure, args.steps, args.warmup,
                         blob=blob if closure == "mlp" else None)
        s_bytes = 4 if storage == "f32" else 2
        nb = roofline.bytes_per_lup(s_bytes)
        bw = roofline.achieved_bandwidth(r["mlups"] * 1e6, nb)
        r.update({"bytes_per_lup": nb, "achieved_GBps": bw / 1e9,
                  "hbm_frac": bw / roofline.HBM_PEAK_BPS,
                  "pattern_GBps": nb * n ** 3 / (r["pattern_ms"] * 1e-3) / 1e9})
        results[v] = r
        log(f"bench: {v}: {r['mlups']:.0f} MLUPS, {r['ms_per_step']:.3f} ms/step, "
            f"{bw / 1e9:.0f} GB/s algorithmic ({100 * bw / roofline.HBM_PEAK_BPS:.1f}% of 8 TB/s; "
            f"access-pattern probe {r['pattern_GBps']:.0f} GB/s)")

    base = results.get("f32") or next(iter(results.values()))
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline()
        log(f"bench: oracle {cpu['value']:.2f} MLUPS on {cpu['cores']} cores")

    nb = base["bytes_per_lup"]
    measured = measured_traffic() if n == 512 else {}
    traffic = measured.get("f32")
    out = {
        "metric": "MLUPS & % HBM roofline, D3Q27 512^3: FP32 vs FP16-store(+learned closure)",
        "value": round(base["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(base["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q27 cumulant, {n}^3 periodic, random-phase field seed 0 "
                               "(k^4 exp(-2(k/8)^2), u_rms 0.03), omega 1.9, FP32-stored populations",
                   "n": n, "storage": "f32", "closure": "none", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(base["achieved_GBps"], 1),
                     "peak": roofline.HBM_PEAK_BPS / 1e9, "unit": "GB/s",
                     "frac": round(base["hbm_frac"], 4),
                     "traffic": traffic, "traffic_unit": "HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_stream_collide", "bytes_per_lup": nb,
                     "bytes_per_launch": nb * n ** 3},
        "cpu_baseline": cpu,
        "pattern_probe": {"GBps": round(base["pattern_GBps"], 1), "ms_per_pass": round(base["pattern_ms"], 4),
                          "kernel_frac_of_pattern": round(base["achieved_GBps"] / base["pattern_GBps"], 4)},
        "copy_probe": {"GBps": round(cbw["GBps"], 1), "bytes": cbw["bytes"],
                       "frac_of_peak": round(cbw["GBps"] * 1e9 / roofline.HBM_PEAK_BPS, 4),
                       "kernel_frac_of_copy": round(base["achieved_GBps"] / cbw["GBps"], 4)},
        "closure_weights": blob_src,
        "variants": {k: {"mlups": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                         "achieved_GBps": round(v["achieved_GBps"], 1),
                         "hbm_frac": round(v["hbm_frac"], 4), "bytes_per_lup": v["bytes_per_lup"],
                         "ratio_vs_f32": round(v["mlups"] / base["mlups"], 3),
                         "traffic": measured.get(k),
                         "pattern_probe_GBps": round(v["pattern_GBps"], 1),
                         "frac_of_pattern_probe": round(v["achieved_GBps"] / v["pattern_GBps"], 4)}
                     for k, v in results.items()},
    }
    out["targets"] = targets(results, base)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
