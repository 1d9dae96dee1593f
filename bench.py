"""Benchmark: grayscale reconstruction by dilation on one MI355X.

Default workload: one 16384 x 16384 uint8 image, 8-connectivity, synthetic
tissue-like input (12 800 bright disks on a blurred noise background,
seed 0), marker = max(mask - 30, 0). A step is one complete
``mr_recon_dilate`` call (clip, tile rounds, seed compaction, queue phase) on
an input already resident in HBM; every timed step works on its own fresh
copy of the marker, so nothing is restored inside the timed region.

Prints one JSON line (see the keys below). ``--gpus`` above 1 is refused:
this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=16384)
    ap.add_argument("--dtype", default="u8", choices=["u8", "i32"])
    ap.add_argument("--conn", type=int, default=8, choices=[4, 8])
    ap.add_argument("--tune", default="", help="k=v,... overrides of mr_tune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_0378_amd import build as libbuild
    from paper_1311_0378_amd import mrecon, synth

    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    dev = torch.device("cuda:0")
    S, dt, conn = args.size, args.dtype, args.conn
    tune = None
    if args.tune:
        tune = dict(kv.split("=") for kv in args.tune.split(","))
        tune = {k: int(v) for k, v in tune.items()}

    t0 = time.time()
    n_disks = synth.density_disks(S, S) if S != 16384 else 12800
    marker, mask = synth.make_tile(S, S, n_disks, 0, dt, 0.0)
    log(f"generated {S}x{S} {dt} in {time.time() - t0:.1f}s")
    tdt = torch.uint8 if dt == "u8" else torch.int32
    d_mask = torch.from_numpy(mask).to(dev)
    d_src = torch.from_numpy(marker).to(dev)
    K, W = args.steps, args.warmup
    copies = [torch.empty_like(d_src) for _ in range(K)]
    ws = mrecon.alloc_workspace(
        mrecon.workspace_bytes(mrecon.MR_OP_RECON, S, S, tdt, conn, tune), dev)
    stream = torch.cuda.current_stream()

    for i in range(W):
        copies[0].copy_(d_src)
        mrecon.recon_dilate(copies[0], d_mask, conn, tune=tune, workspace=ws, stream=stream)
    for c in copies:
        c.copy_(d_src)
    torch.cuda.synchronize()

    t_start = time.perf_counter()
    for i in range(K):
        mrecon.recon_dilate(copies[i], d_mask, conn, tune=tune, workspace=ws, stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    counters = mrecon.read_counters(ws)

    npx = S * S
    ms_per_step = elapsed * 1e3 / K
    value = npx * K / elapsed / 1e6
    T = 1 if dt == "u8" else 4
    result = {
        "metric": "reconstructed Mpixel/s (bit-exact)",
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": {"workload": f"recon_dilate {S}x{S} {dt} conn{conn}, {n_disks} disks, seed 0",
                   "global_batch": 1, "parallelism": "single-gpu"},
        "counters": counters,
    }

    got = copies[K - 1].cpu().numpy()
    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        want, ocnt = oracle.recon_dilate(marker, mask, conn)
        t_or = time.perf_counter() - t1
        if not args.no_verify:
            result["bit_exact"] = bool(np.array_equal(got, want))
            log("bit-exact vs oracle:", result["bit_exact"])
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = {
                "value": round(npx / t_or / 1e6, 2), "unit": "Mpixel/s", "cores": 1,
                "kind": "oracle",
                "sample": f"the full {S}x{S} image, one sequential run ({t_or:.1f} s) on "
                          f"{cpu_model()} ({os.cpu_count()} threads visible)"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
