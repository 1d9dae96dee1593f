"""Benchmark: grayscale reconstruction by dilation on one MI355X.

Workload (default): one 16384 x 16384 uint8 image, 8-connectivity, synthetic
tissue-like input (12 800 bright disks of radius 5-15 on a Gaussian-blurred
noise background, seed 0), marker = max(mask - 30, 0).

A step is one complete ``mr_recon_dilate`` call -- clip, tile rounds, and
(when the tuning leaves work for it) the seed pass and the queue phase -- on
an input already resident in HBM. Every timed step works on its own fresh
marker copy and its own workspace, so nothing is restored inside the timed
region and every launch's tile count can be read back afterwards.

Prints one JSON line. ``roofline`` is for the dominant kernel, the tile
round: algorithmic bytes per launch = tiles visited x (interior pixels per
tile) x 3 bytes per pixel (read J, read the mask, write J), over the launch's
duration measured with HIP events on the call's stream during the timed
steps. ``--gpus`` above 1 is refused: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published peak


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


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1311_0378_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(workload_key: str):
    """HBM bytes per tile-round launch from the committed rocprofv3 counter
    runs, if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "tile_round_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources") != kernel_source_hash() or rec.get("workload") != workload_key:
        return None
    return rec.get("hbm_bytes_per_launch")


def summarize_traffic(fetch_csv: str, write_csv: str, args) -> None:
    """HBM traffic per tile-round launch: the FETCH_SIZE and WRITE_SIZE
    counters (KiB per dispatch) of the tile-round dispatches, each scaled by
    known bytes / counter reading of the 1 GiB calibration copy in the same
    run."""
    import csv

    def per_dispatch(path, counter):
        rows = {}
        for r in csv.DictReader(open(path)):
            if r.get("Counter_Name", r.get("counter_name")) != counter:
                continue
            did = int(r.get("Dispatch_Id", r.get("dispatch_id")))
            name = r.get("Kernel_Name", r.get("kernel_name"))
            val = float(r.get("Counter_Value", r.get("value")))
            rows.setdefault(did, [name, 0.0])[1] += val
        return [rows[k] for k in sorted(rows)]

    out = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        disp = per_dispatch(path, counter)
        copy_kib = [v for n, v in disp if "copy" in n.lower() or "elementwise" in n.lower()]
        tiles = [v for n, v in disp if "k_tile_round" in n]
        if not copy_kib or not tiles:
            raise SystemExit(f"{path}: no calibration copy or tile-round dispatch found")
        scale = (1 << 30) / (max(copy_kib) * 1024.0)
        out[key] = {"scale": scale, "kib_per_launch_raw": [round(v, 1) for v in tiles],
                    "bytes_per_launch": [v * 1024.0 * scale for v in tiles]}
    n = min(len(out["fetch"]["bytes_per_launch"]), len(out["write"]["bytes_per_launch"]))
    per_launch = [out["fetch"]["bytes_per_launch"][i] + out["write"]["bytes_per_launch"][i]
                  for i in range(n)]
    rec = {
        "workload": f"recon {args.size}x{args.size} {args.dtype} conn{args.conn}",
        "kernel_sources": kernel_source_hash(),
        "fetch_scale": out["fetch"]["scale"], "write_scale": out["write"]["scale"],
        "hbm_bytes_per_launch": sum(per_launch) / max(1, n),
        "launches": n,
        "fetch_kib_raw": out["fetch"]["kib_per_launch_raw"],
        "write_kib_raw": out["write"]["kib_per_launch_raw"],
    }
    path = os.path.join(ROOT, "profiles", "tile_round_traffic.json")
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))


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
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="copy 1 GiB on the device first (counter calibration)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--calibrate-copy run into profiles/tile_round_traffic.json and exit")
    args = ap.parse_args()

    if args.traffic_from:
        summarize_traffic(*args.traffic_from, args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
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
        tune = {k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))}

    t0 = time.time()
    n_disks = 12800 if S == 16384 else synth.density_disks(S, S)
    marker, mask = synth.make_tile(S, S, n_disks, 0, dt, 0.0)
    log(f"generated {S}x{S} {dt} in {time.time() - t0:.1f}s")
    tdt = torch.uint8 if dt == "u8" else torch.int32
    T = 1 if dt == "u8" else 4
    d_mask = torch.from_numpy(mask).to(dev)
    d_src = torch.from_numpy(marker).to(dev)
    K, W = args.steps, args.warmup
    wsb = mrecon.workspace_bytes(mrecon.MR_OP_RECON, S, S, tdt, conn, tune)
    copies = [torch.empty_like(d_src) for _ in range(K)]
    wss = [mrecon.alloc_workspace(wsb, dev) for _ in range(K)]
    stream = torch.cuda.current_stream()

    if args.calibrate_copy:
        a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    for i in range(W):
        copies[0].copy_(d_src)
        mrecon.recon_dilate(copies[0], d_mask, conn, tune=tune, workspace=wss[0], stream=stream)
    for c in copies:
        c.copy_(d_src)
    torch.cuda.synchronize()

    mrecon.timing_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(K):
        mrecon.recon_dilate(copies[i], d_mask, conn, tune=tune, workspace=wss[i], stream=stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    mrecon.timing_enable(False)
    launches = mrecon.timing_collect()

    # per-launch algorithmic bytes of the tile rounds, matched by round number
    n_tiles = ((S + 61) // 62) ** 2
    px_per_tile = S * S / n_tiles
    bytes_per_visit = 3 * T * px_per_tile
    per_step = []
    li = 0
    tile_ms, tile_bytes, tile_launches = 0.0, 0.0, 0
    seed_ms = queue_ms = 0.0
    for i in range(K):
        rt = mrecon.read_round_tiles(wss[i])
        cnt = mrecon.read_counters(wss[i])
        step_tiles = 0
        # launches of step i: tile rounds 1..R, then optionally seed and queue
        while li < len(launches):
            kind, rnd, ms = launches[li]
            if kind == "tile_round":
                if rnd == 1 and step_tiles:
                    break  # next step's first round
                visits = rt[rnd - 1] if rnd - 1 < len(rt) else 0
                step_tiles += visits
                if visits:
                    tile_ms += ms
                    tile_bytes += visits * bytes_per_visit
                    tile_launches += 1
            elif kind == "seed":
                seed_ms += ms
            elif kind == "queue":
                queue_ms += ms
            li += 1
        per_step.append({"tiles": step_tiles, "counters": cnt})

    npx = S * S
    ms_per_step = elapsed * 1e3 / K
    value = npx * K / elapsed / 1e6
    achieved = tile_bytes / (tile_ms * 1e-3) / 1e9 if tile_ms else 0.0
    b_alg_step = sum(p["tiles"] for p in per_step) / K * bytes_per_visit
    workload_key = f"recon {S}x{S} {dt} conn{conn}"
    traffic = load_traffic(workload_key)
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
        "roofline": {
            "bound": "hbm",
            "kernel": "k_tile_round",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "launches": tile_launches,
            "avg_launch_ms": round(tile_ms / max(1, tile_launches), 4),
            "bytes_per_tile_visit": round(bytes_per_visit, 1),
        },
        "whole_call": {
            "b_alg_gb_per_step": round(b_alg_step / 1e9, 4),
            "b_alg_gbs": round(b_alg_step / (ms_per_step * 1e-3) / 1e9, 1),
            "passes_equivalent": round(b_alg_step / (3 * T * npx), 3),
            "tile_round_ms_per_step": round(tile_ms / K, 4),
            "seed_ms_per_step": round(seed_ms / K, 4),
            "queue_ms_per_step": round(queue_ms / K, 4),
        },
        "counters_last_step": per_step[-1]["counters"],
        "tune": tune or "library default",
    }

    got = copies[K - 1].cpu().numpy()
    if not args.no_verify or not args.no_cpu_baseline:
        import oracle
        t1 = time.perf_counter()
        want, _ = oracle.recon_dilate(marker, mask, conn)
        t_or = time.perf_counter() - t1
        if not args.no_verify:
            result["bit_exact"] = bool(np.array_equal(got, want))
            log("bit-exact vs oracle:", result["bit_exact"])
        if not args.no_cpu_baseline:
            result["cpu_baseline"] = {
                "value": round(npx / t_or / 1e6, 2), "unit": "Mpixel/s", "cores": 1,
                "kind": "oracle",
                "sample": f"the whole {S}x{S} {dt} image, one sequential oracle run "
                          f"({t_or:.1f} s) on {cpu_model()}, {os.cpu_count()} threads visible"}
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
