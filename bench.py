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
steps. ``--gpus`` above 1 is refused: the library runs on one GPU.

More legs are added to the same line (``--legs``):

* ``i32``: the int32 variant of the headline image (values scaled to
  0..65535), measured the same way with its own ``roofline`` and
  ``bit_exact``.
* ``small``: the cache-resident configurations, 1024^2 recon conn8 and the
  4096^2 image's recon conn4 / conn8 and fill-holes conn4 / conn8: per-call
  p50 / p99 over 30 calls and Mpx/s, each checked against the oracle.
* ``batched``: 512 uneven u8 tiles (sides log-uniform 256-4096, per-tile
  seeds, ~1.0 Gpixel in all), reconstruction 8-conn: one ``mr_recon_dilate``
  per tile on one stream versus one batched launch sequence with the
  autotuner's settings (replayed as a HIP graph when the settings allow it).
  Every batched result is checked against the oracle, on all host cores,
  which also gives the leg's all-cores CPU baseline.
* ``served``: 2000 jobs (sides log-uniform 512-8192, 70 % reconstruction /
  30 % fill-holes, ~15 Gpixel). Each job is a window of one of two seeded
  8192 x 8192 images, its first column on a 64-byte boundary. Run twice: with
  the jobs in pinned host memory (PCIe in and out) and with the jobs already
  in HBM (device-to-device copies into and out of the arena). Compared each
  time: sequential per-job launches (copy in, one call, copy out, wait)
  versus the continuous-batching server with an 8 GiB arena and 128 job slots
  (--serve-slots), first back to back, then on one Poisson arrival trace at
  0.8 x the sequential capacity (p50/p99 of completion - arrival). Untimed
  passes afterwards hash every result of the sequential path and of the
  server, which must agree job by job, and every job is checked against the
  oracle on all host cores (the leg's all-cores CPU baseline).
* ``erode``: reconstruction by erosion (``mr_recon_erode``) on a 16384 x
  16384 u8 image, 8-conn, the same mask with the marker raised by 30: a
  complement pass, the reconstruction by dilation, the complement back.
  Checked against the oracle, whose time on one core is reported beside it.
* ``ops``: the other Table II operations on the same 16384^2 image: RGB2Gray,
  opening by the 13 x 13 disk, distance transform, CCL, area threshold,
  h-dome and regional maxima, each with its time, algorithmic bytes against
  the HBM peak, an oracle check, and the oracle's own time on one core
  (``cpu_oracle``; the opening's on the windows it checks).

The line also carries ``copy_bandwidth``: what a plain 1 GiB device copy
reaches, beside the 8 TB/s peak the rooflines use.

``--atomic-probe`` instead times the device atomic-rate probe
(``mr_probe_atomics``: relaxed device-scope add, and load + compare-and-swap,
on pseudo-random words of a 256 MiB and a 4 GiB buffer, every wave slot busy)
and prints its own JSON line: the ceiling for the queue phase's atomics.

``--random-probe`` times the random-access probe (``mr_probe_random``, the
paper's micro-benchmark for irregular access, Sec. V-A / Table III): plain
random reads and writes of 32-bit words of a 4K x 4K matrix (the paper's
64 MiB) and of a 4 GiB one (past the 256 MiB Infinity Cache), 10 million
operations (the paper's count) and 2^28, at positions drawn on the host into
an index vector. It prints its own JSON line in MB/s of 4-byte words, the
paper's unit, and in G operations/s.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import platform
import queue
import sys
import time
from concurrent.futures import ThreadPoolExecutor

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
    """Hash of the code (line comments and blank lines dropped) of the sources
    that define the tile-round kernel."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1311_0378_amd", "csrc")
    for f in ("mr_internal.h", "mr_kernels.hip"):
        for line in open(os.path.join(csrc, f), encoding="utf-8"):
            code = line.split("//", 1)[0].rstrip()
            if code:
                h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def traffic_path(size: int, dtype: str, conn: int) -> str:
    return os.path.join(ROOT, "profiles", f"tile_round_traffic_{size}_{dtype}_conn{conn}.json")


def load_traffic(workload_key: str, path: str):
    """HBM bytes per tile-round launch from the committed rocprofv3 counter
    runs, if they were taken on the current kernel sources."""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources") != kernel_source_hash() or rec.get("workload") != workload_key:
        return None
    return rec.get("hbm_bytes_per_launch")


def summarize_served_trace(trace_dir: str) -> None:
    """Busy time per server pass from a rocprofv3 kernel + memory-copy trace
    of the served leg. The passes are the stretches of k_server_* launches
    (gaps over 50 ms split them); for each: the window, the host<->device
    copies (memory-copy trace; device-to-device copies are kernels), the
    tile-round launches and the union of all activity. Prints one JSON line."""
    import csv

    def rows(name):
        path = os.path.join(trace_dir, name)
        return list(csv.DictReader(open(path))) if os.path.exists(path) else []

    def union_ms(iv):
        tot, cur = 0, None
        for a, b in sorted(iv):
            if cur is None or a > cur[1]:
                if cur:
                    tot += cur[1] - cur[0]
                cur = [a, b]
            else:
                cur[1] = max(cur[1], b)
        if cur:
            tot += cur[1] - cur[0]
        return round(tot / 1e6, 2)

    span = lambda r: (int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
    K, M = rows("run_kernel_trace.csv"), rows("run_memory_copy_trace.csv")
    starts = sorted(span(r)[0] for r in K if "k_server_" in r["Kernel_Name"])
    if not starts:
        sys.exit(f"no k_server_* launches in {trace_dir}/run_kernel_trace.csv")
    passes, cur = [], [starts[0]]
    for t in starts[1:]:
        if t - cur[-1] > 50e6:
            passes.append(cur)
            cur = [t]
        else:
            cur.append(t)
    passes.append(cur)
    out = []
    for p in passes:
        lo, hi = p[0], p[-1]
        k = [r for r in K if lo <= span(r)[0] <= hi]
        m = [r for r in M if lo <= span(r)[0] <= hi]
        rounds = [r for r in k if "k_tile_round" in r["Kernel_Name"]]
        out.append({"window_ms": round((hi - lo) / 1e6, 1), "host_copies": len(m),
                    "host_copy_busy_ms": union_ms([span(r) for r in m]),
                    "round_launches": len(rounds),
                    "round_busy_ms": union_ms([span(r) for r in rounds]),
                    "round_avg_us": round(sum(b - a for a, b in map(span, rounds))
                                          / max(1, len(rounds)) / 1e3, 1),
                    "any_busy_ms": union_ms([span(r) for r in k + m])})
    print(json.dumps({"served_trace": out}))


def summarize_traffic(fetch_csv: str, write_csv: str, args) -> None:
    """HBM traffic per tile-round launch: the FETCH_SIZE and WRITE_SIZE
    counters (KiB per dispatch) of the tile-round dispatches, each scaled by
    known bytes / counter reading of the 1 GiB calibration pass (the
    bitwise-not kernel of --calibrate-copy) in the same run."""
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
        copy_kib = [v for n, v in disp if "bitwise_not" in n.lower() or "bitwisenot" in n.lower()]
        tiles = [v for n, v in disp if "k_tile_round" in n]
        if not copy_kib or not tiles:
            raise SystemExit(f"{path}: no calibration pass or tile-round dispatch found")
        scale = (1 << 30) / (copy_kib[0] * 1024.0)
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
    path = traffic_path(args.size, args.dtype, args.conn)
    json.dump(rec, open(path, "w"), indent=1)
    print(json.dumps(rec))

def pct(xs, q) -> float:
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def measure_recon(args, torch, mrecon, dev, marker, mask, conn, tune) -> dict:
    """K whole mr_recon_dilate calls on fresh marker copies resident in HBM
    (after W warm-up calls), with the tile rounds timed by the library's
    events on the call's stream; every output checked equal, the last one
    against the oracle."""
    S = marker.shape[0]
    dt = "u8" if marker.dtype == np.uint8 else "i32"
    T = 1 if dt == "u8" else 4
    d_mask = torch.from_numpy(mask).to(dev)
    d_src = torch.from_numpy(marker).to(dev)
    K, W = args.steps, args.warmup
    wsb = mrecon.workspace_bytes(mrecon.MR_OP_RECON, S, S, d_src.dtype, conn, tune)
    copies = [torch.empty_like(d_src) for _ in range(K)]
    wss = [mrecon.alloc_workspace(wsb, dev) for _ in range(K)]
    stream = torch.cuda.current_stream()
    for i in range(W):
        copies[0].copy_(d_src)
        mrecon.recon_dilate(copies[0], d_mask, conn, tune=tune, workspace=wss[0], stream=stream)
    for c in copies:
        c.copy_(d_src)
    torch.cuda.synchronize()

    # span mode: one pair of events per run of consecutive tile rounds (its
    # average launch duration includes the dispatch gaps between them);
    # "launches" brackets every launch, at a few microseconds per event
    mrecon.timing_enable(args.timing)
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
    seed_ms = queue_ms = tq_ms = 0.0
    for i in range(K):
        mrecon.status(wss[i], stream)
        rt = mrecon.read_round_tiles(wss[i])
        cnt = mrecon.read_counters(wss[i])
        step_tiles = 0
        # launches of step i: tile rounds 1..R, then optionally seed and queue
        while li < len(launches):
            kind, rnd, ms, nl = launches[li]
            if kind == "tile_round":
                if rnd == 1 and step_tiles:
                    break  # next step's first round
                # every launch counts, also the few that find an empty list
                # after convergence, as in a profiler's per-kernel average; a
                # span record covers rounds rnd .. rnd + nl - 1
                visits = sum(rt[r - 1] for r in range(rnd, rnd + nl) if r - 1 < len(rt))
                step_tiles += visits
                tile_ms += ms
                tile_bytes += visits * bytes_per_visit
                tile_launches += nl
            elif kind == "seed":
                seed_ms += ms
            elif kind == "queue":
                queue_ms += ms
            elif kind == "tile_queue":
                tq_ms += ms
            li += 1
        per_step.append({"tiles": step_tiles, "counters": cnt, "round_tiles": rt})

    npx = S * S
    ms_per_step = elapsed * 1e3 / K
    achieved = tile_bytes / (tile_ms * 1e-3) / 1e9 if tile_ms else 0.0
    b_alg_step = sum(p["tiles"] for p in per_step) / K * bytes_per_visit
    workload_key = f"recon {S}x{S} {dt} conn{conn}"
    traffic = load_traffic(workload_key, traffic_path(S, dt, conn))
    out = {
        "mpx_s": round(npx * K / elapsed / 1e6, 1),
        "ms_per_call": round(ms_per_step, 4),
        "roofline": {
            "bound": "hbm",
            "kernel": "k_tile_round_pf" if dt == "u8" else "k_tile_round",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "launches": tile_launches,
            "avg_launch_ms": round(tile_ms / max(1, tile_launches), 4),
            "bytes_per_tile_visit": round(bytes_per_visit, 1),
            "timing": args.timing,
        },
        "whole_call": {
            "b_alg_gb_per_step": round(b_alg_step / 1e9, 4),
            "b_alg_gbs": round(b_alg_step / (ms_per_step * 1e-3) / 1e9, 1),
            "frac_of_peak": round(b_alg_step / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "passes_equivalent": round(b_alg_step / (3 * T * npx), 3),
            "tile_round_ms_per_step": round(tile_ms / K, 4),
            "seed_ms_per_step": round(seed_ms / K, 4),
            "queue_ms_per_step": round(queue_ms / K, 4),
            "tile_queue_ms_per_step": round(tq_ms / K, 4),
        },
        "counters_last_step": per_step[-1]["counters"],
        "round_tiles_last_step": [int(x) for x in per_step[-1]["round_tiles"]],
        "tune": tune or "library default",
    }
    # every timed output must be the same image; the last one then goes to
    # the oracle
    same = all(torch.equal(copies[i], copies[K - 1]) for i in range(K - 1))
    if not args.no_verify:
        import oracle
        got = copies[K - 1].cpu().numpy()
        want, _ = oracle.recon_dilate(marker, mask, conn)
        out["bit_exact"] = bool(same and np.array_equal(got, want))
        out["bit_exact_outputs_checked"] = K
        log(f"recon {S}x{S} {dt}: {ms_per_step:.3f} ms per call, bit-exact vs oracle:",
            out["bit_exact"])
    del copies, wss, d_mask, d_src
    return out


def copy_bandwidth(torch, dev, nbytes: int = 1 << 30, reps: int = 10) -> dict:
    """Achievable HBM bandwidth: a device-to-device copy of 1 GiB (read +
    write counted), timed with events, best of `reps`."""
    a = torch.ones(nbytes, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    best = 1e30
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    gbs = 2 * nbytes / (best * 1e-3) / 1e9
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "how": "torch device copy of 1 GiB, bytes read + written, best of 10"}


def leg_small(args, dev) -> dict:
    """The cache-resident configurations: 1024^2 u8 recon conn8, and on the
    4096^2 image (800 disks, 5 % rings) recon conn4 and conn8 and fill-holes
    conn4 and conn8 of the thresholded image. Each: per-call time over reps
    (p50 / p99) on fresh inputs in HBM, Mpx/s at p50, and the last output
    against the oracle."""
    import torch
    import oracle
    from paper_1311_0378_amd import mrecon, synth

    reps, warm = 30, 3
    stream = torch.cuda.current_stream()
    m1, k1 = synth.single_1024()
    m4, k4, b4 = synth.single_4096()
    cases = [("recon 1024x1024 u8 conn8", m1, k1, 8), ("recon 4096x4096 u8 conn4", m4, k4, 4),
             ("recon 4096x4096 u8 conn8", m4, k4, 8), ("fill 4096x4096 u8 conn4", b4, None, 4),
             ("fill 4096x4096 u8 conn8", b4, None, 8)]
    out = {}
    for name, a, m, conn in cases:
        src = torch.from_numpy(a).to(dev)
        dm = torch.from_numpy(m).to(dev) if m is not None else None
        op = mrecon.MR_OP_RECON if m is not None else mrecon.MR_OP_FILL
        ws = mrecon.alloc_workspace(mrecon.workspace_bytes(op, *a.shape, src.dtype, conn), dev)
        work = torch.empty_like(src)
        times = []
        for r in range(warm + reps):
            work.copy_(src)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            if m is not None:
                mrecon.recon_dilate(work, dm, conn, workspace=ws, stream=stream)
            else:
                mrecon.fill_holes(work, conn, workspace=ws, stream=stream)
            e1.record(stream)
            e1.synchronize()
            if r >= warm:
                times.append(e0.elapsed_time(e1))
        mrecon.status(ws, stream)
        ok = None
        if not args.no_verify:
            want = (oracle.recon_dilate(a, m, conn) if m is not None else oracle.fill_holes(a, conn))[0]
            ok = bool(np.array_equal(work.cpu().numpy(), want))
        p50 = pct(times, 50)
        out[name] = {"ms_p50": round(p50, 4), "ms_p99": round(pct(times, 99), 4),
                     "mpx_s": round(a.size / p50 / 1e3, 1), "reps": reps, "bit_exact": ok}
        log(f"small: {name} {p50:.3f} ms, exact {ok}")
    return out


def leg_batched(args, dev) -> dict:
    """512 uneven tiles: per-tile calls versus one batched launch sequence."""
    import torch
    import oracle
    from paper_1311_0378_amd import mrecon, synth

    n = args.batch_n
    shapes = synth.batch_shapes(n)
    t0 = time.time()
    with ThreadPoolExecutor(4) as ex:
        tiles = list(ex.map(lambda i: synth.batch_tile(i, *shapes[i], n=n), range(n)))
    npx = sum(H * W for H, W in shapes)
    log(f"batched: generated {n} tiles, {npx / 1e9:.3f} Gpx, in {time.time() - t0:.1f}s")
    src = [torch.from_numpy(m).to(dev) for m, _ in tiles]
    msk = [torch.from_numpy(k).to(dev) for _, k in tiles]
    work = [x.clone() for x in src]
    items = [(w, k, mrecon.MR_OP_RECON) for w, k in zip(work, msk)]
    stream = torch.cuda.current_stream()
    reps, warm = args.batch_reps, 1

    def restore():
        for w, x in zip(work, src):
            w.copy_(x)
        torch.cuda.synchronize()

    # one call per tile, library defaults, one workspace reused in stream order
    ws = mrecon.alloc_workspace(max(mrecon.workspace_bytes(mrecon.MR_OP_RECON, H, W, torch.uint8, 8)
                                    for H, W in shapes), dev)
    per_tile_s, lat_ms = [], []
    for rep in range(warm + reps):
        restore()
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
        t1 = time.perf_counter()
        evs[0].record(stream)
        for i in range(n):
            mrecon.recon_dilate(work[i], msk[i], 8, workspace=ws, stream=stream)
            evs[i + 1].record(stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        if rep >= warm:
            per_tile_s.append(dt)
            lat_ms += [evs[i].elapsed_time(evs[i + 1]) for i in range(n)]
    per_tile_out = [w.clone() for w in work]
    log(f"batched: per-tile calls {np.median(per_tile_s) * 1e3:.1f} ms")

    restore()
    t1 = time.time()
    tune = mrecon.autotune(items, 8, stream=stream)
    tuned = {"sweep_rounds": tune.sweep_rounds, "max_sweeps": tune.max_sweeps,
             "tail_rounds": tune.tail_rounds, "first_sweeps": tune.first_sweeps}
    log(f"batched: autotune {tuned} in {time.time() - t1:.1f}s")
    wsb = mrecon.alloc_workspace(mrecon.batch_workspace_bytes(items, 8, tune), dev)
    graph = (mrecon.BatchGraph(items, 8, tune, wsb)
             if tune.sweep_rounds > 0 or tune.tail_rounds > 0 else None)
    batched_s = []
    for rep in range(warm + reps):
        restore()
        t1 = time.perf_counter()
        if graph is not None:
            graph.launch(stream)
        else:
            mrecon.batch(items, 8, tune, wsb, stream)
        torch.cuda.synchronize()
        if rep >= warm:
            batched_s.append(time.perf_counter() - t1)
    log(f"batched: one launch sequence {np.median(batched_s) * 1e3:.1f} ms")

    same = all(bool(torch.equal(a, b)) for a, b in zip(work, per_tile_out))
    exact = True
    cpu_all = None
    if not args.no_verify:
        outs = [w.cpu().numpy() for w in work]
        threads = min(16, os.cpu_count() or 1)
        t1 = time.perf_counter()
        with ThreadPoolExecutor(threads) as ex:
            wants = list(ex.map(lambda i: oracle.recon_dilate(tiles[i][0], tiles[i][1], 8)[0],
                                range(n)))
        t_or = time.perf_counter() - t1
        exact = all(bool(np.array_equal(outs[i], wants[i])) for i in range(n))
        cpu_all = {"value": round(npx / t_or / 1e6, 1), "unit": "Mpixel/s", "cores": threads,
                   "kind": "oracle", "sample": f"all {n} tiles, one tile per thread at a time, "
                                              f"{t_or:.1f} s on {cpu_model()}"}
        log("batched: bit-exact vs oracle:", exact)
    if graph is not None:
        graph.close()
    med_pt, med_b = float(np.median(per_tile_s)), float(np.median(batched_s))
    return {
        "workload": f"{n} u8 tiles, sides log-uniform 256-4096, recon conn8, "
                    f"{npx / 1e9:.3f} Gpx",
        "per_tile": {"mpx_s": round(npx / med_pt / 1e6, 1), "ms_p50": round(med_pt * 1e3, 2),
                     "ms_p99": round(pct(per_tile_s, 99) * 1e3, 2),
                     "tile_latency_ms_p50": round(pct(lat_ms, 50), 4),
                     "tile_latency_ms_p99": round(pct(lat_ms, 99), 4)},
        "batched": {"mpx_s": round(npx / med_b / 1e6, 1), "ms_p50": round(med_b * 1e3, 2),
                    "ms_p99": round(pct(batched_s, 99) * 1e3, 2),
                    "mode": "hip graph" if graph is not None else "direct launches",
                    "tune": tuned},
        "speedup": round(med_pt / med_b, 3),
        "reps": reps,
        "bit_exact": bool(exact and same) if not args.no_verify else None,
        "batched_equals_per_tile": same,
        "cpu_baseline_all_cores": cpu_all,
    }


def leg_erode(args, dev) -> dict:
    """Reconstruction by erosion on the headline's image size: complement
    pass, reconstruction by dilation, complement back, on fresh marker copies
    resident in HBM."""
    import torch
    from paper_1311_0378_amd import mrecon, synth

    S, conn = 16384, 8
    t0 = time.time()
    marker, mask = synth.make_erode_tile(S, S, 12800, 0, "u8", 0.0)
    log(f"erode: generated {S}x{S} u8 in {time.time() - t0:.1f}s")
    d_mask = torch.from_numpy(mask).to(dev)
    d_src = torch.from_numpy(marker).to(dev)
    K, W = args.steps, args.warmup
    wsb = mrecon.erode_workspace_bytes(S, S, S, torch.uint8, conn)
    copies = [torch.empty_like(d_src) for _ in range(K)]
    ws = mrecon.alloc_workspace(wsb, dev)
    stream = torch.cuda.current_stream()
    tune = None
    if args.erode_tune:
        tune = {k: int(v) for k, v in (kv.split("=") for kv in args.erode_tune.split(","))}
    for i in range(W):
        copies[0].copy_(d_src)
        mrecon.recon_erode(copies[0], d_mask, conn, tune=tune, workspace=ws, stream=stream)
    for c in copies:
        c.copy_(d_src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mrecon.timing_enable("spans")  # as in the headline's timed steps
    a.record(stream)
    for i in range(K):
        mrecon.recon_erode(copies[i], d_mask, conn, tune=tune, workspace=ws, stream=stream)
    b.record(stream)
    b.synchronize()
    mrecon.timing_enable(False)
    recs = mrecon.timing_collect()
    ms = a.elapsed_time(b) / K
    cnt = mrecon.read_counters(ws)
    # the tile rounds of the last call: its records follow the last round-1 record
    first = max(i for i, r in enumerate(recs) if r[0] == "tile_round" and r[1] == 1)
    tr = [r for r in recs[first:] if r[0] == "tile_round"]
    tile_ms = sum(r[2] for r in tr)
    rt = mrecon.read_round_tiles(ws)
    visits = sum(rt[:-1])
    n_tiles = ((S + 61) // 62) ** 2
    achieved = visits * 3 * S * S / n_tiles / (tile_ms * 1e-3) / 1e9
    out = {"workload": f"recon_erode {S}x{S} u8 conn{conn}, 12800 disks, seed 0, "
                       "marker = min(mask + 30, 255)",
           "mpx_s": round(S * S / ms / 1e3, 1), "ms_per_call": round(ms, 4),
           "complement_bytes_per_call": 6 * S * S, "tune": tune or "library default",
           "counters_last_call": {k: cnt[k] for k in ("rounds", "tiles", "pops", "sweeps")},
           "roofline_tile_round_last_call": {
               "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
               "launches": sum(r[3] for r in tr), "tile_round_ms": round(tile_ms, 4),
               "timing": "spans"}}
    log(f"erode: {ms:.3f} ms per call")
    if not args.no_verify:
        import oracle
        t = time.perf_counter()
        want, _ = oracle.recon_erode(marker, mask, conn)
        secs = time.perf_counter() - t
        out["cpu_oracle"] = {"s": round(secs, 3), "mpx_s": round(marker.size / secs / 1e6, 2),
                             "cores": 1, "kind": "oracle"}
        out["bit_exact"] = bool(np.array_equal(copies[K - 1].cpu().numpy(), want))
        log("erode: bit-exact vs oracle:", out["bit_exact"])
    del copies, ws, d_mask, d_src
    return out


def leg_served(args, dev) -> dict:
    """Serving trace: sequential per-job launches versus the server, with the
    jobs in host memory (PCIe in and out) and with the jobs already in HBM
    (device-to-device copies into and out of the arena)."""
    import torch
    import xxhash
    import oracle
    from paper_1311_0378_amd import mrecon, synth

    n = args.serve_n
    jobs = synth.serving_jobs(n)
    wins = synth.serving_windows(jobs)
    t0 = time.time()
    bm, bk, bf = synth.serving_banks()
    side = bm.shape[1]
    npx = sum(H * W for _, H, W in jobs)
    log(f"served: {n} jobs, {npx / 1e9:.2f} Gpx, banks ready in {time.time() - t0:.1f}s")

    # every job's oracle result, hashed, on the host's cores after the GPU
    # passes (run beside them it would hold the interpreter lock in its array
    # copies and delay the serving loop)
    def oracle_hash(i):
        kind, H, W = jobs[i]
        y, x = wins[i]
        if kind == "recon":
            want = oracle.recon_dilate(np.ascontiguousarray(bm[y:y + H, x:x + W]),
                                       np.ascontiguousarray(bk[y:y + H, x:x + W]), 8)[0]
        else:
            want = oracle.fill_holes(np.ascontiguousarray(bf[y:y + H, x:x + W]), 8)[0]
        return xxhash.xxh3_64_intdigest(want)

    u8 = torch.uint8
    stream = torch.cuda.current_stream()
    hip = ctypes.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    hip.hipMemcpy2DAsync.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                     ctypes.c_size_t, ctypes.c_size_t, ctypes.c_size_t,
                                     ctypes.c_int, ctypes.c_void_p]
    H2D, D2H, D2D = 1, 2, 3
    max_jobs = args.serve_slots
    arena = 8 << 30

    def copy2d(dst, dpitch, src, spitch, H, W, kind):
        rc = hip.hipMemcpy2DAsync(dst, dpitch, src, spitch, W, H, kind, stream.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"hipMemcpy2DAsync failed ({rc})")

    def res_view(buf, i):
        _, H, W = jobs[i]
        ld = (W + 63) // 64 * 64
        return buf[:H * ld].view(H, ld)[:, :W]

    d0 = torch.empty((side, side), dtype=u8, device=dev)
    d1 = torch.empty((side, side), dtype=u8, device=dev)
    ws = mrecon.alloc_workspace(max(mrecon.workspace_bytes(op, side, side, u8, 8)
                                    for op in (mrecon.MR_OP_RECON, mrecon.MR_OP_FILL)), dev)

    def wait_until(t):
        while True:
            d = t - time.perf_counter()
            if d <= 0:
                return
            time.sleep(min(d, 2e-4))

    def run_mode(where):
        on_dev = where == "device"
        if on_dev:
            banks = [torch.from_numpy(x).to(dev) for x in (bm, bk, bf)]
        else:
            banks = [torch.from_numpy(x).pin_memory() for x in (bm, bk, bf)]
        pm, pk, pf = banks
        cin, cout = (D2D, D2D) if on_dev else (H2D, D2H)

        def views(i):
            kind, H, W = jobs[i]
            y, x = wins[i]
            if kind == "recon":
                return pm[y:y + H, x:x + W], pk[y:y + H, x:x + W]
            return pf[y:y + H, x:x + W], None

        # result buffers: H rows of W, 64-byte aligned row pitch, in blocks
        # of host pinned memory or of HBM
        pool = queue.SimpleQueue()
        for _ in range(max_jobs + 16):
            pool.put(torch.empty(side * side, dtype=u8, device=dev) if on_dev
                     else torch.empty(side * side, dtype=u8, pin_memory=True))

        def digest(i, buf, hashes):
            r = res_view(buf, i)
            r = r.cpu() if on_dev else r
            hashes[i] = xxhash.xxh3_64_intdigest(np.ascontiguousarray(r.numpy()))
            pool.put(buf)

        def recycle(i, buf, hashes):
            pool.put(buf)

        def run_sequential(arr, hashing=False):
            hasher = ThreadPoolExecutor(4)
            consume = digest if hashing else recycle
            hashes, lat, futs = [None] * n, [0.0] * n, []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(n):
                if arr is not None:
                    wait_until(t0 + arr[i])
                kind, H, W = jobs[i]
                a, m = views(i)
                buf = pool.get()
                copy2d(d0.data_ptr(), side, a.data_ptr(), side, H, W, cin)
                if m is not None:
                    copy2d(d1.data_ptr(), side, m.data_ptr(), side, H, W, cin)
                    mrecon.recon_dilate(d0[:H, :W], d1[:H, :W], 8, workspace=ws, stream=stream)
                else:
                    mrecon.fill_holes(d0[:H, :W], 8, workspace=ws, stream=stream)
                copy2d(buf.data_ptr(), (W + 63) // 64 * 64, d0.data_ptr(), side, H, W, cout)
                stream.synchronize()
                lat[i] = time.perf_counter() - t0 - (arr[i] if arr is not None else 0.0)
                futs.append(hasher.submit(consume, i, buf, hashes))
            span = time.perf_counter() - t0 - (arr[0] if arr is not None else 0.0)
            hasher.shutdown()
            for f in futs:
                f.result()
            return hashes, lat, span

        def run_served(arr, hashing=False):
            hasher = ThreadPoolExecutor(4)
            consume = digest if hashing else recycle
            srv = mrecon.Server(arena, max_jobs=max_jobs, dtype=u8, conn=8, device=dev,
                                stream=stream, rounds_per_step=args.serve_rounds)
            hashes, lat, futs = [None] * n, [0.0] * n, []
            owned = {}
            i = done = 0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            while done < n:
                now = time.perf_counter() - t0
                while i < n and (arr is None or arr[i] <= now):
                    try:
                        buf = pool.get_nowait()
                    except queue.Empty:
                        break
                    a, m = views(i)
                    jid = srv.submit(a, m, out=res_view(buf, i))
                    if jid is None:
                        pool.put(buf)
                        break
                    owned[jid] = (i, buf)
                    i += 1
                if srv.stats()["resident"]:
                    srv.step()
                elif i < n and arr is not None:
                    wait_until(t0 + arr[i])
                for jid, _ in srv.poll():
                    k, buf = owned.pop(jid)
                    lat[k] = time.perf_counter() - t0 - (arr[k] if arr is not None else 0.0)
                    futs.append(hasher.submit(consume, k, buf, hashes))
                    done += 1
            span = time.perf_counter() - t0 - (arr[0] if arr is not None else 0.0)
            rounds = srv.stats()["rounds"]
            srv.close()
            hasher.shutdown()
            for f in futs:
                f.result()
            return hashes, lat, span, rounds

        def summary(lat, span):
            return {"mpx_s": round(npx / span / 1e6, 1),
                    "latency_ms_p50": round(pct(lat, 50) * 1e3, 2),
                    "latency_ms_p99": round(pct(lat, 99) * 1e3, 2), "span_s": round(span, 3)}

        # timed passes: results land in their buffers, which are reused
        _, lat_sb, span_sb = run_sequential(None)
        log(f"served ({where}): sequential back to back {span_sb:.2f}s")
        _, lat_vb, span_vb, rounds_vb = run_served(None)
        log(f"served ({where}): server back to back {span_vb:.2f}s, {rounds_vb} rounds")
        rate = args.serve_load * n / span_sb
        arr = synth.poisson_arrivals(n, rate)
        _, lat_st, span_st = run_sequential(arr)
        log(f"served ({where}): sequential on the trace {span_st:.2f}s")
        _, lat_vt, span_vt, rounds_vt = run_served(arr)
        log(f"served ({where}): server on the trace {span_vt:.2f}s")
        # untimed verification passes: every result hashed, job by job
        ref, _, _ = run_sequential(None, hashing=True)
        h_vb, _, _, _ = run_served(None, hashing=True)
        h_vt, _, _, _ = run_served(arr, hashing=True)
        agree = ref == h_vb == h_vt and None not in ref
        del banks, pm, pk, pf
        return ref, {
            "jobs_in": "HBM (device-to-device copies into and out of the arena)" if on_dev
                       else "pinned host memory (PCIe in and out)",
            "back_to_back": {"sequential": summary(lat_sb, span_sb),
                             "served": summary(lat_vb, span_vb), "served_rounds": rounds_vb},
            "trace": {"rate_jobs_s": round(rate, 2),
                      "load_vs_sequential_capacity": args.serve_load,
                      "sequential": summary(lat_st, span_st), "served": summary(lat_vt, span_vt),
                      "served_rounds": rounds_vt},
            "results_agree": bool(agree),
        }

    ref_host, host = run_mode("host")
    torch.cuda.empty_cache()
    ref_dev, device = run_mode("device")
    t1 = time.time()
    threads = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(threads) as ex:
        want = list(ex.map(oracle_hash, range(n)))
    t_or = time.time() - t1
    log(f"served: oracle over all {n} jobs in {t_or:.1f}s")
    host["oracle_bit_exact"] = ref_host == want
    device["oracle_bit_exact"] = ref_dev == want
    log("served: host jobs agree:", host["results_agree"], "oracle:", host["oracle_bit_exact"],
        "| device jobs agree:", device["results_agree"], "oracle:", device["oracle_bit_exact"])
    return {
        "workload": f"{n} jobs, sides log-uniform 512-8192, 70% recon / 30% fill-holes, u8 "
                    f"conn8, {npx / 1e9:.2f} Gpx",
        "arena_gib": arena >> 30, "max_jobs": max_jobs,
        "rounds_per_step": args.serve_rounds or "library default",
        "host_jobs": host,
        "device_jobs": device,
        "oracle_checked_jobs": n,
        "cpu_baseline_all_cores": {
            "value": round(npx / t_or / 1e6, 1), "unit": "Mpixel/s", "cores": threads,
            "kind": "oracle", "sample": f"all {n} jobs, one job per thread at a time (window "
                                       f"copies and hashing included), {t_or:.1f} s on "
                                       f"{cpu_model()}"},
    }


def leg_ops(args, dev, mask) -> dict:
    """The other Table II operations on the headline's 16384^2 workload:
    RGB2Gray on a colour image made from the mask, opening by the 13 x 13
    disk on the mask, the distance transform, CCL and area threshold on the
    binary image (mask >= 128), h-dome (h = 20) and regional maxima on the
    mask. Each is timed with events around K calls on inputs resident in HBM
    and checked against the oracle (the opening on sampled windows, the others
    on the whole image)."""
    import torch
    import oracle
    from paper_1311_0378_amd import ops, synth

    S = mask.shape[0]
    npx = S * mask.shape[1]
    K = max(1, min(args.steps, 5))
    stream = torch.cuda.current_stream()
    out = {"workload": f"{S}x{S}, from the headline's mask (12800 disks, seed 0)", "calls": K}
    t0 = time.time()
    binary = synth.binary_from_mask(mask)
    rgb = synth.rgb_from_mask(mask)
    log(f"ops: inputs in {time.time() - t0:.1f}s")
    d_mask = torch.from_numpy(mask).to(dev)
    d_bin = torch.from_numpy(binary).to(dev)

    def timed(fn, prep=None):
        """ms per call over K calls (prep runs before each, outside the
        timing of that call), and the last call's output."""
        res, total = None, 0.0
        fn() if prep is None else (prep(), fn())  # warm-up
        for _ in range(K):
            if prep is not None:
                prep()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            res = fn()
            b.record(stream)
            b.synchronize()
            total += a.elapsed_time(b)
        return total / K, res

    def line(ms, alg_bytes, exact, **kw):
        gbs = alg_bytes / (ms * 1e-3) / 1e9
        d = {"ms": round(ms, 4), "mpx_s": round(npx / ms / 1e3, 1),
             "algorithmic_gb": round(alg_bytes / 1e9, 4),
             "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)},
             "bit_exact": exact}
        d.update(kw)
        return d

    verify = not args.no_verify

    def cpu(fn, px=npx):
        """Run one oracle computation on one host core: its result and the
        oracle's rate beside the GPU's (the oracle as it stands, untuned)."""
        t = time.perf_counter()
        r = fn()
        s = time.perf_counter() - t
        return r, {"s": round(s, 3), "mpx_s": round(px / s / 1e6, 2), "cores": 1,
                   "kind": "oracle"}

    # RGB2Gray: 3 bytes in, 1 out per pixel
    d_rgb = torch.from_numpy(rgb).to(dev)
    gray = torch.empty((S, S), dtype=torch.uint8, device=dev)
    ms, _ = timed(lambda: ops.rgb2gray(d_rgb, out=gray))
    ok, c = None, None
    if verify:
        want, c = cpu(lambda: oracle.rgb2gray(rgb))
        ok = bool(np.array_equal(gray.cpu().numpy(), want))
    out["rgb2gray"] = line(ms, 4 * npx, ok, cpu_oracle=c)
    log(f"ops: rgb2gray {ms:.3f} ms, exact {ok}")
    del d_rgb, gray

    # opening: erosion and dilation, each 1 byte in and 1 out per pixel
    o = torch.empty_like(d_mask)
    wso = torch.empty(S * S, dtype=torch.uint8, device=dev)
    ms, _ = timed(lambda: ops.open_disk13(d_mask, out=o, workspace=wso))
    ok, c = None, None
    if verify:
        rng = np.random.default_rng(11)
        got = o.cpu().numpy()
        ok, secs, px = True, 0.0, 0
        for _ in range(48):
            y, x = (int(v) for v in rng.integers(0, S - 256, 2))
            y0, x0 = max(0, y - 12), max(0, x - 12)
            y1, x1 = min(S, y + 256 + 12), min(S, x + 256 + 12)
            want, cw = cpu(lambda: oracle.open_disk13(mask[y0:y1, x0:x1]), (y1 - y0) * (x1 - x0))
            secs += cw["s"]
            px += (y1 - y0) * (x1 - x0)
            ok &= bool(np.array_equal(got[y:y + 256, x:x + 256],
                                      want[y - y0:y - y0 + 256, x - x0:x - x0 + 256]))
        c = {"s": round(secs, 3), "mpx_s": round(px / max(secs, 1e-9) / 1e6, 2), "cores": 1,
             "kind": "oracle", "sample": "the 48 checked windows with their margins"}
    out["open_disk13"] = line(ms, 4 * npx, ok, cpu_oracle=c,
                              check="48 windows of 256x256 (12-pixel margin)",
                              note="two passes (erosion, dilation); bound by instruction "
                                   "issue rather than HBM")
    log(f"ops: open {ms:.3f} ms, exact {ok}")
    del o, wso

    # distance transform: 1 byte in, 4 out per pixel (round 1; later rounds
    # revisit a few tiles)
    dist = torch.empty((S, S), dtype=torch.int32, device=dev)
    wsd = torch.empty(ops.lib().mr_distance_transform_workspace_bytes(S, S, 8),
                      dtype=torch.uint8, device=dev)
    ms, _ = timed(lambda: ops.distance_transform(d_bin, 8, out=dist, workspace=wsd))
    ok, c = None, None
    if verify:
        want, c = cpu(lambda: oracle.distance_transform(binary, 8))
        ok = bool(np.array_equal(dist.cpu().numpy(), want))
    out["distance_transform"] = line(ms, 5 * npx, ok, conn=8, cpu_oracle=c)
    log(f"ops: distance transform {ms:.3f} ms, exact {ok}")
    del dist, wsd

    # CCL: 1 byte in, 4-byte labels out; then area threshold on the labels
    # (4 bytes read and 4 written per pixel)
    lab = torch.empty((S, S), dtype=torch.int32, device=dev)
    wsc = torch.empty(ops.lib().mr_ccl_workspace_bytes(S, S), dtype=torch.uint8, device=dev)
    ms, _ = timed(lambda: ops.ccl(d_bin, 8, out=lab, workspace=wsc))
    ok, c, want_lab = None, None, None
    if verify:
        want_lab, c = cpu(lambda: oracle.ccl(binary, 8))
        ok = bool(np.array_equal(lab.cpu().numpy(), want_lab))
    out["ccl"] = line(ms, 5 * npx, ok, conn=8, cpu_oracle=c)
    log(f"ops: ccl {ms:.3f} ms, exact {ok}")
    del wsc
    lab2 = torch.empty_like(lab)
    wsa = torch.empty(ops.lib().mr_area_threshold_workspace_bytes(S, S), dtype=torch.uint8,
                      device=dev)
    lo, hi = 150, 500
    ms, _ = timed(lambda: ops.area_threshold(lab2, lo, hi, workspace=wsa),
                  prep=lambda: lab2.copy_(lab))
    ok, c = None, None
    if verify:
        want, c = cpu(lambda: oracle.area_threshold(want_lab, lo, hi)[0])
        ok = bool(np.array_equal(lab2.cpu().numpy(), want))
    out["area_threshold"] = line(ms, 8 * npx, ok, range=[lo, hi], cpu_oracle=c)
    log(f"ops: area threshold {ms:.3f} ms, exact {ok}")
    del lab, lab2, wsa

    # h-dome and regional maxima: a reconstruction each, plus two streaming
    # passes (the minimum is the reconstruction's 3 bytes per pixel)
    h = 20
    hd = torch.empty_like(d_mask)
    wsh = torch.empty(ops.hdome_workspace_bytes(S, S, S, torch.uint8, 8), dtype=torch.uint8,
                      device=dev)
    ms, _ = timed(lambda: ops.hdome(hd, h, 8, workspace=wsh), prep=lambda: hd.copy_(d_mask))
    ok, c = None, None
    if verify:
        want, c = cpu(lambda: oracle.hdome(mask, h, 8))
        ok = bool(np.array_equal(hd.cpu().numpy(), want))
    out["hdome"] = line(ms, 3 * npx, ok, h=h, cpu_oracle=c)
    log(f"ops: h-dome {ms:.3f} ms, exact {ok}")
    rm = torch.empty_like(d_mask)
    ms, _ = timed(lambda: ops.regional_maxima(d_mask, 8, out=rm, workspace=wsh))
    ok, c = None, None
    if verify:
        want, c = cpu(lambda: oracle.regional_maxima(mask, 8))
        ok = bool(np.array_equal(rm.cpu().numpy(), want))
    out["regional_maxima"] = line(ms, 3 * npx, ok, cpu_oracle=c)
    log(f"ops: regional maxima {ms:.3f} ms, exact {ok}")
    del hd, rm, wsh, d_mask, d_bin
    return out


def queue_planes(args, torch, mrecon, dev, reps: int = 3) -> dict:
    """The queue phase on uint8 pixels with the dword compare-and-swap
    (workspace sized by the default tune) against the widened 32-bit plane
    (workspace sized by the queue tune): whole mr_recon_dilate calls after
    1, 2 and 4 tile rounds, min of `reps` after a warm-up, each result
    compared with the oracle."""
    import oracle
    from paper_1311_0378_amd import synth
    S = args.size
    marker, mask = synth.make_tile(S, S, 12800 if S == 16384 else synth.density_disks(S, S), 0,
                                   "u8", 0.0)
    want = torch.from_numpy(oracle.recon_dilate(marker, mask, args.conn)[0]).to(dev)
    d_mask = torch.from_numpy(mask).to(dev)
    d_src = torch.from_numpy(marker).to(dev)
    out = {"workload": f"recon_dilate {S}x{S} u8 conn{args.conn}, 12800 disks, seed 0",
           "cases": []}
    for rounds in (1, 2, 4):
        tune = {"sweep_rounds": rounds}
        nb_cas = mrecon.workspace_bytes(mrecon.MR_OP_RECON, S, S, torch.uint8, args.conn, None)
        for label, sized in (("dword CAS", None), ("widened plane", tune)):
            nb = mrecon.workspace_bytes(mrecon.MR_OP_RECON, S, S, torch.uint8, args.conn, sized)
            ws = mrecon.alloc_workspace(nb, dev)
            w = d_src.clone()
            mrecon.recon_dilate(w, d_mask, args.conn, tune=tune, workspace=ws)
            times = []
            for _ in range(reps):
                w.copy_(d_src)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                mrecon.recon_dilate(w, d_mask, args.conn, tune=tune, workspace=ws)
                torch.cuda.synchronize()
                times.append((time.perf_counter() - t0) * 1e3)
            c = mrecon.read_counters(ws)
            out["cases"].append({"rounds_before_queue": rounds, "raise": label,
                                 "ms_per_call": round(min(times), 3),
                                 "workspace_mb": round(nb / 1e6, 1), "pops": c["pops"],
                                 "pushes": c["pushes"], "cas_retries": c["cas_retries"],
                                 # (the library sizes widened planes only for
                                 # schedules of one or two rounds)
                                 "widened_plane_in_workspace": nb > nb_cas,
                                 "bit_exact": bool(torch.equal(w, want))})
            log(f"queue planes: {out['cases'][-1]}")
            del ws, w
    return out


def atomic_probe(torch, mrecon, dev, reps: int = 5) -> dict:
    """Relaxed device-scope atomics on pseudo-random words, every wave slot of
    the GPU busy: the ceiling the queue phase's atomics are measured against."""
    waves = 16384  # 256 CUs x 32 wave slots, twice over
    cases = []
    for log2_words in (26, 30):  # 256 MiB (the 16384^2 u8 image's size), 4 GiB
        words = torch.zeros(1 << log2_words, dtype=torch.int32, device=dev)
        for kind, name, per_lane in ((mrecon.MR_PROBE_ADD, "add", 256),
                                     (mrecon.MR_PROBE_CAS, "load+cas", 64)):
            ops = waves * 64 * per_lane
            mrecon.probe_atomics(words, kind, per_lane, waves, seed=1)  # warm-up
            times = []
            for r in range(reps):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                mrecon.probe_atomics(words, kind, per_lane, waves, seed=2 + r)
                b.record()
                b.synchronize()
                times.append(a.elapsed_time(b))
            ms = sorted(times)[len(times) // 2]
            cases.append({"kind": name, "buffer_mib": (4 << log2_words) >> 20, "waves": waves,
                          "per_lane": per_lane, "ops": ops, "ms_median": round(ms, 4),
                          "g_ops_s": round(ops / ms / 1e6, 2)})
            log(f"probe {name} {(4 << log2_words) >> 20} MiB: {ms:.3f} ms, "
                f"{ops / ms / 1e6:.1f} G ops/s")
        total = int(words.to(torch.int64).sum())
        expect = (reps + 1) * waves * 64 * (256 + 64)
        if total != expect:
            raise RuntimeError(f"probe lost operations: {total} != {expect}")
        del words
    return {"probe": "device atomics, relaxed, device scope, pseudo-random words",
            "cases": cases}


def random_probe(torch, mrecon, dev, reps: int = 5) -> dict:
    """Plain random reads and writes of 32-bit words at host-drawn positions
    (the index vector streams in order; only the matrix accesses scatter).
    For each case the best launch shape of a small sweep is kept."""
    import numpy as np
    cases = []
    rng = np.random.default_rng(1311)
    for log2_words in (24, 30):  # 4K x 4K int32 (64 MiB), 4 GiB
        words = torch.zeros(1 << log2_words, dtype=torch.int32, device=dev)
        words.copy_(torch.arange(1 << log2_words, dtype=torch.int32, device=dev) * -1640531535)
        mask = (1 << log2_words) - 1
        for n_ops in (10_000_000, 1 << 28):
            idx_np = rng.integers(0, 1 << log2_words, n_ops, dtype=np.uint32)
            idx = torch.from_numpy(idx_np.view(np.int32)).to(dev)
            del idx_np
            for kind, name in ((mrecon.MR_RANDOM_READ, "read"), (mrecon.MR_RANDOM_WRITE, "write")):
                best = None
                for waves in (2048, 8192, 32768):
                    sums = torch.empty(waves * 64, dtype=torch.int32, device=dev)
                    mrecon.probe_random(words, idx, kind, waves, sums)  # warm-up
                    times = []
                    for _ in range(reps):
                        a = torch.cuda.Event(enable_timing=True)
                        b = torch.cuda.Event(enable_timing=True)
                        a.record()
                        mrecon.probe_random(words, idx, kind, waves, sums)
                        b.record()
                        b.synchronize()
                        times.append(a.elapsed_time(b))
                    ms = sorted(times)[len(times) // 2]
                    if kind == mrecon.MR_RANDOM_READ:
                        # the kernel's sums against torch's own gather (mod 2^32)
                        got = int(sums.to(torch.int64).sum()) & 0xFFFFFFFF
                        ref = int(words[idx.to(torch.int64) & mask].to(torch.int64).sum()) \
                            & 0xFFFFFFFF
                        if got != ref:
                            raise RuntimeError(f"random read probe: sums {got} != {ref}")
                    if best is None or ms < best[0]:
                        best = (ms, waves)
                    del sums
                ms, waves = best
                cases.append({"kind": name, "matrix_mib": (4 << log2_words) >> 20, "ops": n_ops,
                              "waves": waves, "ms_median": round(ms, 4),
                              "g_ops_s": round(n_ops / ms / 1e6, 2),
                              "mb_s": round(4 * n_ops / ms / 1e3, 0)})
                log(f"random {name} {(4 << log2_words) >> 20} MiB, {n_ops} ops, {waves} waves: "
                    f"{ms:.3f} ms, {n_ops / ms / 1e6:.2f} G ops/s, {4 * n_ops / ms / 1e3:.0f} MB/s")
            del idx
        del words
    return {"probe": "plain random reads and writes of 32-bit words at host-drawn positions",
            "unit_mb_s": "MB/s of 4-byte words (10^6 B/s)", "cases": cases,
            "paper_table3_gpu_mb_s": {"read": 895, "write": 126}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=16384)
    ap.add_argument("--dtype", default="u8", choices=["u8", "i32"])
    ap.add_argument("--conn", type=int, default=8, choices=[4, 8])
    ap.add_argument("--tune", default="", help="k=v,... overrides of mr_tune")
    ap.add_argument("--legs", default="i32,small,batched,served,erode,ops",
                    help="extra legs after the headline: comma list of i32, small, batched, "
                         "served, erode, ops, or none")
    ap.add_argument("--erode-tune", default="sweep_rounds=-1,tail_rounds=0",
                    help="k=v,... mr_tune overrides for the erode leg (default: tile rounds until "
                         "none is dirty, the fastest schedule measured for that workload)")
    ap.add_argument("--batch-n", type=int, default=512)
    ap.add_argument("--batch-reps", type=int, default=5)
    ap.add_argument("--serve-n", type=int, default=2000)
    ap.add_argument("--serve-load", type=float, default=0.8)
    ap.add_argument("--serve-slots", type=int, default=128,
                    help="server job slots (jobs resident at once)")
    ap.add_argument("--serve-rounds", type=int, default=None,
                    help="tile rounds per server step (library default when omitted)")
    ap.add_argument("--timing", default="spans", choices=["spans", "launches"],
                    help="launch timing inside the timed steps (see mr_timing_enable)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-verify", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device pass first (counter calibration)")
    ap.add_argument("--atomic-probe", action="store_true",
                    help="time the device atomic-rate probe (mr_probe_atomics) on a 256 MiB and "
                         "a 4 GiB buffer, print one JSON line and exit")
    ap.add_argument("--random-probe", action="store_true",
                    help="time the random-access probe (mr_probe_random) on a 64 MiB and a 4 GiB "
                         "matrix, print one JSON line and exit")
    ap.add_argument("--queue-planes", action="store_true",
                    help="time the queue phase with the dword compare-and-swap and with the "
                         "widened plane (uint8, 1/2/4 rounds first), print one JSON line and exit")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 --pmc counter CSVs (FETCH_SIZE, WRITE_SIZE) of a "
                         "--calibrate-copy run into "
                         "profiles/tile_round_traffic_<size>_<dtype>_conn<conn>.json and exit")
    ap.add_argument("--served-trace", metavar="TRACE_DIR",
                    help="summarise a rocprofv3 --kernel-trace --memory-copy-trace run of the "
                         "served leg (busy time per server pass), print one JSON line and exit")
    args = ap.parse_args()

    if args.served_trace:
        summarize_served_trace(args.served_trace)
        return
    if args.traffic_from:
        summarize_traffic(*args.traffic_from, args)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1311_0378_amd import build as libbuild
    from paper_1311_0378_amd import mrecon, synth

    if not os.path.exists(libbuild.LIB):
        libbuild.build()
    dev = torch.device("cuda:0")
    if args.atomic_probe:
        print(json.dumps(atomic_probe(torch, mrecon, dev)), flush=True)
        return
    if args.random_probe:
        print(json.dumps(random_probe(torch, mrecon, dev)), flush=True)
        return
    if args.queue_planes:
        print(json.dumps(queue_planes(args, torch, mrecon, dev)), flush=True)
        return
    S, dt, conn = args.size, args.dtype, args.conn
    tune = None
    if args.tune:
        tune = {k: int(v) for k, v in (kv.split("=") for kv in args.tune.split(","))}

    t0 = time.time()
    n_disks = 12800 if S == 16384 else synth.density_disks(S, S)
    marker, mask = synth.make_tile(S, S, n_disks, 0, dt, 0.0)
    log(f"generated {S}x{S} {dt} in {time.time() - t0:.1f}s")

    if args.calibrate_copy:
        # a 1 GiB elementwise pass (read 1 GiB, write 1 GiB) under a kernel
        # name nothing else in the run uses, so the counter summary can pick
        # it out
        a = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.bitwise_not(a, out=b)
        torch.cuda.synchronize()
        del a, b

    result = {
        "metric": "reconstructed Mpixel/s (bit-exact) + %HBM roofline; batched vs per-tile; p50/p99",
        "value": None,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dt,
        "data": "synthetic",
        "config": {"workload": f"recon_dilate {S}x{S} {dt} conn{conn}, {n_disks} disks, seed 0",
                   "image": f"{S}x{S}", "pixel": dt, "conn": conn},
    }
    head = measure_recon(args, torch, mrecon, dev, marker, mask, conn, tune)
    result["value"] = head.pop("mpx_s")
    result["ms_per_step"] = head.pop("ms_per_call")
    result.update(head)
    if not args.no_cpu_baseline:
        import oracle
        # the oracle as it stands, one thread, on the whole image: median of 3
        times = []
        for _ in range(3):
            t1 = time.perf_counter()
            oracle.recon_dilate(marker, mask, conn)
            times.append(time.perf_counter() - t1)
        t_or = float(np.median(times))
        result["cpu_baseline"] = {
            "value": round(S * S / t_or / 1e6, 2), "unit": "Mpixel/s", "cores": 1,
            "kind": "oracle",
            "sample": f"the whole {S}x{S} {dt} image, median of 3 sequential oracle runs "
                      f"({', '.join(f'{x:.2f}' for x in times)} s) on {cpu_model()}, "
                      f"{os.cpu_count()} threads visible"}
    result["copy_bandwidth"] = copy_bandwidth(torch, dev)
    legs = [x for x in args.legs.split(",") if x and x != "none"]
    unknown = set(legs) - {"i32", "small", "batched", "served", "erode", "ops"}
    if unknown:
        raise SystemExit(f"unknown legs: {sorted(unknown)}")
    torch.cuda.empty_cache()
    if "i32" in legs and dt == "u8":
        # the int32 variant of the same workload (values scaled to 0..65535)
        t0 = time.time()
        marker32, mask32 = synth.make_tile(S, S, n_disks, 0, "i32", 0.0)
        log(f"i32: generated in {time.time() - t0:.1f}s")
        leg = measure_recon(args, torch, mrecon, dev, marker32, mask32, conn, tune)
        leg["workload"] = f"recon_dilate {S}x{S} i32 conn{conn}, {n_disks} disks, seed 0, " \
                          "values scaled to 0..65535"
        result["i32"] = leg
        del marker32, mask32
        torch.cuda.empty_cache()
    if "small" in legs:
        result["small"] = leg_small(args, dev)
        torch.cuda.empty_cache()
    if "batched" in legs:
        result["batched"] = leg_batched(args, dev)
        torch.cuda.empty_cache()
    if "served" in legs:
        result["served"] = leg_served(args, dev)
        torch.cuda.empty_cache()
    if "erode" in legs:
        result["erode"] = leg_erode(args, dev)
        torch.cuda.empty_cache()
    if "ops" in legs:
        if dt == "u8":
            result["ops"] = leg_ops(args, dev, mask)
        else:
            u8_mask = synth.make_tile(S, S, n_disks, 0, "u8", 0.0)[1]
            result["ops"] = leg_ops(args, dev, u8_mask)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
