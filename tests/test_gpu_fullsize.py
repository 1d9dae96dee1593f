"""Parity at full workload sizes, in the launch configuration the benchmark
times (library defaults), and at the largest plane the interface accepts.

* 16384 x 16384 reconstruction, u8 and i32 (values scaled to 0..65535),
  8-connectivity: every pixel against the oracle; and the int32 copy of the
  u8 workload with every value times 257 against 257 times the u8 result.
* 65535 x 65535 u8 (H * pitch just below 2^32): the mask carries walls of
  zeros every 4096 rows and columns. Under 4- or 8-connectivity nothing can
  propagate through a zero-mask wall one pixel thick (the wall pixels stay at
  0, and pixels on either side are not neighbours), so every walled block is
  an independent reconstruction: all 256 blocks, the ragged last row and
  column of blocks included, are checked exactly against the oracle run on
  the block alone.
* The 512-tile batch at full size, autotuned and replayed as the benchmark
  times it, and all 2000 serving jobs through the server (from host memory
  and from device memory): every image against the oracle.
"""
import numpy as np
import pytest

import oracle
from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import DEV, first_mismatch, gpu_recon  # noqa: E402
from paper_1311_0378_amd import mrecon  # noqa: E402


@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_16384_full_image(dt):
    marker, mask = synth.single_16384(dt)
    print(f"[gpu] 16384x16384 {dt} conn8", flush=True)
    got = gpu_recon(marker, mask, 8)
    want, _ = oracle.recon_dilate(marker, mask, 8)
    assert np.array_equal(got, want), first_mismatch(got, want)


def test_16384_i32_copy_of_u8_is_257_times():
    # the int32 copy of the uint8 workload with every value times 257: the
    # order of values is the same, so R(257 M, 257 I) = 257 R(M, I) (both
    # runs on the GPU, then the uint8 one against the oracle as well)
    marker, mask = synth.single_16384("u8")
    print("[gpu] 16384x16384 u8 and its x257 int32 copy, conn8", flush=True)
    got8 = gpu_recon(marker, mask, 8)
    got32 = gpu_recon(marker.astype(np.int32) * 257, mask.astype(np.int32) * 257, 8)
    want = got8.astype(np.int32) * 257
    assert np.array_equal(got32, want), first_mismatch(got32, want)
    want8, _ = oracle.recon_dilate(marker, mask, 8)
    assert np.array_equal(got8, want8), first_mismatch(got8, want8)


def _walled_inputs(H, W, step, seed):
    g = torch.Generator(device=DEV)
    g.manual_seed(seed)
    noise = torch.randint(0, 256, (H, W), generator=g, device=DEV, dtype=torch.uint8)
    mask = torch.empty_like(noise)
    # spatially correlated values: 5 x 5 box mean in row bands (fp16 holds
    # every sum of 25 u8 values / 25 closely enough for test data)
    band = 4096
    for y0 in range(0, H, band):
        y1 = min(H, y0 + band)
        a, b = max(0, y0 - 2), min(H, y1 + 2)
        blk = noise[a:b].to(torch.float16)[None, None]
        m = torch.nn.functional.avg_pool2d(blk, 5, stride=1, padding=2, count_include_pad=False)
        mask[y0:y1] = m[0, 0, y0 - a:y0 - a + (y1 - y0)].round().clamp(0, 255).to(torch.uint8)
        del blk, m
    del noise
    mask[::step, :] = 0
    mask[:, ::step] = 0
    marker = (mask.to(torch.int16) - 30).clamp(min=0).to(torch.uint8)
    return marker, mask


@pytest.mark.parametrize("conn", [8])
def test_max_plane_walled_blocks(conn):
    from concurrent.futures import ThreadPoolExecutor
    H = W = 65535
    step = 4096
    print(f"[gpu] {H}x{W} u8 walled every {step}, conn{conn}", flush=True)
    marker, mask = _walled_inputs(H, W, step, seed=7)
    R = marker.clone()
    ws = mrecon.alloc_workspace(mrecon.workspace_bytes(mrecon.MR_OP_RECON, H, W, torch.uint8,
                                                       conn), R.device)
    mrecon.recon_dilate(R, mask, conn, workspace=ws)
    torch.cuda.synchronize()
    mrecon.status(ws)
    del ws
    # every walled block (16 x 16 of them; the last row and column of blocks
    # are 4095 pixels wide) exactly against the oracle run on the block
    # alone, walls included, on host threads. Every pixel of the plane lies
    # in at least one block.
    last = (H - 1) // step

    def block(b):
        by, bx = divmod(b, last + 1)
        y0, x0 = by * step, bx * step
        y1, x1 = min(H, y0 + step + 1), min(W, x0 + step + 1)
        mk = marker[y0:y1, x0:x1].cpu().numpy()
        ms = mask[y0:y1, x0:x1].cpu().numpy()
        got = R[y0:y1, x0:x1].cpu().numpy()
        want, _ = oracle.recon_dilate(mk, ms, conn)
        return None if np.array_equal(got, want) else f"block ({by},{bx}): " + first_mismatch(got, want)

    n_blocks = (last + 1) ** 2
    with ThreadPoolExecutor(16) as ex:
        bad = [r for r in ex.map(block, range(n_blocks)) if r]
    print(f"[gpu] {n_blocks} blocks checked, {len(bad)} differ", flush=True)
    assert not bad, bad[:4]


def _oracle_all(jobs, conn):
    """Oracle results of (marker-or-image, mask-or-None) jobs, on threads."""
    from concurrent.futures import ThreadPoolExecutor

    def one(job):
        a, m = job
        return (oracle.recon_dilate(a, m, conn) if m is not None else oracle.fill_holes(a, conn))[0]

    with ThreadPoolExecutor(16) as ex:
        return list(ex.map(one, jobs))


def test_batch_512_tiles_full():
    # the batched workload at its full size (sides log-uniform 256-4096,
    # about 1.0 Gpx), autotuned and replayed the way the benchmark times it
    from concurrent.futures import ThreadPoolExecutor
    n = 512
    shapes = synth.batch_shapes(n)
    with ThreadPoolExecutor(8) as ex:
        tiles = list(ex.map(lambda i: synth.batch_tile(i, *shapes[i], n=n), range(n)))
    print(f"[gpu] batch of {n} tiles, {sum(h * w for h, w in shapes) / 1e9:.2f} Gpx", flush=True)
    src = [torch.from_numpy(m).to(DEV) for m, _ in tiles]
    msk = [torch.from_numpy(k).to(DEV) for _, k in tiles]
    work = [x.clone() for x in src]
    items = [(w, k, mrecon.MR_OP_RECON) for w, k in zip(work, msk)]
    tune = mrecon.autotune(items, 8)
    ws = mrecon.alloc_workspace(mrecon.batch_workspace_bytes(items, 8, tune), DEV)
    if tune.sweep_rounds > 0 or tune.tail_rounds > 0:
        g = mrecon.BatchGraph(items, 8, tune, ws)
        g.launch()
        torch.cuda.synchronize()
        g.close()
    else:
        mrecon.batch(items, 8, tune, ws)
    want = _oracle_all(tiles, 8)
    for i in range(n):
        got = work[i].cpu().numpy()
        assert np.array_equal(got, want[i]), f"tile {i} {shapes[i]}: " + first_mismatch(got, want[i])


def _serving_inputs(jobs, wins):
    bm, bk, bf = synth.serving_banks()
    inputs = []
    for (kind, H, W), (y, x) in zip(jobs, wins):
        if kind == "recon":
            inputs.append((bm[y:y + H, x:x + W], bk[y:y + H, x:x + W]))
        else:
            inputs.append((bf[y:y + H, x:x + W], None))
    return inputs


def _oracle_one(job, conn=8):
    a, m = job
    a = np.ascontiguousarray(a)
    if m is None:
        return oracle.fill_holes(a, conn)[0]
    return oracle.recon_dilate(a, np.ascontiguousarray(m), conn)[0]


@pytest.mark.parametrize("device_jobs", [False, True], ids=["host_jobs", "device_jobs"])
def test_serving_jobs_full_sizes(device_jobs):
    # All 2000 jobs of the serving workload (windows of the two serving
    # images, sides 512-8192, recon and fill-holes mixed) through the server
    # with its default settings. Each result is checked against the oracle on
    # host threads as it arrives. Host jobs are windows of the images in
    # pinned memory, answered into pinned buffers; device jobs are windows of
    # the images held in HBM, answered into device buffers.
    import queue
    from concurrent.futures import ThreadPoolExecutor
    n = 2000
    jobs = synth.serving_jobs(n)
    wins = synth.serving_windows(jobs)
    inputs = _serving_inputs(jobs, wins)
    print(f"[gpu] server, all {n} serving jobs, device_jobs={device_jobs}", flush=True)
    banks = [torch.from_numpy(b) for b in synth.serving_banks()]
    banks = [b.to(DEV) for b in banks] if device_jobs else [b.pin_memory() for b in banks]
    bm, bk, bf = banks
    srcs = []
    for (kind, H, W), (y, x) in zip(jobs, wins):
        srcs.append((bm[y:y + H, x:x + W], bk[y:y + H, x:x + W]) if kind == "recon"
                    else (bf[y:y + H, x:x + W], None))
    # result buffers: a pool of pinned ones for host jobs, recycled after each
    # check; device jobs get a fresh device tensor per job
    side = max(H for _, H, _ in jobs), max(W for _, _, W in jobs)
    free = queue.Queue()
    if not device_jobs:
        for _ in range(64):
            free.put(torch.empty(side[0] * side[1], dtype=torch.uint8, pin_memory=True))
    srv = mrecon.Server(8 << 30, max_jobs=32)
    pool = ThreadPoolExecutor(16)
    checks = []

    def check_one(i, res, buf):
        want = _oracle_one(inputs[i])
        ok = np.array_equal(res, want)
        msg = None if ok else f"job {i} {jobs[i]}: " + first_mismatch(res, want)
        if buf is not None:
            free.put(buf)
        return msg

    pending, owned = list(range(n)), {}
    while pending or owned:
        while pending:
            i = pending[0]
            a, m = srcs[i]
            H, W = a.shape
            buf = None
            if device_jobs:
                out = None
            else:
                try:
                    buf = free.get_nowait()
                except queue.Empty:
                    break
                out = buf[:H * W].view(H, W)
            jid = srv.submit(a, m, out=out)
            if jid is None:
                if buf is not None:
                    free.put(buf)
                break
            owned[jid] = (pending.pop(0), buf)
        srv.step()
        for jid, res in srv.poll():
            i, buf = owned.pop(jid)
            r = res.cpu().numpy() if device_jobs else res.numpy()
            checks.append(pool.submit(check_one, i, r, buf))
    srv.close()
    bad = [r for r in (c.result() for c in checks) if r]
    pool.shutdown()
    assert len(checks) == n
    assert not bad, bad[:4]
