"""Schedule invariance under repetition.

The tile queue and the queue phase share pixels, bitmap rows, flags and ring
entries between waves on different compute units and dies without cache-wide
fences: their ordering rests on device-scope atomics and waited stores. A
rare ordering fault would show up as a pixel that differs from the unique
result on some runs only. These tests rerun the same inputs many times over a
spread of schedules (rounds before the switch, sweep caps, persistent grid
sizes, the tile queue, the converge mode), and every output must be
byte-identical to the oracle. A mismatch fails at once (with the run, tune and
first differing pixel); a wave that stops waiting for work raises the
watchdog status, which the status check turns into a failure, so a stall ends
the run instead of hanging it.

Also here: converge-mode calls alternated over two streams from one thread,
and a call on a side stream with a workspace the binding allocates.
"""
import numpy as np
import pytest

import oracle
from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import DEV, first_mismatch  # noqa: E402
from paper_1311_0378_amd import mrecon  # noqa: E402

# rounds before the queue phase / tile queue, sweep caps, grid sizes, first-round caps
STRESS_TUNES = [
    None,
    dict(sweep_rounds=1, max_sweeps=1),
    dict(sweep_rounds=1, max_sweeps=16, persistent_blocks=1),
    dict(sweep_rounds=2, max_sweeps=2, persistent_blocks=7),
    dict(sweep_rounds=3, max_sweeps=16, persistent_blocks=64),
    dict(sweep_rounds=8, max_sweeps=3),
    dict(sweep_rounds=-1, tail_rounds=1, max_sweeps=1),
    dict(sweep_rounds=-1, tail_rounds=1, max_sweeps=16),
    dict(sweep_rounds=-1, tail_rounds=2, max_sweeps=2),
    dict(sweep_rounds=-1, tail_rounds=8),
    dict(sweep_rounds=-1, tail_rounds=0),
    dict(sweep_rounds=-1, tail_rounds=0, converge_rounds=2),
    # first-round caps (the default is 1): full first visits, and two
    # iterations with the tile queue right after
    dict(sweep_rounds=-1, tail_rounds=8, first_sweeps=16),
    dict(sweep_rounds=-1, tail_rounds=2, first_sweeps=2, max_sweeps=3),
]


def _inputs(name):
    from test_oracle_pins import serpentine
    if name == "synth_u8":
        return synth.make_tile(1024, 1024, 200, 11, "u8", 0.05), "recon"
    if name == "synth_i32":
        return synth.make_tile(640, 700, 90, 12, "i32", 0.05), "recon"
    if name == "serpentine":
        return serpentine(200, 260, 13), "recon"
    if name == "fill_u8":
        f = synth.quantize(synth.make_field(700, 650, 120, 14, 0.3), "u8")
        return (synth.binary_from_mask(f), None), "fill"
    raise KeyError(name)


@pytest.mark.parametrize("name", ["synth_u8", "synth_i32", "serpentine", "fill_u8"])
@pytest.mark.parametrize("conn", [4, 8])
def test_schedule_invariance_repeated(name, conn):
    (a, m), op = _inputs(name)
    if op == "recon":
        want, _ = oracle.recon_dilate(a, m, conn)
    else:
        want, _ = oracle.fill_holes(a, conn)
    src = torch.from_numpy(a).to(DEV)
    d_mask = torch.from_numpy(m).to(DEV) if m is not None else None
    d_want = torch.from_numpy(want).to(DEV)
    work = torch.empty_like(src)
    H, W = a.shape
    mr_op = mrecon.MR_OP_RECON if op == "recon" else mrecon.MR_OP_FILL
    wss = {}
    reps = 25
    print(f"[gpu] stress {name} {a.shape} conn{conn}: {reps} x {len(STRESS_TUNES)} runs",
          flush=True)
    for rep in range(reps):
        for ti, tune in enumerate(STRESS_TUNES):
            if ti not in wss:
                wss[ti] = mrecon.alloc_workspace(
                    mrecon.workspace_bytes(mr_op, H, W, src.dtype, conn, tune), DEV)
            work.copy_(src)
            if op == "recon":
                mrecon.recon_dilate(work, d_mask, conn, tune=tune, workspace=wss[ti])
            else:
                mrecon.fill_holes(work, conn, tune=tune, workspace=wss[ti])
            mrecon.status(wss[ti])  # raises on a watchdog give-up
            if not torch.equal(work, d_want):
                got = work.cpu().numpy()
                pytest.fail(f"run {rep}, tune {tune}: " + first_mismatch(got, want))


def test_converge_mode_two_streams_alternating():
    # Each converge-mode call may return with its last poll copy still in
    # flight; a call that follows at once on another stream, with its own
    # workspace, must not read that copy as its own count.
    marker, mask = synth.make_tile(512, 600, 60, 21, "u8", 0.0)
    want, _ = oracle.recon_dilate(marker, mask, 8)
    tune = dict(sweep_rounds=-1, tail_rounds=0)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    src = torch.from_numpy(marker).to(DEV)
    k = torch.from_numpy(mask).to(DEV)
    ws = [mrecon.alloc_workspace(mrecon.workspace_bytes(mrecon.MR_OP_RECON, *marker.shape,
                                                        torch.uint8, 8, tune), DEV)
          for _ in streams]
    outs = []
    torch.cuda.synchronize()
    print("[gpu] converge mode alternating over two streams, 40 calls", flush=True)
    for i in range(40):
        s = streams[i & 1]
        with torch.cuda.stream(s):
            o = src.clone()
        mrecon.recon_dilate(o, k, 8, tune=tune, workspace=ws[i & 1], stream=s)
        outs.append(o)
    torch.cuda.synchronize()
    for i, o in enumerate(outs):
        got = o.cpu().numpy()
        assert np.array_equal(got, want), f"call {i}: " + first_mismatch(got, want)


def test_side_stream_binding_workspace():
    # The binding allocates the workspace on the current stream while the
    # call runs on a side stream; once the call returns, that block must not
    # be handed to new tensors on the current stream before the side
    # stream's kernels are done with it.
    marker, mask = synth.make_tile(1024, 1024, 200, 22, "u8", 0.0)
    want, _ = oracle.recon_dilate(marker, mask, 8)
    side = torch.cuda.Stream()
    src = torch.from_numpy(marker).to(DEV)
    k = torch.from_numpy(mask).to(DEV)
    nbytes = mrecon.workspace_bytes(mrecon.MR_OP_RECON, 1024, 1024, torch.uint8, 8)
    print("[gpu] side-stream calls with binding-allocated workspaces", flush=True)
    for i in range(10):
        torch.cuda.synchronize()
        o = src.clone()
        side.wait_stream(torch.cuda.current_stream())
        mrecon.recon_dilate(o, k, 8, stream=side)
        # new allocations of the same size on the current stream, written at once
        junk = [torch.full((nbytes,), 0xA5, dtype=torch.uint8, device=DEV) for _ in range(4)]
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        del junk
        got = o.cpu().numpy()
        assert np.array_equal(got, want), f"call {i}: " + first_mismatch(got, want)
