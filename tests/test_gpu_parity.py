"""Parity of the HIP path with the CPU oracle, element by element (bit-exact).

The result of reconstruction and of fill-holes is unique (the least fixed
point of the geodesic dilation), and all arithmetic is integer, so every
pixel must match exactly, for every tuning of the sweep/queue split.
"""
import glob
import os

import numpy as np
import pytest

import oracle
import refs
from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only hosts too
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import first_mismatch, gpu_fill, gpu_recon  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

TUNES = [None, dict(sweep_rounds=1, max_sweeps=1), dict(sweep_rounds=2, max_sweeps=3),
         dict(sweep_rounds=-1), dict(sweep_rounds=8, persistent_blocks=3),
         dict(sweep_rounds=-1, converge_rounds=2), dict(sweep_rounds=-1, tail_rounds=1),
         dict(sweep_rounds=-1, tail_rounds=2, max_sweeps=1),
         dict(sweep_rounds=-1, first_sweeps=16), dict(sweep_rounds=-1, tail_rounds=2, first_sweeps=3),
         dict(sweep_rounds=3, first_sweeps=1024)]


def check(got, want):
    assert np.array_equal(got, want), first_mismatch(got, want)


@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))),
                         ids=os.path.basename)
def test_golden(path):
    g = refs.load_golden(path)
    if g["op"] == "recon":
        got = gpu_recon(g["marker"], g["mask"], g["conn"])
    else:
        got = gpu_fill(g["input"], g["conn"])
    check(got, g["expected"])


SHAPES = [(1, 1), (1, 200), (200, 1), (2, 3), (61, 62), (62, 62), (63, 64), (64, 65),
          (124, 125), (130, 70), (187, 251)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_recon_random_shapes(shape, conn, dt):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1] * 10 + conn + (dt == "i32"))
    if dt == "u8":
        mask = rng.integers(0, 6, shape).astype(np.uint8)
        marker = rng.integers(0, 6, shape).astype(np.uint8)
    else:
        mask = rng.integers(-2**31, 2**31, shape, dtype=np.int64).astype(np.int32)
        marker = rng.integers(-2**31, 2**31, shape, dtype=np.int64).astype(np.int32)
    want, _ = oracle.recon_dilate(marker, mask, conn)
    check(gpu_recon(marker, mask, conn), want)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("conn", [4, 8])
def test_fill_random_shapes(shape, conn):
    rng = np.random.default_rng(sum(shape) + conn)
    img = rng.integers(0, 5, shape).astype(np.uint8)
    want, _ = oracle.fill_holes(img, conn)
    check(gpu_fill(img, conn), want)


@pytest.mark.parametrize("tune", TUNES, ids=str)
@pytest.mark.parametrize("conn", [4, 8])
def test_recon_synthetic_tunes(tune, conn):
    marker, mask = synth.make_tile(300, 517, 30, 3, "u8", 0.1)
    want, _ = oracle.recon_dilate(marker, mask, conn)
    check(gpu_recon(marker, mask, conn, tune=tune), want)


@pytest.mark.parametrize("tune", TUNES, ids=str)
@pytest.mark.parametrize("conn", [4, 8])
def test_fill_synthetic_tunes(tune, conn):
    img = synth.binary_from_mask(synth.quantize(synth.make_field(311, 400, 60, 5, 0.4), "u8"))
    want, _ = oracle.fill_holes(img, conn)
    check(gpu_fill(img, conn, tune=tune), want)


@pytest.mark.parametrize("conn", [4, 8])
def test_serpentine_queue_heavy(conn):
    from test_oracle_pins import serpentine
    marker, mask = serpentine(127, 129, 7)
    want, _ = oracle.recon_dilate(marker, mask, conn)
    # the last tunes stop the tile rounds early and leave the long corridor to
    # the seed pass and the queue phase
    for tune in (None, dict(sweep_rounds=1, max_sweeps=1), dict(sweep_rounds=-1, converge_rounds=1),
                 dict(sweep_rounds=-1, converge_rounds=5), dict(sweep_rounds=-1, tail_rounds=1),
                 dict(sweep_rounds=-1, tail_rounds=1, max_sweeps=1)):
        got, c = gpu_recon(marker, mask, conn, tune=tune, counters=True)
        check(got, want)


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("tail", [1, 3])
def test_serpentine_tile_queue(conn, tail):
    """A corridor through 10 x 12 tiles: the tile queue carries the chain from
    tile to tile, requeueing tiles that are marked while they are visited."""
    from test_oracle_pins import serpentine
    marker, mask = serpentine(600, 700, 11)
    want, _ = oracle.recon_dilate(marker, mask, conn)
    for ms in (16, 1):
        got, c = gpu_recon(marker, mask, conn, tune=dict(sweep_rounds=-1, tail_rounds=tail,
                                                          max_sweeps=ms), counters=True)
        check(got, want)
        assert c["rounds"] == tail and c["tiles"] > 0


@pytest.mark.parametrize("W", [1, 5, 17, 62, 63, 77, 130])
@pytest.mark.parametrize("conn", [4, 8])
def test_aligned_pitch_shapes(W, conn):
    """Rows padded to a multiple of 16 bytes take the staged wide-load path;
    odd widths leave ragged tails inside the padding and at the plane end."""
    rng = np.random.default_rng(W * 10 + conn)
    for H in (1, 3, 66, 131):
        mask = rng.integers(0, 7, (H, W)).astype(np.uint8)
        marker = rng.integers(0, 7, (H, W)).astype(np.uint8)
        pad = (-W) % 16
        want, _ = oracle.recon_dilate(marker, mask, conn)
        check(gpu_recon(marker, mask, conn, pad=pad), want)
        wantf, _ = oracle.fill_holes(mask, conn)
        check(gpu_fill(mask, conn, pad=pad), wantf)


def test_pitched_rows():
    marker, mask = synth.make_tile(200, 333, 20, 8, "u8", 0.0)
    want, _ = oracle.recon_dilate(marker, mask, 8)
    check(gpu_recon(marker, mask, 8, pad=37), want)
    img = synth.binary_from_mask(mask)
    wantf, _ = oracle.fill_holes(img, 8)
    check(gpu_fill(img, 8, pad=13), wantf)


def test_i32_full_range_fill():
    rng = np.random.default_rng(5)
    img = rng.integers(-2**31, 2**31, (150, 170), dtype=np.int64).astype(np.int32)
    for conn in (4, 8):
        want, _ = oracle.fill_holes(img, conn)
        check(gpu_fill(img, conn), want)


def test_clip_marker_above_mask():
    marker, mask = synth.make_tile(256, 256, 12, 1, "u8", 0.0)
    marker = np.maximum(marker, 100).astype(np.uint8)  # many pixels above the mask
    want, _ = oracle.recon_dilate(marker, mask, 8)
    check(gpu_recon(marker, mask, 8, tune=dict(sweep_rounds=1, max_sweeps=1)), want)


def test_counters():
    marker, mask = synth.make_tile(256, 256, 12, 1, "u8", 0.0)
    want, _ = oracle.recon_dilate(marker, mask, 8)
    got, c = gpu_recon(marker, mask, 8, tune=dict(sweep_rounds=1, max_sweeps=1), counters=True)
    check(got, want)
    assert c["rounds"] == 1 and c["tiles"] == 25  # one visit of each 62x62 tile
    assert c["pops"] >= c["seeds"] > 0


@pytest.mark.parametrize("conn", [4, 8])
def test_queue_widened_plane_and_dword_cas(conn):
    # uint8 queue phase: with a workspace sized by the queue tune the pixels
    # are raised on a widened 32-bit plane (no compare-and-swap retries);
    # sized by the default tune, the same call raises them with the dword
    # compare-and-swap. Both must give the oracle's result, on a synthetic
    # tile and on a serpentine corridor, pitched rows included.
    from gpu_util import to_dev
    from paper_1311_0378_amd import mrecon
    from test_oracle_pins import serpentine
    tune = dict(sweep_rounds=1, max_sweeps=1)
    for marker, mask in (synth.make_tile(300, 411, 40, 2, "u8", 0.0), serpentine(127, 129, 7)):
        want, _ = oracle.recon_dilate(marker, mask, conn)
        for sized, pad in ((tune, 0), (None, 0), (tune, 13)):
            m, k = to_dev(marker, pad), to_dev(mask, pad)
            nb = mrecon.workspace_bytes(mrecon.MR_OP_RECON, *marker.shape, m.dtype, conn, sized)
            ws = mrecon.alloc_workspace(nb, m.device)
            print(f"[gpu] queue plane {marker.shape} conn{conn} sized={sized} pad={pad}",
                  flush=True)
            mrecon.recon_dilate(m, k, conn, tune=tune, workspace=ws)
            c = mrecon.read_counters(ws)
            check(m.cpu().numpy(), want)
            assert c["pops"] > 0
            if sized is not None:
                assert c["cas_retries"] == 0
    # fill-holes and a batch on widened planes
    img = synth.binary_from_mask(synth.make_tile(257, 300, 30, 4, "u8", 0.2)[1])
    wantf, _ = oracle.fill_holes(img, conn)
    check(gpu_fill(img, conn, tune=tune), wantf)
    items = [synth.make_tile(h, w, 10, 5 + i, "u8", 0.0) for i, (h, w) in
             enumerate([(130, 200), (64, 64), (311, 97)])]
    ms = [torch.from_numpy(a).cuda() for a, _ in items]
    ks = [torch.from_numpy(b).cuda() for _, b in items]
    mrecon.batch([(a, b, mrecon.MR_OP_RECON) for a, b in zip(ms, ks)], conn, tune=tune)
    for (a, b), got in zip(items, ms):
        check(got.cpu().numpy(), oracle.recon_dilate(a, b, conn)[0])


# ---------------------------------------------------------- workload sizes

def test_workload_1024():
    marker, mask = synth.single_1024()
    want, _ = oracle.recon_dilate(marker, mask, 8)
    check(gpu_recon(marker, mask, 8), want)


@pytest.fixture(scope="module")
def w4096():
    return synth.single_4096()


@pytest.mark.parametrize("conn", [4, 8])
def test_workload_4096_recon(w4096, conn):
    marker, mask, _ = w4096
    want, _ = oracle.recon_dilate(marker, mask, conn)
    check(gpu_recon(marker, mask, conn), want)


@pytest.mark.parametrize("conn", [4, 8])
def test_workload_4096_fill(w4096, conn):
    img = w4096[2]
    want, _ = oracle.fill_holes(img, conn)
    check(gpu_fill(img, conn), want)


@pytest.mark.parametrize("conn", [4, 8])
def test_converge_batches_and_cap(conn):
    """Converge mode enqueues the next batch of 8 rounds before it reads the
    previous batch's count. A cap that falls inside a batch enqueued ahead
    stops the rounds there and hands the rest to the queue phase; without a
    cap the rounds run in whole batches until none is dirty."""
    from test_oracle_pins import serpentine
    # a corridor through 10 x 12 tiles needs far more rounds than the caps
    marker, mask = serpentine(600, 700, 11)
    want, _ = oracle.recon_dilate(marker, mask, conn)
    for cap in (12, 20):
        tune = dict(sweep_rounds=-1, tail_rounds=0, converge_rounds=cap, max_sweeps=1)
        got, c = gpu_recon(marker, mask, conn, tune=tune, counters=True)
        check(got, want)
        assert c["rounds"] == cap and c["pops"] > 0
    # a corridor through 3 x 3 tiles converges in rounds alone
    marker, mask = serpentine(127, 129, 7)
    want, _ = oracle.recon_dilate(marker, mask, conn)
    got, c = gpu_recon(marker, mask, conn, tune=dict(sweep_rounds=-1, tail_rounds=0),
                       counters=True)
    check(got, want)
    assert c["rounds"] < 1000 and (c["rounds"] - 1) % 8 == 0 and c["pops"] == 0
