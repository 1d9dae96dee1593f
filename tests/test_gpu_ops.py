"""Parity of the Table II operations beside reconstruction (include/mr_ops.h)
with the oracle, element by element. Every result here is unique and
integer, so the bar is bit-exactness: h-dome and regional maxima on the
reconstruction engine, RGB2Gray, erosion / dilation / opening by the 13 x 13
disk, the distance transform, connected components and area threshold.
Shapes cover single pixels, ragged edges of the kernels' tiles, pitched rows
and the degenerate inputs of each operation; the full-size workload sizes
are checked exactly where the oracle is quick and on sampled windows where
it is not."""
import numpy as np
import pytest

import oracle
from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import DEV, first_mismatch, to_dev  # noqa: E402
from paper_1311_0378_amd import ops  # noqa: E402


def check(got, want, what=""):
    assert np.array_equal(got, want), what + first_mismatch(got, want)


SHAPES = [(1, 1), (1, 97), (97, 1), (2, 3), (61, 62), (63, 64), (64, 65), (130, 70),
          (187, 251), (300, 517)]


# ------------------------------------------------------ h-dome, regional max

@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_hdome_and_rmax_random(shape, conn, dt):
    rng = np.random.default_rng(shape[0] * 7 + shape[1] + conn)
    if dt == "u8":
        f = rng.integers(0, 9, shape).astype(np.uint8) * 25
        hs = [0, 1, 30, 300]
    else:
        f = (rng.integers(-3, 4, shape).astype(np.int64) * 600_000_000).astype(np.int32)
        hs = [0, 1, 700_000_000, 2**31 - 1]
    print(f"[gpu] hdome/rmax {shape} {dt} conn{conn}", flush=True)
    for h in hs:
        d = to_dev(f)
        ops.hdome(d, h, conn)
        check(d.cpu().numpy(), oracle.hdome(f, h, conn), f"h={h}: ")
    check(ops.regional_maxima(to_dev(f), conn).cpu().numpy(), oracle.regional_maxima(f, conn))


def test_rmax_constant_min_and_pitched():
    f = np.zeros((70, 90), np.uint8)
    check(ops.regional_maxima(to_dev(f), 8).cpu().numpy(), np.full((70, 90), 255, np.uint8))
    g = np.full((33, 40), np.iinfo(np.int32).min, np.int32)
    check(ops.regional_maxima(to_dev(g), 4).cpu().numpy(), np.full((33, 40), 255, np.uint8))
    _, mask = synth.make_tile(300, 411, 40, 9, "u8", 0.1)
    d = to_dev(mask, pad=29)
    check(ops.regional_maxima(d, 8).cpu().numpy(), oracle.regional_maxima(mask, 8))
    ops.hdome(d, 40, 8)
    check(d.cpu().numpy(), oracle.hdome(mask, 40, 8))


@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_hdome_rmax_word_path_partial_words(dt):
    # 16-byte aligned planes and pitch with a ragged last word per row: the
    # streaming passes take whole 16-byte words and finish each row pixel by
    # pixel; the output plane is aligned too, so regional maxima writes words
    _, mask = synth.make_tile(150, 411, 30, 3, dt, 0.1)
    d = to_dev(mask, pad=5)  # pitch 416
    out = torch.full((150, 416), 7, dtype=torch.uint8, device=DEV)[:, :411]
    ops.regional_maxima(d, 8, out=out)
    check(out.cpu().numpy(), oracle.regional_maxima(mask, 8))
    h = 40 if dt == "u8" else 40 * 257
    ops.hdome(d, h, 8)
    check(d.cpu().numpy(), oracle.hdome(mask, h, 8))


@pytest.mark.parametrize("conn", [4, 8])
def test_hdome_rmax_synthetic_4096(conn):
    _, mask, _ = synth.single_4096()
    print(f"[gpu] hdome/rmax 4096^2 conn{conn}", flush=True)
    d = to_dev(mask)
    ops.hdome(d, 20, conn)
    check(d.cpu().numpy(), oracle.hdome(mask, 20, conn))
    check(ops.regional_maxima(to_dev(mask), conn).cpu().numpy(), oracle.regional_maxima(mask, conn))


# ---------------------------------------------------------------- RGB2Gray

def test_rgb2gray_every_colour():
    v = np.arange(256, dtype=np.uint8)
    r, g, b = np.meshgrid(v, v, v, indexing="ij")
    rgb = np.stack([r, g, b], -1).reshape(4096, 4096, 3)
    print("[gpu] rgb2gray over all 2^24 colours", flush=True)
    got = ops.rgb2gray(torch.from_numpy(rgb).to(DEV)).cpu().numpy()
    check(got, oracle.rgb2gray(rgb))


@pytest.mark.parametrize("shape", [(1, 1), (3, 15), (5, 16), (7, 17), (64, 1000), (33, 4097)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("pad", [0, 5, 16])
def test_rgb2gray_shapes_and_pitches(shape, pad):
    rng = np.random.default_rng(shape[1] + pad)
    H, W = shape
    rgb = rng.integers(0, 256, (H, W, 3)).astype(np.uint8)
    big = torch.zeros((H, W + pad, 3), dtype=torch.uint8)
    big[:, :W] = torch.from_numpy(rgb)
    d = big.to(DEV)[:, :W]
    out = torch.full((H, W + pad), 7, dtype=torch.uint8, device=DEV)[:, :W]
    ops.rgb2gray(d, out=out)
    check(out.cpu().numpy(), oracle.rgb2gray(rgb))


# -------------------------------------------------------- 13 x 13 disk

DISK_SHAPES = [(1, 1), (1, 600), (600, 1), (5, 40), (13, 13), (63, 511), (64, 512), (65, 513),
               (129, 1030), (200, 777), (128, 239), (127, 240), (129, 241), (257, 480),
               (256, 481), (300, 721)]


@pytest.mark.parametrize("shape", DISK_SHAPES, ids=lambda s: f"{s[0]}x{s[1]}")
def test_disk_erode_dilate_open(shape):
    rng = np.random.default_rng(sum(shape))
    f = rng.integers(0, 256, shape).astype(np.uint8)
    print(f"[gpu] disk13 {shape}", flush=True)
    d = to_dev(f)
    check(ops.disk13(ops.MR_DISK_ERODE, d).cpu().numpy(), oracle.erode_disk13(f), "erode: ")
    check(ops.disk13(ops.MR_DISK_DILATE, d).cpu().numpy(), oracle.dilate_disk13(f), "dilate: ")
    check(ops.open_disk13(d).cpu().numpy(), oracle.open_disk13(f), "open: ")


def test_disk_open_pitched_synthetic():
    _, mask = synth.make_tile(700, 1100, 140, 4, "u8", 0.05)
    for pad in (3, 64):
        d = to_dev(mask, pad=pad)
        check(ops.open_disk13(d).cpu().numpy(), oracle.open_disk13(mask), f"pad {pad}: ")


# ------------------------------------------------------- distance transform

@pytest.mark.parametrize("shape", SHAPES + [(640, 700)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("conn", [4, 8])
def test_dt_random(shape, conn):
    rng = np.random.default_rng(shape[0] + 3 * shape[1] + conn)
    img = ((rng.random(shape) < 0.93) * 255).astype(np.uint8)
    print(f"[gpu] dt {shape} conn{conn}", flush=True)
    check(ops.distance_transform(to_dev(img), conn).cpu().numpy(),
          oracle.distance_transform(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_dt_edge_cases(conn):
    for img in (np.ones((130, 200), np.uint8), np.zeros((130, 200), np.uint8)):
        check(ops.distance_transform(to_dev(img), conn).cpu().numpy(),
              oracle.distance_transform(img, conn))
    # one background pixel in a corner of a large image: the wave crosses
    # dozens of tiles diagonally, one round per tile hop
    img = np.ones((1500, 1300), np.uint8)
    img[0, 0] = 0
    print(f"[gpu] dt single corner seed conn{conn}", flush=True)
    check(ops.distance_transform(to_dev(img, pad=17), conn).cpu().numpy(),
          oracle.distance_transform(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_dt_synthetic_4096(conn):
    _, _, img = synth.single_4096()
    print(f"[gpu] dt 4096^2 conn{conn}", flush=True)
    check(ops.distance_transform(to_dev(img), conn).cpu().numpy(),
          oracle.distance_transform(img, conn))


# ------------------------------------------------- components, area threshold

@pytest.mark.parametrize("shape", SHAPES + [(640, 700)], ids=lambda s: f"{s[0]}x{s[1]}")
@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("p", [0.4, 0.6])
def test_ccl_random(shape, conn, p):
    rng = np.random.default_rng(shape[0] * 31 + shape[1] + conn + int(10 * p))
    img = ((rng.random(shape) < p) * 255).astype(np.uint8)
    print(f"[gpu] ccl {shape} conn{conn} p={p}", flush=True)
    got = ops.ccl(to_dev(img), conn).cpu().numpy()
    check(got, oracle.ccl(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_ccl_snakes_and_edges(conn):
    from test_oracle_pins import serpentine
    _, mask = serpentine(301, 257, 3)
    img = (mask > 0).astype(np.uint8)
    want = oracle.ccl(img, conn)
    check(ops.ccl(to_dev(img, pad=9), conn).cpu().numpy(), want)
    # label rows with a pitch: the forest lives in the workspace, not in place
    out = torch.full((301, 257 + 7), 5, dtype=torch.int32, device=DEV)[:, :257]
    ops.ccl(to_dev(img), conn, out=out)
    check(out.cpu().numpy(), want, "pitched labels: ")
    for img in (np.zeros((70, 130), np.uint8), np.ones((70, 130), np.uint8)):
        check(ops.ccl(to_dev(img), conn).cpu().numpy(), oracle.ccl(img, conn))
    # stripes one pixel wide joined at alternate ends: one component that
    # crosses every tile border many times
    img = np.zeros((300, 200), np.uint8)
    img[::2] = 1
    img[1::4, -1] = 1
    img[3::4, 0] = 1
    check(ops.ccl(to_dev(img), conn).cpu().numpy(), oracle.ccl(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_ccl_area_synthetic_4096(conn):
    _, _, img = synth.single_4096()
    print(f"[gpu] ccl + area 4096^2 conn{conn}", flush=True)
    lab = ops.ccl(to_dev(img), conn)
    want = oracle.ccl(img, conn)
    check(lab.cpu().numpy(), want)
    for lo, hi in [(150, 500), (1, 10**9), (700, 100)]:
        l2 = lab.clone()
        _, ws = ops.area_threshold(l2, lo, hi)
        w2, areas = oracle.area_threshold(want, lo, hi)
        check(l2.cpu().numpy(), w2, f"[{lo},{hi}]: ")
        got_areas = ws[: 4 * (want.size + 1)].view(torch.int32).cpu().numpy()
        assert np.array_equal(got_areas, areas.astype(np.int32))


@pytest.mark.parametrize("H,W,pad", [(97, 131, 3), (64, 128, 4), (33, 200, 0), (5, 4, 0)])
def test_area_threshold_random_labels(H, W, pad):
    # (widths and pitches that are multiples of 4 take the 16-byte word path)
    rng = np.random.default_rng(5 + W)
    lab = rng.integers(0, min(40, H * W + 1), (H, W)).astype(np.int32)
    lab[rng.random((H, W)) < 0.3] = 0
    lab[0, 0] = H * W  # the largest label a plane can hold
    for lo, hi in [(0, 10**9), (60, 90), (100, 100), (5, 4), (1, 1)]:
        d = to_dev(lab, pad=pad)
        ops.area_threshold(d, lo, hi)
        check(d.cpu().numpy(), oracle.area_threshold(lab, lo, hi)[0], f"[{lo},{hi}]: ")
