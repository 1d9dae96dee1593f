"""Pins for the CPU oracle: it must agree with routes that share nothing with it.

The oracle is a sequential raster / anti-raster + FIFO hybrid (Sec. V-C.2,
Algorithm 1). It is checked here against the operator's definition (brute
fixed-point iteration via scipy), a second algorithm family (widest-path
Dijkstra), textbook special cases reached through library routines
(``scipy.ndimage.label``, ``binary_fill_holes``), hand-derived golden
fixtures and structural invariants. The last test plants mistakes in copies
of the oracle and checks that these pins catch every one of them.
"""
import glob
import itertools
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
import refs
from paper_1311_0378_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------ exhaustive 3x3

def _three_state_stack(H, W):
    """Every image whose pixels take the (marker, mask) states
    (0,0), (0,1), (1,1) -- all distinct clipped binary pairs."""
    n = H * W
    codes = np.array(list(itertools.product(range(3), repeat=n)), dtype=np.uint8)
    marker = (codes == 2).astype(np.uint8).reshape(-1, H, W)
    mask = (codes >= 1).astype(np.uint8).reshape(-1, H, W)
    return marker, mask


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape", [(3, 3), (2, 4), (4, 2), (1, 7)])
def test_exhaustive_binary_vs_bruteforce(conn, shape):
    marker, mask = _three_state_stack(*shape)
    want = refs.brute_recon_batch(marker, mask, conn)
    for i in range(marker.shape[0]):
        got, _ = oracle.recon_dilate(marker[i], mask[i], conn)
        if not np.array_equal(got, want[i]):
            pytest.fail(f"state {i}: marker\n{marker[i]}\nmask\n{mask[i]}\n"
                        f"got\n{got}\nwant\n{want[i]}")


# ------------------------------------------------------------- serpentine

def serpentine(H, W, seed, dtype=np.uint8):
    """A one-pixel corridor that snakes through the image (rightwards on even
    lanes, leftwards on odd ones), with the only marker pixel at its far end
    and mask values that fall slowly away from that end. Scans in either
    raster order resolve little of it, so the queue phase carries most of the
    propagation, through many bottlenecks."""
    rng = np.random.default_rng(seed)
    mask = np.zeros((H, W), dtype=np.int64)
    path = []
    for lane, y in enumerate(range(0, H, 2)):
        xs = range(W) if lane % 2 == 0 else range(W - 1, -1, -1)
        path += [(y, x) for x in xs]
        if y + 1 < H:
            path.append((y + 1, W - 1 if lane % 2 == 0 else 0))
    vals = np.linspace(0, 215, len(path)).astype(np.int64) + rng.integers(0, 41, len(path))
    for (y, x), v in zip(path, vals):
        mask[y, x] = v
    marker = np.zeros_like(mask)
    y, x = path[-1]
    marker[y, x] = mask[y, x] = 255
    return marker.astype(dtype), mask.astype(dtype)


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("shape", [(15, 17), (30, 9), (9, 40)])
def test_serpentine_vs_bruteforce(conn, shape):
    marker, mask = serpentine(*shape, seed=sum(shape))
    got, cnt = oracle.recon_dilate(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.brute_recon(marker, mask, conn))
    np.testing.assert_array_equal(got, refs.widest_path(marker, mask, conn))
    assert cnt["pops"] > shape[0] * shape[1] // 4  # the queue phase did the work


# ------------------------------------------------------ random vs definition

@settings(max_examples=150, deadline=None)
@given(H=st.integers(1, 14), W=st.integers(1, 14), levels=st.sampled_from([2, 3, 4, 0]),
       conn=st.sampled_from([4, 8]), dt=st.sampled_from(["u8", "i32"]),
       seed=st.integers(0, 2**31 - 1))
def test_random_vs_bruteforce(H, W, levels, conn, dt, seed):
    rng = np.random.default_rng(seed)
    if dt == "u8":
        hi = levels if levels else 256
        mask = rng.integers(0, hi, (H, W)).astype(np.uint8)
        marker = rng.integers(0, hi, (H, W)).astype(np.uint8)
    else:
        if levels:
            vals = rng.integers(-2**31, 2**31 - 1, levels, dtype=np.int64)
            mask = rng.choice(vals, (H, W)).astype(np.int32)
            marker = rng.choice(vals, (H, W)).astype(np.int32)
        else:
            mask = rng.integers(-2**31, 2**31, (H, W), dtype=np.int64).astype(np.int32)
            marker = rng.integers(-2**31, 2**31, (H, W), dtype=np.int64).astype(np.int32)
    # half the cases keep marker <= mask, half exercise the clip
    if seed % 2:
        marker = np.minimum(marker, mask)
    got, _ = oracle.recon_dilate(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.brute_recon(marker, mask, conn))


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_synthetic_tile_vs_bruteforce(conn, dt):
    marker, mask = synth.make_tile(96, 120, 6, 11, dt, 0.3)
    got, cnt = oracle.recon_dilate(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.brute_recon(marker, mask, conn))
    assert cnt["passes"] == 2 and cnt["pops"] == cnt["pushes"]


# -------------------------------------------------- second algorithm family

@pytest.mark.parametrize("conn", [4, 8])
def test_vs_widest_path_synthetic(conn):
    marker, mask = synth.make_tile(64, 80, 3, 5, "u8", 0.0)
    got, _ = oracle.recon_dilate(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.widest_path(marker, mask, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_vs_widest_path_i32_full_range(conn):
    rng = np.random.default_rng(conn)
    mask = rng.integers(-2**31, 2**31, (40, 37), dtype=np.int64).astype(np.int32)
    marker = rng.integers(-2**31, 2**31, (40, 37), dtype=np.int64).astype(np.int32)
    got, _ = oracle.recon_dilate(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.widest_path(marker, mask, conn))


# ------------------------------------------------------- binary special case

@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("p", [0.45, 0.6])
def test_binary_components(conn, p):
    rng = np.random.default_rng(int(p * 100) + conn)
    mask = np.where(rng.random((70, 90)) < p, 255, 0).astype(np.uint8)
    marker = np.where(rng.random((70, 90)) < 0.01, 255, 0).astype(np.uint8)
    got, _ = oracle.recon_dilate(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.binary_recon(marker, mask, conn))


# ---------------------------------------------------------------- fill-holes

@pytest.mark.parametrize("conn", [4, 8])
def test_fill_binary_vs_scipy(conn):
    mask = synth.quantize(synth.make_field(160, 200, 40, 3, 0.5), "u8")
    img = synth.binary_from_mask(mask)
    got, _ = oracle.fill_holes(img, conn)
    np.testing.assert_array_equal(got, refs.binary_fill(img, conn))
    assert (got != img).any(), "the workload should contain holes"


@pytest.mark.parametrize("conn", [4, 8])
def test_fill_binary_random_vs_scipy(conn):
    rng = np.random.default_rng(40 + conn)
    img = np.where(rng.random((50, 61)) < 0.55, 255, 0).astype(np.uint8)
    got, _ = oracle.fill_holes(img, conn)
    np.testing.assert_array_equal(got, refs.binary_fill(img, conn))


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_fill_grey_vs_minmax(conn, dt):
    rng = np.random.default_rng(7 * conn)
    if dt == "u8":
        img = rng.integers(0, 6, (23, 29)).astype(np.uint8)
    else:
        img = rng.integers(-2**31, 2**31, (23, 29), dtype=np.int64).astype(np.int32)
    got, _ = oracle.fill_holes(img, conn)
    np.testing.assert_array_equal(got, refs.minmax_fill(img, conn))


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (2, 5), (6, 2)])
def test_fill_all_border_is_identity(shape):
    rng = np.random.default_rng(3)
    img = rng.integers(0, 256, shape).astype(np.uint8)
    for conn in (4, 8):
        got, _ = oracle.fill_holes(img, conn)
        np.testing.assert_array_equal(got, img)


# ------------------------------------------------------------------- golden

@pytest.mark.parametrize("path", sorted(glob.glob(os.path.join(GOLDEN, "*.txt"))),
                         ids=os.path.basename)
def test_golden(path):
    g = refs.load_golden(path)
    if g["op"] == "recon":
        got, _ = oracle.recon_dilate(g["marker"], g["mask"], g["conn"])
    else:
        got, _ = oracle.fill_holes(g["input"], g["conn"])
    np.testing.assert_array_equal(got, g["expected"])


# --------------------------------------------------------------- invariants

@pytest.fixture(scope="module", params=["u8", "i32"])
def tile(request):
    marker, mask = synth.make_tile(100, 130, 8, 21, request.param, 0.0)
    return marker, mask


@pytest.mark.parametrize("conn", [4, 8])
def test_invariants(tile, conn):
    marker, mask = tile
    R, _ = oracle.recon_dilate(marker, mask, conn)
    J0 = np.minimum(marker, mask)
    assert (J0 <= R).all() and (R <= mask).all()
    np.testing.assert_array_equal(oracle.recon_dilate(R, mask, conn)[0], R)  # idempotent
    np.testing.assert_array_equal(refs.geodesic_step(R, mask, conn), R)      # fixed point
    # monotone in the marker and in the mask
    bump = np.minimum(marker.astype(np.int64) + 3, np.iinfo(marker.dtype).max).astype(marker.dtype)
    assert (oracle.recon_dilate(bump, mask, conn)[0] >= R).all()
    mask_up = np.minimum(mask.astype(np.int64) + 2, np.iinfo(mask.dtype).max).astype(mask.dtype)
    assert (oracle.recon_dilate(marker, mask_up, conn)[0] >= R).all()
    # geometric equivariance
    for f in (np.transpose, np.fliplr, np.flipud, np.rot90):
        got, _ = oracle.recon_dilate(np.ascontiguousarray(f(marker)),
                                     np.ascontiguousarray(f(mask)), conn)
        np.testing.assert_array_equal(got, f(R))
    # marker = mask gives the mask; the lowest marker gives the lowest image
    np.testing.assert_array_equal(oracle.recon_dilate(mask, mask, conn)[0], mask)
    low = np.full_like(mask, np.iinfo(mask.dtype).min)
    np.testing.assert_array_equal(oracle.recon_dilate(low, mask, conn)[0], low)
    # h-dome bound: 0 <= I - R(I - h, I) <= h
    h = 30 if mask.dtype == np.uint8 else 7710
    dome = np.maximum(mask.astype(np.int64) - h, np.iinfo(mask.dtype).min).astype(mask.dtype)
    d = mask.astype(np.int64) - oracle.recon_dilate(dome, mask, conn)[0].astype(np.int64)
    assert d.min() >= 0 and d.max() <= h


def test_conn4_below_conn8(tile):
    marker, mask = tile
    assert (oracle.recon_dilate(marker, mask, 4)[0] <= oracle.recon_dilate(marker, mask, 8)[0]).all()


@pytest.mark.parametrize("conn", [4, 8])
def test_increasing_map_commutes(conn):
    """R(phi M, phi I) = phi R(M, I) for the increasing map phi(v) = 257 v,
    which ties the i32 result to the u8 result."""
    marker, mask = synth.make_tile(90, 77, 5, 4, "u8", 0.0)
    R8, _ = oracle.recon_dilate(marker, mask, conn)
    R32, _ = oracle.recon_dilate(marker.astype(np.int32) * 257, mask.astype(np.int32) * 257, conn)
    np.testing.assert_array_equal(R32, R8.astype(np.int32) * 257)


@pytest.mark.parametrize("conn", [4, 8])
def test_fill_invariants(conn):
    img = synth.quantize(synth.make_field(80, 96, 10, 9, 0.4), "u8")
    out, _ = oracle.fill_holes(img, conn)
    assert (out >= img).all()
    np.testing.assert_array_equal(out[[0, -1], :], img[[0, -1], :])
    np.testing.assert_array_equal(out[:, [0, -1]], img[:, [0, -1]])
    np.testing.assert_array_equal(oracle.fill_holes(out, conn)[0], out)
    o4, _ = oracle.fill_holes(img, 4)
    o8, _ = oracle.fill_holes(img, 8)
    assert (o8 <= o4).all()  # an 8-connected flood escapes more holes


# --------------------------------------------------- planted mistakes caught

def _battery(plant):
    """Run a cheap selection of the pins above on a planted oracle and return
    the names of the pins that fail."""
    fails = []
    rng = np.random.default_rng(123)
    for conn in (4, 8):
        marker, mask = _three_state_stack(3, 3)
        want = refs.brute_recon_batch(marker, mask, conn)
        for i in range(0, marker.shape[0], 7):
            got, _ = oracle.recon_dilate(marker[i], mask[i], conn, plant=plant)
            if not np.array_equal(got, want[i]):
                fails.append(f"exhaustive3x3/conn{conn}")
                break
        for t in range(30):
            H, W = rng.integers(2, 12, 2)
            mask = rng.integers(0, 4, (H, W)).astype(np.uint8)
            marker = rng.integers(0, 4, (H, W)).astype(np.uint8)
            got, _ = oracle.recon_dilate(marker, mask, conn, plant=plant)
            if not np.array_equal(got, refs.brute_recon(marker, mask, conn)):
                fails.append(f"random/conn{conn}")
                break
        marker, mask = synth.make_tile(48, 56, 2, 5, "u8", 0.0)
        got, _ = oracle.recon_dilate(marker, mask, conn, plant=plant)
        if not np.array_equal(got, refs.widest_path(marker, mask, conn)):
            fails.append(f"widest/conn{conn}")
        marker, mask = serpentine(15, 17, 1)
        got, _ = oracle.recon_dilate(marker, mask, conn, plant=plant)
        if not np.array_equal(got, refs.brute_recon(marker, mask, conn)):
            fails.append(f"serpentine/conn{conn}")
        img = synth.binary_from_mask(synth.quantize(synth.make_field(64, 64, 12, 9, 0.5), "u8"))
        got, _ = oracle.fill_holes(img, conn, plant=plant)
        if not np.array_equal(got, refs.binary_fill(img, conn)):
            fails.append(f"fill/conn{conn}")
        for t in range(30):
            H, W = rng.integers(2, 12, 2)
            mask = rng.integers(0, 4, (H, W)).astype(np.uint8)
            marker = rng.integers(0, 4, (H, W)).astype(np.uint8)
            got, _ = oracle.recon_erode(marker, mask, conn, plant=plant)
            if not np.array_equal(got, refs.brute_erode(marker, mask, conn)):
                fails.append(f"erode-random/conn{conn}")
                break
        marker, mask = synth.make_erode_tile(40, 44, 2, 5, "u8", 0.0)
        got, _ = oracle.recon_erode(marker, mask, conn, plant=plant)
        if not np.array_equal(got, refs.minimax_path(marker, mask, conn)):
            fails.append(f"erode-minimax/conn{conn}")
    return fails


@pytest.mark.parametrize("plant", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_planted_mistakes_are_caught(plant):
    """Each planted mistake (a neighbour missing from the seed test, a skipped queue phase, a
    wrong operator, a mask read at the wrong pixel, wrap-around at the edge, missing border
    seeds, an off-by-one loop bound, an erosion marker clipped with max instead of min, an
    erosion mask not complemented) must fail at least one pin."""
    oracle.build(plant=plant, force=True)
    assert _battery(plant), f"planted mistake {plant} slipped through every pin"


def test_clean_oracle_passes_battery():
    assert _battery(0) == []


# ------------------------------------------------- reconstruction by erosion

@settings(max_examples=120, deadline=None)
@given(H=st.integers(1, 14), W=st.integers(1, 14), levels=st.sampled_from([2, 3, 4, 0]),
       conn=st.sampled_from([4, 8]), dt=st.sampled_from(["u8", "i32"]),
       seed=st.integers(0, 2**31 - 1))
def test_erode_random_vs_bruteforce(H, W, levels, conn, dt, seed):
    rng = np.random.default_rng(seed)
    if dt == "u8":
        hi = levels if levels else 256
        mask = rng.integers(0, hi, (H, W)).astype(np.uint8)
        marker = rng.integers(0, hi, (H, W)).astype(np.uint8)
    else:
        lo, top = (-2**31, 2**31)
        if levels:
            vals = rng.integers(lo, top - 1, levels, dtype=np.int64)
            mask = rng.choice(vals, (H, W)).astype(np.int32)
            marker = rng.choice(vals, (H, W)).astype(np.int32)
        else:
            mask = rng.integers(lo, top, (H, W), dtype=np.int64).astype(np.int32)
            marker = rng.integers(lo, top, (H, W), dtype=np.int64).astype(np.int32)
    if seed % 2:  # half the cases keep marker >= mask, half exercise the clip
        marker = np.maximum(marker, mask)
    got, _ = oracle.recon_erode(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.brute_erode(marker, mask, conn))


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_erode_synthetic_vs_bruteforce_and_minimax(conn, dt):
    marker, mask = synth.make_erode_tile(72, 90, 4, 3, dt, 0.3)
    got, _ = oracle.recon_erode(marker, mask, conn)
    np.testing.assert_array_equal(got, refs.brute_erode(marker, mask, conn))
    np.testing.assert_array_equal(got, refs.minimax_path(marker, mask, conn))


@pytest.mark.parametrize("conn", [4, 8])
def test_erode_binary_components(conn):
    # binary special case: marker all high except seeds of 0; the result keeps
    # 0 on the background components (mask == 0) that hold a seed, 1 elsewhere
    rng = np.random.default_rng(conn + 10)
    mask = (rng.random((40, 50)) < 0.45).astype(np.uint8)
    seeds = rng.random((40, 50)) < 0.02
    marker = np.where(seeds, 0, 1).astype(np.uint8)
    got, _ = oracle.recon_erode(marker, mask, conn)
    lab, _ = refs.ndi.label(mask == 0, structure=refs.footprint(conn))
    keep = np.unique(lab[seeds & (mask == 0)])
    keep = keep[keep > 0]
    expect = np.where(np.isin(lab, keep), 0, 1).astype(np.uint8)
    np.testing.assert_array_equal(got, expect)


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", ["u8", "i32"])
def test_erode_invariants(conn, dt):
    marker, mask = synth.make_erode_tile(80, 64, 4, 9, dt, 0.2)
    E, _ = oracle.recon_erode(marker, mask, conn)
    assert (mask <= E).all() and (E <= np.maximum(marker, mask)).all()
    # a fixed point of the elementary geodesic erosion, and idempotent
    fp = refs.footprint(conn)
    step = np.maximum(refs.ndi.grey_erosion(E, footprint=fp, mode="constant",
                                            cval=refs.maxval(E.dtype)), mask)
    np.testing.assert_array_equal(step, E)
    E2, _ = oracle.recon_erode(E, mask, conn)
    np.testing.assert_array_equal(E2, E)
    # 8-connectivity reaches at least as far down as 4-connectivity
    if conn == 8:
        E4, _ = oracle.recon_erode(marker, mask, 4)
        assert (E <= E4).all()
