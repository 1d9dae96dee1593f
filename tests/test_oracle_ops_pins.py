"""Pins of the oracle for the Table II operations beside reconstruction.

Each operation is checked against something other than itself: a library
routine that computes the same thing (scipy.ndimage), the definition worked
out by brute force on small inputs, values fixed by the definition's
constants (worked examples written out by hand), and invariants. The last
tests plant one mistake at a time in a copy of the oracle and show that the
pins catch it.
"""
import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
import refs

# ---------------------------------------------------------------- RGB2Gray


def test_rgb2gray_exhaustive_within_one_of_real_weights():
    # every 24-bit colour: within 1 of round(0.299 R + 0.587 G + 0.114 B),
    # the BT.601 luma in real arithmetic
    v = np.arange(256, dtype=np.uint8)
    r, g, b = np.meshgrid(v, v, v, indexing="ij")
    rgb = np.stack([r, g, b], -1).reshape(4096, 4096, 3)
    got = oracle.rgb2gray(rgb).astype(np.int64)
    real = np.rint(0.299 * rgb[..., 0] + 0.587 * rgb[..., 1] + 0.114 * rgb[..., 2]).astype(np.int64)
    assert np.abs(got - real).max() <= 1


def test_rgb2gray_gray_is_fixed_and_hand_values():
    # R = G = B = v gives v (the weights sum to one); pure primaries at full
    # scale, worked by hand: 4899*255 + 8192 = 1257437 -> 76;
    # 9617*255 + 8192 = 2460527 -> 150; 1868*255 + 8192 = 484532 -> 29
    v = np.arange(256, dtype=np.uint8)
    grey = np.stack([v, v, v], -1)[None]
    assert np.array_equal(oracle.rgb2gray(grey)[0], v)
    prim = np.array([[[255, 0, 0], [0, 255, 0], [0, 0, 255], [255, 255, 255], [0, 0, 0]]],
                    np.uint8)
    assert oracle.rgb2gray(prim).tolist() == [[76, 150, 29, 255, 0]]


def test_rgb2gray_monotone_per_channel():
    rng = np.random.default_rng(1)
    a = rng.integers(0, 255, (64, 64, 3)).astype(np.uint8)
    base = oracle.rgb2gray(a).astype(int)
    for c in range(3):
        b = a.copy()
        b[..., c] += 1
        assert (oracle.rgb2gray(b).astype(int) >= base).all()


# ------------------------------------------------------- opening, 13x13 disk

DISK = np.array([[dy * dy + dx * dx <= 36 for dx in range(-6, 7)] for dy in range(-6, 7)])


def test_disk_shape_from_erosion_of_a_point():
    # eroding a white image with one black pixel paints the structuring
    # element: 113 offsets in the radius-6 disk (13 + 2 * (11 + 11 + 11 + 9 + 7 + 1))
    f = np.full((31, 31), 255, np.uint8)
    f[15, 15] = 0
    e = oracle.erode_disk13(f)
    assert int((e == 0).sum()) == 113
    assert np.array_equal(e[9:22, 9:22] == 0, DISK)


@pytest.mark.parametrize("shape", [(1, 1), (5, 40), (37, 29), (64, 70)])
def test_erode_dilate_open_vs_scipy(shape):
    rng = np.random.default_rng(sum(shape))
    f = rng.integers(0, 256, shape).astype(np.uint8)
    # pixels outside are ignored: constant padding with the identity of each
    e = ndi.grey_erosion(f, footprint=DISK, mode="constant", cval=255)
    d = ndi.grey_dilation(f, footprint=DISK, mode="constant", cval=0)
    o = ndi.grey_dilation(e, footprint=DISK, mode="constant", cval=0)
    assert np.array_equal(oracle.erode_disk13(f), e)
    assert np.array_equal(oracle.dilate_disk13(f), d)
    assert np.array_equal(oracle.open_disk13(f), o)


def test_open_invariants_and_objects():
    rng = np.random.default_rng(7)
    f = ndi.uniform_filter(rng.integers(0, 256, (80, 90)).astype(np.float64), 5).astype(np.uint8)
    o = oracle.open_disk13(f)
    assert (o <= f).all()                                  # anti-extensive
    assert np.array_equal(oracle.open_disk13(o), o)        # idempotent
    g = f.copy()
    g[10:20, 10:20] = np.maximum(g[10:20, 10:20], 5)
    assert (oracle.open_disk13(g) >= o).all()              # increasing
    # a bright 5 x 5 square on black is removed; a bright radius-6 disk stays
    b = np.zeros((40, 40), np.uint8)
    b[5:10, 5:10] = 200
    b[20:33, 20:33][DISK] = 180
    ob = oracle.open_disk13(b)
    assert ob[5:10, 5:10].max() == 0
    assert np.array_equal(ob[20:33, 20:33][DISK], np.full(113, 180, np.uint8))


# ------------------------------------------------------- distance transform


def _brute_dt(img, conn):
    H, W = img.shape
    bg = np.argwhere(img == 0)
    out = np.full((H, W), -1, np.int32)
    if not len(bg):
        return out
    for y in range(H):
        for x in range(W):
            dy = np.abs(bg[:, 0] - y)
            dx = np.abs(bg[:, 1] - x)
            out[y, x] = (np.maximum(dy, dx) if conn == 8 else dy + dx).min()
    return out


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("seed", range(4))
def test_dt_vs_bruteforce_and_scipy(conn, seed):
    rng = np.random.default_rng(seed)
    img = ((rng.random((23, 31)) < 0.85) * int(rng.integers(1, 256))).astype(np.uint8)
    want = _brute_dt(img, conn)
    got = oracle.distance_transform(img, conn)
    assert np.array_equal(got, want)
    metric = "chessboard" if conn == 8 else "taxicab"
    assert np.array_equal(got, ndi.distance_transform_cdt(img, metric=metric))


@pytest.mark.parametrize("conn", [4, 8])
def test_dt_disks_vs_scipy(conn):
    from paper_1311_0378_amd import synth
    img = synth.binary_from_mask(synth.make_tile(300, 260, 40, 5, "u8", 0.2)[1])
    metric = "chessboard" if conn == 8 else "taxicab"
    assert np.array_equal(oracle.distance_transform(img, conn),
                          ndi.distance_transform_cdt(img, metric=metric))


def test_dt_edge_cases():
    assert (oracle.distance_transform(np.ones((4, 5), np.uint8), 8) == -1).all()
    assert (oracle.distance_transform(np.zeros((4, 5), np.uint8), 8) == 0).all()
    # a single background pixel in a corner: chessboard and city block
    img = np.ones((4, 5), np.uint8)
    img[0, 0] = 0
    yy, xx = np.mgrid[:4, :5]
    assert np.array_equal(oracle.distance_transform(img, 8), np.maximum(yy, xx))
    assert np.array_equal(oracle.distance_transform(img, 4), yy + xx)


def test_dt_lipschitz():
    rng = np.random.default_rng(3)
    img = (rng.random((50, 60)) < 0.97).astype(np.uint8)
    for conn in (4, 8):
        d = oracle.distance_transform(img, conn).astype(int)
        assert (np.abs(np.diff(d, axis=0)) <= 1).all() and (np.abs(np.diff(d, axis=1)) <= 1).all()


# -------------------------------------------------- connected components


def _canonical(lab):
    """Relabel a partition so each component carries its smallest linear
    index + 1 (background 0)."""
    out = np.zeros(lab.shape, np.int64)
    flat = lab.ravel()
    idx = np.arange(flat.size)
    n = int(flat.max()) if flat.size else 0
    first = np.full(n + 1, np.iinfo(np.int64).max)
    np.minimum.at(first, flat, idx)
    nz = flat > 0
    out.ravel()[nz] = first[flat[nz]] + 1
    return out.astype(np.int32)


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("p", [0.3, 0.55, 0.8])
def test_ccl_vs_scipy_label(conn, p):
    rng = np.random.default_rng(int(p * 100) + conn)
    img = (rng.random((70, 90)) < p).astype(np.uint8) * 255
    lab, _ = ndi.label(img > 0, structure=refs.footprint(conn))
    assert np.array_equal(oracle.ccl(img, conn), _canonical(lab))


def test_ccl_hand_example():
    # two objects under 4-connectivity that touch only diagonally, one under 8
    img = np.array([[1, 1, 0, 0],
                    [0, 1, 0, 1],
                    [0, 0, 1, 1]], np.uint8)
    assert oracle.ccl(img, 4).tolist() == [[1, 1, 0, 0], [0, 1, 0, 8], [0, 0, 8, 8]]
    assert oracle.ccl(img, 8).tolist() == [[1, 1, 0, 0], [0, 1, 0, 1], [0, 0, 1, 1]]


def test_ccl_snake_and_edges():
    # a one-pixel snake whose smallest index is its far end
    img = np.zeros((9, 9), np.uint8)
    img[0, 8] = img[1:, 8].any()
    img[:, 8] = 1
    img[8, :] = 1
    img[2:, 0] = 1
    lab = oracle.ccl(img, 4)
    assert set(np.unique(lab)) == {0, 9}
    assert (oracle.ccl(np.zeros((3, 3), np.uint8), 8) == 0).all()
    assert (oracle.ccl(np.ones((3, 3), np.uint8), 4) == 1).all()


# ----------------------------------------------------------- area threshold


@pytest.mark.parametrize("lo,hi", [(0, 10 ** 9), (5, 40), (1, 1), (3, 3), (50, 20)])
def test_area_threshold_vs_scipy_sums(lo, hi):
    rng = np.random.default_rng(lo + hi)
    img = (rng.random((60, 70)) < 0.45).astype(np.uint8)
    lab = oracle.ccl(img, 8)
    out, areas = oracle.area_threshold(lab, lo, hi)
    ids = np.unique(lab[lab > 0])
    sizes = ndi.sum_labels(np.ones_like(lab), lab, ids)
    assert np.array_equal(areas[ids], sizes.astype(np.int64))
    keep = ids[(sizes >= lo) & (sizes <= hi)]
    assert np.array_equal(out, np.where(np.isin(lab, keep), lab, 0))


def test_area_threshold_bounds_inclusive():
    lab = np.array([[1, 1, 0, 4], [0, 0, 0, 4], [9, 0, 0, 4]], np.int32)
    assert oracle.area_threshold(lab, 2, 3)[0].tolist() == [[1, 1, 0, 4], [0, 0, 0, 4],
                                                             [0, 0, 0, 4]]
    assert oracle.area_threshold(lab, 1, 2)[0].tolist() == [[1, 1, 0, 0], [0, 0, 0, 0],
                                                             [9, 0, 0, 0]]


# ------------------------------------------------- h-dome, regional maxima


def _brute_regional_maxima(f, conn):
    """Plateaus (equal-valued components) with no higher neighbour."""
    out = np.zeros(f.shape, np.uint8)
    fp = refs.footprint(conn)
    for v in np.unique(f):
        lab, n = ndi.label(f == v, structure=fp)
        for k in range(1, n + 1):
            comp = lab == k
            ring = ndi.binary_dilation(comp, structure=fp) & ~comp
            if not ring.any() or f[ring].max() < v:
                out[comp] = 255
    return out


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("dt", [np.uint8, np.int32])
@pytest.mark.parametrize("seed", range(3))
def test_regional_maxima_vs_plateaus(conn, dt, seed):
    rng = np.random.default_rng(seed * 10 + conn)
    f = rng.integers(0, 5, (17, 23)).astype(dt)
    if dt == np.int32:
        f = (f.astype(np.int64) * 1_000_000_000 - 2_000_000_000).astype(np.int32)
    assert np.array_equal(oracle.regional_maxima(f, conn), _brute_regional_maxima(f, conn))


def test_regional_maxima_constant_images():
    for v in (0, 7, 255):
        f = np.full((5, 6), v, np.uint8)
        assert (oracle.regional_maxima(f, 8) == 255).all()
    f = np.full((5, 6), np.iinfo(np.int32).min, np.int32)
    assert (oracle.regional_maxima(f, 4) == 255).all()


def test_hdome_hand_example():
    # f = 10 50 20 80 20, h = 30: the marker 0 20 0 50 0 rises to
    # 10 20 20 50 20 under f (the right peak's 50 is held at 20 by the saddle),
    # so both domes are cut at h: 0 30 0 30 0
    f = np.array([[10, 50, 20, 80, 20]], np.uint8)
    assert oracle.hdome(f, 30, 4).tolist() == [[0, 30, 0, 30, 0]]
    assert oracle.hdome(f, 5, 8).tolist() == [[0, 5, 0, 5, 0]]


@pytest.mark.parametrize("conn", [4, 8])
@pytest.mark.parametrize("h", [0, 1, 17, 300])
def test_hdome_vs_widest_path(conn, h):
    rng = np.random.default_rng(h + conn)
    f = ndi.uniform_filter(rng.integers(0, 256, (30, 40)).astype(float), 3).astype(np.uint8)
    marker = np.maximum(f.astype(np.int64) - h, 0).astype(np.uint8)
    R = refs.widest_path(marker, f, conn)
    got = oracle.hdome(f, h, conn)
    assert np.array_equal(got, (f.astype(int) - R.astype(int)).astype(np.uint8))
    assert got.min() >= 0 and got.max() <= h
    if h == 0:
        assert (got == 0).all()
    if h >= 255:
        assert np.array_equal(got, f)


# ------------------------------------------------ planted mistakes are caught

def _ops_battery(plant):
    """True if some pin above fails on the planted oracle."""
    rng = np.random.default_rng(0)

    def rgb():
        prim = np.array([[[255, 0, 0], [0, 255, 0], [0, 0, 255]]], np.uint8)
        return oracle.rgb2gray(prim, plant=plant).tolist() == [[76, 150, 29]]

    def disk():
        f = np.full((31, 31), 255, np.uint8)
        f[15, 15] = 0
        return int((oracle.erode_disk13(f, plant=plant) == 0).sum()) == 113

    def dt():
        img = (rng.random((23, 31)) < 0.85).astype(np.uint8)
        return all(np.array_equal(oracle.distance_transform(img, c, plant=plant),
                                  ndi.distance_transform_cdt(img, metric=m))
                   for c, m in ((8, "chessboard"), (4, "taxicab")))

    def ccl():
        img = (rng.random((40, 50)) < 0.5).astype(np.uint8)
        ok = True
        for c in (4, 8):
            lab, _ = ndi.label(img > 0, structure=refs.footprint(c))
            ok &= np.array_equal(oracle.ccl(img, c, plant=plant), _canonical(lab))
        return ok

    def area():
        lab = np.array([[1, 1, 0, 4], [0, 0, 0, 4], [9, 0, 0, 4]], np.int32)
        return oracle.area_threshold(lab, 2, 3, plant=plant)[0].tolist() == \
            [[1, 1, 0, 4], [0, 0, 0, 4], [0, 0, 0, 4]]

    def hdome():
        # a peak of 5 below h keeps its whole height; the peak of 80 over a
        # saddle of 0 is cut at h = 30
        f = np.array([[0, 5, 0, 80, 20]], np.uint8)
        want = np.array([[0, 5, 0, 30, 0]], np.uint8)
        return np.array_equal(oracle.hdome(f, 30, 4, plant=plant), want)

    def rmax():
        f = rng.integers(0, 4, (15, 17)).astype(np.uint8)
        return np.array_equal(oracle.regional_maxima(f, 8, plant=plant),
                              _brute_regional_maxima(f, 8))

    checks = [rgb, disk, dt, ccl, area, hdome, rmax]
    return not all(c() for c in checks)


@pytest.mark.parametrize("plant", [101, 102, 103, 104, 105, 201, 202])
def test_planted_ops_mistakes_are_caught(plant):
    """Red and blue weights swapped; the disk's rim left out; diagonal
    neighbours dropped from the distance transform; the larger root winning a
    union; the area range open at its lower end; the h-dome marker wrapping
    around instead of saturating; regional maxima taken as domes of height 2."""
    if 100 <= plant < 200:
        oracle.build(plant=plant, force=True)
    assert _ops_battery(plant), f"planted mistake {plant} slipped through every pin"


def test_clean_ops_oracle_passes_battery():
    assert not _ops_battery(0)
