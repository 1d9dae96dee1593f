"""Independent routes to the reconstruction result, used to pin the oracle.

None of this shares code with the oracle (a C sequential hybrid) or with the
GPU engine. Each route reaches the same unique result by a different road:

* ``brute_recon``      -- the definition itself: iterate the elementary
                          geodesic dilation min(dilate(J), mask) to a fixed
                          point, with the dilation done by
                          ``scipy.ndimage.grey_dilation``.
* ``brute_recon_batch``-- the same iteration vectorised over a stack of tiny
                          images with numpy shifts (for exhaustive sweeps).
* ``widest_path``      -- the closed form as a max-bottleneck path problem,
                          solved by Dijkstra with a max-heap.
* ``binary_recon``     -- the binary special case: the mask components (by
                          ``scipy.ndimage.label``) that hold a marker pixel.
* ``minmax_fill``      -- fill-holes closed form: the min over paths to the
                          border of the max along the path (Dijkstra).
* ``binary_fill``      -- ``scipy.ndimage.binary_fill_holes``.
* ``brute_erode``      -- reconstruction by erosion from its definition:
                          iterate max(erode(J), mask) to a fixed point with
                          ``scipy.ndimage.grey_erosion`` (no complement).
* ``minimax_path``     -- its closed form: the min over paths of the max of
                          the start value and the mask along the path.
"""
from __future__ import annotations

import heapq
import re

import numpy as np
import scipy.ndimage as ndi

CROSS = np.array([[0, 1, 0], [1, 1, 1], [0, 1, 0]], dtype=bool)
SQUARE = np.ones((3, 3), dtype=bool)


def footprint(conn: int) -> np.ndarray:
    return CROSS if conn == 4 else SQUARE


def minval(dtype) -> int:
    return int(np.iinfo(dtype).min)


def brute_recon(marker: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    J = np.minimum(marker, mask)
    fp = footprint(conn)
    while True:
        D = ndi.grey_dilation(J, footprint=fp, mode="constant", cval=minval(J.dtype))
        Jn = np.minimum(D, mask)
        if np.array_equal(Jn, J):
            return J
        J = Jn


def _shift(a: np.ndarray, dy: int, dx: int, fill) -> np.ndarray:
    """out[..., y, x] = a[..., y+dy, x+dx], ``fill`` outside."""
    out = np.full_like(a, fill)
    H, W = a.shape[-2:]
    ys, yd = (slice(dy, H), slice(0, H - dy)) if dy >= 0 else (slice(0, H + dy), slice(-dy, H))
    xs, xd = (slice(dx, W), slice(0, W - dx)) if dx >= 0 else (slice(0, W + dx), slice(-dx, W))
    out[..., yd, xd] = a[..., ys, xs]
    return out


def brute_recon_batch(marker: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    """Fixed-point iteration over a stack ``(B, H, W)``."""
    offs = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if conn == 8:
        offs += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    lo = minval(mask.dtype)
    J = np.minimum(marker, mask)
    while True:
        D = J.copy()
        for dy, dx in offs:
            np.maximum(D, _shift(J, dy, dx, lo), out=D)
        Jn = np.minimum(D, mask)
        if np.array_equal(Jn, J):
            return J
        J = Jn


def _nbrs(conn: int):
    n = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    if conn == 8:
        n += [(-1, -1), (-1, 1), (1, -1), (1, 1)]
    return n


def widest_path(marker: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    """R(p) = max over q and paths q->p of min(J0(q), min of mask on the path)."""
    H, W = mask.shape
    J0 = np.minimum(marker, mask).astype(np.int64)
    I = mask.astype(np.int64)
    best = J0.copy()
    heap = [(-int(best[y, x]), y, x) for y in range(H) for x in range(W)]
    heapq.heapify(heap)
    nb = _nbrs(conn)
    while heap:
        negd, y, x = heapq.heappop(heap)
        d = -negd
        if d < best[y, x]:
            continue
        for dy, dx in nb:
            yy, xx = y + dy, x + dx
            if 0 <= yy < H and 0 <= xx < W:
                c = min(d, int(I[yy, xx]))
                if c > best[yy, xx]:
                    best[yy, xx] = c
                    heapq.heappush(heap, (-c, yy, xx))
    return best.astype(mask.dtype)


def binary_recon(marker: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    """Binary images in {0, v}: keep the mask components that hold a marker pixel."""
    fg = mask > 0
    lab, _ = ndi.label(fg, structure=footprint(conn))
    keep = np.unique(lab[(marker > 0) & fg])
    keep = keep[keep > 0]
    return np.where(np.isin(lab, keep) & fg, mask, np.zeros_like(mask))


def minmax_fill(img: np.ndarray, conn: int) -> np.ndarray:
    """out(p) = min over paths p->border of the max of img along the path."""
    H, W = img.shape
    f = img.astype(np.int64)
    INF = np.iinfo(np.int64).max
    best = np.full((H, W), INF, dtype=np.int64)
    heap = []
    for y in range(H):
        for x in range(W):
            if y in (0, H - 1) or x in (0, W - 1):
                best[y, x] = f[y, x]
                heap.append((int(f[y, x]), y, x))
    heapq.heapify(heap)
    nb = _nbrs(conn)
    while heap:
        d, y, x = heapq.heappop(heap)
        if d > best[y, x]:
            continue
        for dy, dx in nb:
            yy, xx = y + dy, x + dx
            if 0 <= yy < H and 0 <= xx < W:
                c = max(d, int(f[yy, xx]))
                if c < best[yy, xx]:
                    best[yy, xx] = c
                    heapq.heappush(heap, (c, yy, xx))
    return best.astype(img.dtype)


def binary_fill(img: np.ndarray, conn: int) -> np.ndarray:
    """Binary image in {0, v}: scipy's hole filling with the background flood
    connectivity given by the structuring element."""
    v = img.max() if img.size and img.max() > 0 else 1
    filled = ndi.binary_fill_holes(img > 0, structure=footprint(conn))
    return np.where(filled, np.asarray(v, img.dtype), np.zeros((), img.dtype)).astype(img.dtype)


def geodesic_step(J: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    """One elementary geodesic dilation (used to check the fixed-point property)."""
    D = ndi.grey_dilation(J, footprint=footprint(conn), mode="constant", cval=minval(J.dtype))
    return np.minimum(D, mask)


def load_golden(path: str) -> dict:
    """Parse a golden fixture.

    ``name: value`` lines are metadata; a bare ``name:`` line opens a block of
    whitespace-separated integer rows; ``#`` starts a comment."""
    meta, blocks, cur = {}, {}, None
    with open(path) as fh:
        for raw in fh:
            line = raw.split("#", 1)[0].strip()
            if not line:
                continue
            m = re.fullmatch(r"([A-Za-z_]\w*):\s*(.*)", line)
            if m and m.group(2) == "":
                cur = m.group(1)
                blocks[cur] = []
            elif m:
                meta[m.group(1)] = m.group(2)
                cur = None
            else:
                blocks[cur].append([int(t) for t in line.split()])
    dt = np.uint8 if meta["dtype"] == "u8" else np.int32
    out = dict(meta)
    out["conn"] = int(meta["conn"])
    for k, rows in blocks.items():
        out[k] = np.array(rows, dtype=np.int64).astype(dt)
    return out


def maxval(dtype) -> int:
    return int(np.iinfo(dtype).max)


def brute_erode(marker: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    J = np.maximum(marker, mask)
    fp = footprint(conn)
    while True:
        E = ndi.grey_erosion(J, footprint=fp, mode="constant", cval=maxval(J.dtype))
        Jn = np.maximum(E, mask)
        if np.array_equal(Jn, J):
            return J
        J = Jn


def minimax_path(marker: np.ndarray, mask: np.ndarray, conn: int) -> np.ndarray:
    """E(p) = min over q and paths q->p of max(J0(q), max of mask on the path),
    J0 = max(marker, mask)."""
    H, W = mask.shape
    I = mask.astype(np.int64)
    best = np.maximum(marker, mask).astype(np.int64)
    heap = [(int(best[y, x]), y, x) for y in range(H) for x in range(W)]
    heapq.heapify(heap)
    nb = _nbrs(conn)
    while heap:
        d, y, x = heapq.heappop(heap)
        if d > best[y, x]:
            continue
        for dy, dx in nb:
            yy, xx = y + dy, x + dx
            if 0 <= yy < H and 0 <= xx < W:
                c = max(d, int(I[yy, xx]))
                if c < best[yy, xx]:
                    best[yy, xx] = c
                    heapq.heappush(heap, (c, yy, xx))
    return best.astype(mask.dtype)
