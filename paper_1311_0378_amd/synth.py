"""Seeded synthetic inputs for grayscale reconstruction and fill-holes.

This module only draws inputs. It holds none of the reconstruction's
arithmetic, so the CPU oracle and the GPU engine can both be fed from it
without sharing any of the method.

The images stand in for the paper's whole-slide brain-tumour tiles (Sec. V,
experimental setup: 4K x 4K tiles), which are not available. They imitate the
structure that matters to a flood-fill: a smooth, low, noisy background with
bright compact blobs (nuclei), some of them hollow rings that enclose holes.

Recipe for ``make_tile(H, W, n_disks, seed, dtype, hollow_frac)``:

1. ``rng = numpy.random.default_rng(seed)``.
2. ``noise = rng.uniform(0, 80, (H, W))`` in float64.
3. ``f = gaussian_filter(noise, sigma=4, mode='reflect', truncate=4.0)``
   (computed in row bands on threads; bit-identical to the one-shot call).
4. Vectors drawn in this order: ``cy, cx`` (integers in [0,H) and [0,W)),
   ``r`` in [5, 15], ``v`` in [150, 250], ``hollow = rng.random(n) < frac``,
   ring width ``w`` in [2, 4].
5. Disk k is painted in order, overwriting ``f`` where
   ``(y-cy)^2 + (x-cx)^2 <= r^2``; a hollow disk paints only where that
   distance squared is ``> (r-w)^2``.
6. u8 mask ``clip(rint(f), 0, 255)``; i32 mask ``clip(rint(f*65535/255), 0,
   65535)`` from the same field.
7. Marker ``max(mask - 30, 0)`` for u8 and ``max(mask - 7710, 0)`` for i32
   (7710 = 30 * 257).
8. Fill-holes input: ``255`` where the u8 mask is ``>= 128``, else ``0``
   (i32: ``65535`` / ``0``).
9. Reconstruction by erosion (``make_erode_tile``): the same mask, and the
   marker raised instead, ``min(mask + 30, 255)`` for u8 and
   ``min(mask + 7710, 65535)`` for i32.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.ndimage as ndi

SIGMA = 4.0
TRUNCATE = 4.0
_RADIUS = int(TRUNCATE * SIGMA + 0.5)  # half-width of the Gaussian window


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def smooth_field(noise: np.ndarray) -> np.ndarray:
    """Gaussian blur of ``noise`` (axis 0 then axis 1, as gaussian_filter does).

    Row bands overlap by the window radius, so every output sample sees the
    same inputs in the same order as the one-shot filter.
    """
    H, W = noise.shape
    out0 = np.empty_like(noise)
    nb = max(1, min(_threads() * 2, H // 64))
    edges = np.linspace(0, H, nb + 1).astype(np.int64)

    def axis0(i):
        a, b = int(edges[i]), int(edges[i + 1])
        lo, hi = max(0, a - _RADIUS), min(H, b + _RADIUS)
        band = ndi.gaussian_filter1d(noise[lo:hi], SIGMA, axis=0, mode="reflect",
                                     truncate=TRUNCATE)
        out0[a:b] = band[a - lo:b - lo]

    out = np.empty_like(noise)

    def axis1(i):
        a, b = int(edges[i]), int(edges[i + 1])
        out[a:b] = ndi.gaussian_filter1d(out0[a:b], SIGMA, axis=1, mode="reflect",
                                         truncate=TRUNCATE)

    with ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(axis0, range(nb)))
        list(ex.map(axis1, range(nb)))
    return out


def _paint_disks(f: np.ndarray, rng: np.random.Generator, n: int, hollow_frac: float) -> None:
    H, W = f.shape
    cy = rng.integers(0, H, n)
    cx = rng.integers(0, W, n)
    r = rng.integers(5, 16, n)
    v = rng.integers(150, 251, n)
    hollow = rng.random(n) < hollow_frac
    w = rng.integers(2, 5, n)
    for k in range(n):
        rk = int(r[k])
        y0, y1 = max(0, int(cy[k]) - rk), min(H, int(cy[k]) + rk + 1)
        x0, x1 = max(0, int(cx[k]) - rk), min(W, int(cx[k]) + rk + 1)
        yy = (np.arange(y0, y1) - int(cy[k]))[:, None]
        xx = (np.arange(x0, x1) - int(cx[k]))[None, :]
        d2 = yy * yy + xx * xx
        sel = d2 <= rk * rk
        if hollow[k]:
            sel &= d2 > (rk - int(w[k])) ** 2
        f[y0:y1, x0:x1][sel] = float(v[k])


def make_field(H: int, W: int, n_disks: int, seed, hollow_frac: float = 0.0) -> np.ndarray:
    """The float64 tissue-like field (steps 1-5)."""
    rng = np.random.default_rng(seed)
    noise = rng.uniform(0.0, 80.0, (H, W))
    f = smooth_field(noise)
    del noise
    _paint_disks(f, rng, int(n_disks), float(hollow_frac))
    return f


def quantize(f: np.ndarray, dtype: str) -> np.ndarray:
    """Step 6: the mask in the requested pixel type."""
    if dtype == "u8":
        return np.clip(np.rint(f), 0, 255).astype(np.uint8)
    if dtype == "i32":
        return np.clip(np.rint(f * (65535.0 / 255.0)), 0, 65535).astype(np.int32)
    raise ValueError(f"dtype must be 'u8' or 'i32', got {dtype!r}")


def marker_from_mask(mask: np.ndarray) -> np.ndarray:
    """Step 7: the marker is the mask lowered by a fixed offset, floored at 0."""
    off = 30 if mask.dtype == np.uint8 else 7710
    return np.maximum(mask.astype(np.int64) - off, 0).astype(mask.dtype)


def binary_from_mask(mask: np.ndarray) -> np.ndarray:
    """Step 8: the thresholded two-level image fill-holes runs on."""
    if mask.dtype == np.uint8:
        return np.where(mask >= 128, 255, 0).astype(np.uint8)
    return np.where(mask >= 128 * 257, 65535, 0).astype(np.int32)


def make_tile(H: int, W: int, n_disks: int, seed, dtype: str = "u8",
              hollow_frac: float = 0.0):
    """Return ``(marker, mask)`` for one synthetic tile."""
    mask = quantize(make_field(H, W, n_disks, seed, hollow_frac), dtype)
    return marker_from_mask(mask), mask


def erode_marker_from_mask(mask: np.ndarray) -> np.ndarray:
    """Step 9: the erosion marker is the mask raised by the same offset,
    capped at the value range's top."""
    off, top = (30, 255) if mask.dtype == np.uint8 else (7710, 65535)
    return np.minimum(mask.astype(np.int64) + off, top).astype(mask.dtype)


def make_erode_tile(H: int, W: int, n_disks: int, seed, dtype: str = "u8",
                    hollow_frac: float = 0.0):
    """Return ``(marker, mask)`` for reconstruction by erosion."""
    mask = quantize(make_field(H, W, n_disks, seed, hollow_frac), dtype)
    return erode_marker_from_mask(mask), mask


def density_disks(H: int, W: int) -> int:
    """Disk count at 200 disks per 1024 x 1024 pixels."""
    return int(round(200.0 * H * W / float(1 << 20)))


# ---------------------------------------------------------------- workloads

def single_1024():
    """1024 x 1024 u8, 200 disks, seed 0, solid disks (8-connected recon)."""
    return make_tile(1024, 1024, 200, 0, "u8", 0.0)


def single_4096():
    """4096 x 4096 u8, 800 disks, seed 0, 5 % hollow rings.

    Returns ``(marker, mask, binary)``; ``binary`` is the fill-holes input."""
    mask = quantize(make_field(4096, 4096, 800, 0, 0.05), "u8")
    return marker_from_mask(mask), mask, binary_from_mask(mask)


def single_16384(dtype: str = "u8"):
    """16384 x 16384, 12 800 disks (the 4096 density x 16), seed 0, solid."""
    return make_tile(16384, 16384, 12800, 0, dtype, 0.0)


def batch_shapes(n: int = 512, lo: int = 256, hi: int = 4096, seed: int = 0):
    """Tile sides drawn log-uniform in [lo, hi], H and W independently."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), (n, 2))
    return [(int(round(math.exp(a))), int(round(math.exp(b)))) for a, b in u]


def batch_tile(i: int, H: int, W: int, n: int = 512, root_seed: int = 0,
               hollow_frac: float = 0.0, dtype: str = "u8"):
    """Tile ``i`` of a batch, seeded by the i-th child of SeedSequence(root)."""
    ss = np.random.SeedSequence(root_seed).spawn(n)[i]
    return make_tile(H, W, density_disks(H, W), ss, dtype, hollow_frac)


def serving_jobs(n: int = 2000, lo: int = 512, hi: int = 8192, seed: int = 1,
                 fill_frac: float = 0.3):
    """Job list for the serving workload: ``[(kind, H, W), ...]``.

    ``kind`` is ``'recon'`` (solid disks) or ``'fill'`` (5 % hollow, binary).
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(math.log(lo), math.log(hi), (n, 2))
    kinds = np.where(rng.random(n) < fill_frac, "fill", "recon")
    return [(str(k), int(round(math.exp(a))), int(round(math.exp(b))))
            for k, (a, b) in zip(kinds, u)]


def serving_banks(side: int = 8192, root_seed: int = 1):
    """The two images serving jobs are windows of, at the batch density:
    ``(marker, mask)`` of a solid-disk field for reconstruction, and the
    binary image of a field with 5 % hollow disks for fill-holes."""
    ss = np.random.SeedSequence(root_seed).spawn(2)
    marker, mask = make_tile(side, side, density_disks(side, side), ss[0], "u8", 0.0)
    fmask = quantize(make_field(side, side, density_disks(side, side), ss[1], 0.05), "u8")
    return marker, mask, binary_from_mask(fmask)


def serving_windows(jobs, side: int = 8192, seed: int = 3, align: int = 64):
    """Top-left corner of each job's window in its bank: the row uniform over
    the rows where the H x W window fits, the column likewise but rounded
    down to a multiple of ``align`` (tile buffers handed over at aligned
    addresses, as an image reader would)."""
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(0, side - H + 1)),
             int(rng.integers(0, side - W + 1)) // align * align) for _, H, W in jobs]


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 2) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


def rgb_from_mask(mask: np.ndarray) -> np.ndarray:
    """An H x W x 3 uint8 colour image made from a u8 mask of this module, for
    the RGB-to-grayscale workload: the brighter a pixel of the mask (tissue,
    blobs), the darker and bluer the colour, as in stained tissue (background
    near white, blobs purple). Channels, with m the mask value:
    R = 235 - (141 m >> 8), G = 225 - (205 m >> 8), B = 240 - (77 m >> 8),
    clipped to 0..255 (integer arithmetic, deterministic)."""
    m = mask.astype(np.int32)
    r = 235 - ((141 * m) >> 8)
    g = 225 - ((205 * m) >> 8)
    b = 240 - ((77 * m) >> 8)
    return np.clip(np.stack([r, g, b], -1), 0, 255).astype(np.uint8)
