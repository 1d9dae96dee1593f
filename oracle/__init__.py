"""CPU oracle for grayscale reconstruction by dilation, its dual by erosion,
fill-holes, the reconstruction-based h-dome and regional maxima, and the
other segmentation operations of Table II: RGB to grayscale, opening with a
13 x 13 disk, distance transform, connected components labeling and area
threshold.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU product path
never imports, links or runs it, and shares no code with it.

The arithmetic lives in ``mro.c`` (a sequential raster / anti-raster scan
pair followed by a FIFO queue phase; Table II, Algorithm 1, Sec. V-C.2) and
``mro_ops.c`` (plain loop nests for the other operations). This module
compiles them with gcc on first use and calls them through ctypes on
C-contiguous numpy arrays; h-dome and regional maxima compose the
reconstruction with numpy pre- and post-steps here.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "mro.c")
SRC_OPS = os.path.join(_HERE, "mro_ops.c")
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra"]

_lock = threading.Lock()
_libs: dict = {}


class Counts(ctypes.Structure):
    _fields_ = [("passes", ctypes.c_uint64), ("seeds", ctypes.c_uint64),
                ("pops", ctypes.c_uint64), ("pushes", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def lib_path(plant: int = 0) -> str:
    if plant:
        return os.path.join(_HERE, "_plant", f"libmro_plant{plant}.so")
    return os.path.join(_HERE, "libmro.so")


def build(plant: int = 0, force: bool = True) -> str:
    """Compile the oracle (``plant`` > 0 builds a copy with a planted mistake:
    1-99 in the reconstruction, 100 and up in the other operations)."""
    out = lib_path(plant)
    srcs = [SRC, SRC_OPS]
    if (not force and os.path.exists(out)
            and all(os.path.getmtime(out) >= os.path.getmtime(x) for x in srcs)):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = f"{out}.tmp{os.getpid()}"
    cmd = ["gcc", *CFLAGS, f"-DMRO_PLANT={int(plant)}", *srcs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def _lib(plant: int = 0):
    with _lock:
        if plant not in _libs:
            path = build(plant, force=False)
            lib = ctypes.CDLL(path)
            i64, c_int, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
            for name in ("mro_recon_dilate_u8", "mro_recon_dilate_i32", "mro_recon_erode_u8",
                         "mro_recon_erode_i32"):
                fn = getattr(lib, name)
                fn.argtypes = [vp, vp, i64, i64, c_int, ctypes.POINTER(Counts)]
                fn.restype = c_int
            for name in ("mro_fill_holes_u8", "mro_fill_holes_i32"):
                fn = getattr(lib, name)
                fn.argtypes = [vp, i64, i64, c_int, ctypes.POINTER(Counts)]
                fn.restype = c_int
            for name in ("mro_rgb2gray", "mro_erode_disk13_u8", "mro_dilate_disk13_u8",
                         "mro_open_disk13_u8"):
                fn = getattr(lib, name)
                fn.argtypes = [vp, vp, i64, i64]
                fn.restype = c_int
            for name in ("mro_distance_transform", "mro_ccl"):
                fn = getattr(lib, name)
                fn.argtypes = [vp, vp, i64, i64, c_int]
                fn.restype = c_int
            lib.mro_area_threshold.argtypes = [vp, i64, i64, i64, i64, vp]
            lib.mro_area_threshold.restype = c_int
            _libs[plant] = lib
        return _libs[plant]


def _suffix(a: np.ndarray) -> str:
    if a.dtype == np.uint8:
        return "u8"
    if a.dtype == np.int32:
        return "i32"
    raise TypeError(f"oracle supports uint8 and int32 images, got {a.dtype}")


def recon_dilate(marker: np.ndarray, mask: np.ndarray, conn: int = 8, plant: int = 0):
    """Reconstruction by dilation of ``marker`` under ``mask``.

    Returns ``(R, counts)``; the inputs are not modified."""
    if marker.shape != mask.shape or marker.dtype != mask.dtype or marker.ndim != 2:
        raise ValueError("marker and mask must be 2-D arrays of one shape and dtype")
    out = np.ascontiguousarray(marker).copy()
    m = np.ascontiguousarray(mask)
    H, W = out.shape
    c = Counts()
    fn = getattr(_lib(plant), f"mro_recon_dilate_{_suffix(out)}")
    rc = fn(out.ctypes.data, m.ctypes.data, H, W, int(conn), ctypes.byref(c))
    if rc != 0:
        raise ValueError(f"oracle recon_dilate failed with status {rc}")
    return out, c.as_dict()


def recon_erode(marker: np.ndarray, mask: np.ndarray, conn: int = 8, plant: int = 0):
    """Reconstruction by erosion of ``marker`` over ``mask`` (the dual of
    Table II's reconstruction, after Vincent 1993): the greatest image below
    max(marker, mask) stable under J <- max(mask, min of J over the
    neighbourhood). Returns ``(E, counts)``; the inputs are not modified."""
    if marker.shape != mask.shape or marker.dtype != mask.dtype or marker.ndim != 2:
        raise ValueError("marker and mask must be 2-D arrays of one shape and dtype")
    out = np.ascontiguousarray(marker).copy()
    m = np.ascontiguousarray(mask)
    H, W = out.shape
    c = Counts()
    fn = getattr(_lib(plant), f"mro_recon_erode_{_suffix(out)}")
    rc = fn(out.ctypes.data, m.ctypes.data, H, W, int(conn), ctypes.byref(c))
    if rc != 0:
        raise ValueError(f"oracle recon_erode failed with status {rc}")
    return out, c.as_dict()


def fill_holes(img: np.ndarray, conn: int = 8, plant: int = 0):
    """Fill-holes of ``img`` with a ``conn``-connected background flood.

    Returns ``(out, counts)``; the input is not modified."""
    if img.ndim != 2:
        raise ValueError("img must be a 2-D array")
    out = np.ascontiguousarray(img).copy()
    H, W = out.shape
    c = Counts()
    fn = getattr(_lib(plant), f"mro_fill_holes_{_suffix(out)}")
    rc = fn(out.ctypes.data, H, W, int(conn), ctypes.byref(c))
    if rc != 0:
        raise ValueError(f"oracle fill_holes failed with status {rc}")
    return out, c.as_dict()


# ------------------------------------------------ reconstruction-based wrappers

def _minmax(dtype):
    info = np.iinfo(dtype)
    return int(info.min), int(info.max)


def hdome(img: np.ndarray, h: int, conn: int = 8, plant: int = 0) -> np.ndarray:
    """h-dome of ``img`` (Vincent 1993, the reconstruction of Table II):
    D_h(f) = f - R(f - h, f), with f - h saturating at the type's minimum.
    Values lie in [0, h]; the result has the input's dtype."""
    if h < 0:
        raise ValueError("h must be >= 0")
    f = np.ascontiguousarray(img)
    lo, _ = _minmax(f.dtype)
    if plant == 201:  # planted mistake: no saturation (the marker wraps around)
        marker = (f.astype(np.int64) - int(h)).astype(f.dtype)
    else:
        marker = np.maximum(f.astype(np.int64) - int(h), lo).astype(f.dtype)
    r, _ = recon_dilate(marker, f, conn, plant if plant < 100 else 0)
    return (f.astype(np.int64) - r.astype(np.int64)).astype(f.dtype)


def regional_maxima(img: np.ndarray, conn: int = 8, plant: int = 0) -> np.ndarray:
    """Regional maxima of ``img`` as a uint8 image, 255 on every pixel of a
    regional maximum (a connected plateau with no higher neighbour) and 0
    elsewhere: the pixels where the dome of height 1, f - R(f - 1, f), is
    positive. f - 1 saturates at the type's minimum, where the dome is 0 even
    on a maximum; a plateau at the minimum that has no higher neighbour is the
    whole image (every pixel is connected to every other), so a constant image
    at the minimum is all maximum."""
    f = np.ascontiguousarray(img)
    lo, _ = _minmax(f.dtype)
    if f.size and int(f.max()) == lo:
        return np.full(f.shape, 255, np.uint8)
    d = hdome(f, 2 if plant == 202 else 1, conn, plant if plant < 100 else 0)  # 202: planted
    return np.where(d > 0, 255, 0).astype(np.uint8)


# ----------------------------------------------------- other Table II operations

def _u8_2d(a, name="img"):
    a = np.ascontiguousarray(a)
    if a.dtype != np.uint8 or a.ndim != 2:
        raise TypeError(f"{name} must be a 2-D uint8 array")
    return a


def rgb2gray(rgb: np.ndarray, plant: int = 0) -> np.ndarray:
    """RGB to grayscale of an H x W x 3 uint8 array (BT.601 weights in 14-bit
    fixed point, rounded half up)."""
    rgb = np.ascontiguousarray(rgb)
    if rgb.dtype != np.uint8 or rgb.ndim != 3 or rgb.shape[2] != 3:
        raise TypeError("rgb must be an H x W x 3 uint8 array")
    H, W, _ = rgb.shape
    out = np.empty((H, W), np.uint8)
    plant = _ops_plant(plant)
    if _lib(plant).mro_rgb2gray(rgb.ctypes.data, out.ctypes.data, H, W) != 0:
        raise ValueError("oracle rgb2gray failed")
    return out


def _ops_plant(plant):
    """Plants 100-199 live in mro_ops.c; others leave it untouched."""
    return plant if 100 <= plant < 200 else 0


def _disk_op(name, img, plant):
    plant = _ops_plant(plant)
    f = _u8_2d(img)
    out = np.empty_like(f)
    if getattr(_lib(plant), name)(f.ctypes.data, out.ctypes.data, *f.shape) != 0:
        raise ValueError(f"oracle {name} failed")
    return out


def erode_disk13(img, plant: int = 0):
    """Flat erosion by the radius-6 disk (13 x 13 box), outside ignored."""
    return _disk_op("mro_erode_disk13_u8", img, plant)


def dilate_disk13(img, plant: int = 0):
    """Flat dilation by the radius-6 disk (13 x 13 box), outside ignored."""
    return _disk_op("mro_dilate_disk13_u8", img, plant)


def open_disk13(img, plant: int = 0):
    """Morphological opening by the radius-6 disk: dilation of the erosion."""
    return _disk_op("mro_open_disk13_u8", img, plant)


def distance_transform(img: np.ndarray, conn: int = 8, plant: int = 0) -> np.ndarray:
    """Distance of every pixel to the nearest background (zero) pixel in
    G-steps (8: chessboard, 4: city block), int32; -1 everywhere when the image
    has no background pixel."""
    f = _u8_2d(img)
    out = np.empty(f.shape, np.int32)
    plant = _ops_plant(plant)
    if _lib(plant).mro_distance_transform(f.ctypes.data, out.ctypes.data, *f.shape,
                                          int(conn)) != 0:
        raise ValueError("oracle distance_transform failed")
    return out


def ccl(img: np.ndarray, conn: int = 8, plant: int = 0) -> np.ndarray:
    """Connected components of the nonzero pixels, int32 labels: 0 for the
    background, smallest linear index of the component + 1 elsewhere."""
    f = _u8_2d(img)
    out = np.empty(f.shape, np.int32)
    plant = _ops_plant(plant)
    if _lib(plant).mro_ccl(f.ctypes.data, out.ctypes.data, *f.shape, int(conn)) != 0:
        raise ValueError("oracle ccl failed")
    return out


def area_threshold(labels: np.ndarray, min_area: int, max_area: int, plant: int = 0):
    """Zero every component of ``labels`` (as ccl writes them) whose pixel
    count is outside [min_area, max_area]. Returns (labels, areas) with
    areas[l] the count of label l."""
    lab = np.ascontiguousarray(labels).copy()
    if lab.dtype != np.int32 or lab.ndim != 2:
        raise TypeError("labels must be a 2-D int32 array")
    H, W = lab.shape
    areas = np.zeros(H * W + 1, np.int64)
    plant = _ops_plant(plant)
    if _lib(plant).mro_area_threshold(lab.ctypes.data, H, W, int(min_area), int(max_area),
                                      areas.ctypes.data) != 0:
        raise ValueError("oracle area_threshold failed")
    return lab, areas
