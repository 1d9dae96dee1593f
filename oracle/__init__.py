"""CPU oracle for grayscale reconstruction by dilation, its dual by erosion,
and fill-holes.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package. The GPU product path
never imports, links or runs it, and shares no code with it.

The arithmetic lives in ``mro.c`` (a sequential raster / anti-raster scan
pair followed by a FIFO queue phase; Table II, Algorithm 1, Sec. V-C.2). This
module compiles it with gcc on first use and calls it through ctypes on
C-contiguous numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "mro.c")
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
    """Compile the oracle (``plant`` > 0 builds a copy with a planted mistake)."""
    out = lib_path(plant)
    if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
        return out
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = f"{out}.tmp{os.getpid()}"
    cmd = ["gcc", *CFLAGS, f"-DMRO_PLANT={int(plant)}", SRC, "-o", tmp]
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
