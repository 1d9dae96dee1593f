"""ctypes binding of the Table II operations in include/mr_ops.h. Argument
marshalling only: every step runs in the HIP kernels of ``libmrecon.so``
(there is no fallback; a missing library raises at the first call).

All functions take and return torch CUDA tensors and enqueue on ``stream``
(default: the current stream). Workspaces the binding allocates are recorded
on that stream.
"""
from __future__ import annotations

import ctypes

import torch

from . import mrecon
from .mrecon import MR_EINVAL, MrError, _check, _stream_ptr, _tune_ptr

MR_DISK_ERODE, MR_DISK_DILATE = 0, 1

_bound = False


def lib():
    """The loaded library with the mr_ops.h signatures set."""
    global _bound
    L = mrecon.lib()
    if not _bound:
        i64, c_int, vp, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t
        TP = ctypes.POINTER(mrecon.Tune)
        L.mr_hdome_workspace_bytes.argtypes = [i64, i64, i64, c_int, c_int, TP]
        L.mr_hdome_workspace_bytes.restype = sz
        L.mr_hdome.argtypes = [vp, i64, i64, i64, c_int, c_int, i64, vp, sz, TP, vp]
        L.mr_hdome.restype = c_int
        L.mr_regional_maxima.argtypes = [vp, vp, i64, i64, i64, i64, c_int, c_int, vp, sz, TP, vp]
        L.mr_regional_maxima.restype = c_int
        L.mr_rgb2gray.argtypes = [vp, i64, vp, i64, i64, i64, vp]
        L.mr_rgb2gray.restype = c_int
        L.mr_open_disk13_workspace_bytes.argtypes = [i64, i64, i64]
        L.mr_open_disk13_workspace_bytes.restype = sz
        L.mr_open_disk13.argtypes = [vp, vp, i64, i64, i64, vp, sz, vp]
        L.mr_open_disk13.restype = c_int
        L.mr_disk13.argtypes = [c_int, vp, vp, i64, i64, i64, vp]
        L.mr_disk13.restype = c_int
        L.mr_distance_transform_workspace_bytes.argtypes = [i64, i64, c_int]
        L.mr_distance_transform_workspace_bytes.restype = sz
        L.mr_distance_transform.argtypes = [vp, vp, i64, i64, i64, i64, c_int, vp, sz, vp]
        L.mr_distance_transform.restype = c_int
        L.mr_ccl_workspace_bytes.argtypes = [i64, i64]
        L.mr_ccl_workspace_bytes.restype = sz
        L.mr_ccl.argtypes = [vp, vp, i64, i64, i64, i64, c_int, vp, sz, vp]
        L.mr_ccl.restype = c_int
        L.mr_area_threshold_workspace_bytes.argtypes = [i64, i64]
        L.mr_area_threshold_workspace_bytes.restype = sz
        L.mr_area_threshold.argtypes = [vp, i64, i64, i64, i64, i64, vp, sz, vp]
        L.mr_area_threshold.restype = c_int
        _bound = True
    return L


def _size(n: int) -> int:
    if n == 0:
        raise MrError(MR_EINVAL, lib().mr_last_error().decode())
    return int(n)


def _ws(nbytes: int, device, stream) -> torch.Tensor:
    return mrecon._call_workspace(nbytes, device, stream)


def _img2d(t: torch.Tensor, dtypes, name="image"):
    if t.dim() != 2 or not t.is_cuda or t.stride(1) != 1:
        raise ValueError(f"{name} must be a 2-D CUDA tensor with unit-stride rows")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must be one of {dtypes}, got {t.dtype}")
    return int(t.shape[0]), int(t.shape[1]), int(t.stride(0))


def hdome_workspace_bytes(H, W, pitch, dtype, conn=8, tune=None) -> int:
    return _size(lib().mr_hdome_workspace_bytes(H, W, pitch, mrecon._DTYPES[dtype], conn,
                                                _tune_ptr(tune)))


def hdome(img: torch.Tensor, h: int, conn: int = 8, tune=None, workspace=None, stream=None):
    """In place: img <- img - R(img - h, img) (the h-dome). Returns img."""
    H, W, p = _img2d(img, (torch.uint8, torch.int32))
    if workspace is None:
        workspace = _ws(hdome_workspace_bytes(H, W, p, img.dtype, conn, tune), img.device, stream)
    _check(lib().mr_hdome(img.data_ptr(), H, W, p, mrecon._DTYPES[img.dtype], conn, int(h),
                          workspace.data_ptr(), workspace.numel(), _tune_ptr(tune),
                          _stream_ptr(stream)))
    return img


def regional_maxima(img: torch.Tensor, conn: int = 8, out=None, tune=None, workspace=None,
                    stream=None) -> torch.Tensor:
    """uint8 image: 255 on the regional maxima of ``img``, 0 elsewhere."""
    H, W, p = _img2d(img, (torch.uint8, torch.int32))
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=img.device)
    _, _, op = _img2d(out, (torch.uint8,), "out")
    if workspace is None:
        workspace = _ws(hdome_workspace_bytes(H, W, p, img.dtype, conn, tune), img.device, stream)
    _check(lib().mr_regional_maxima(img.data_ptr(), out.data_ptr(), H, W, p, op,
                                    mrecon._DTYPES[img.dtype], conn, workspace.data_ptr(),
                                    workspace.numel(), _tune_ptr(tune), _stream_ptr(stream)))
    return out


def rgb2gray(rgb: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """H x W x 3 uint8 (interleaved R, G, B; unit-stride pixels) -> H x W uint8."""
    if rgb.dim() != 3 or rgb.shape[2] != 3 or rgb.dtype != torch.uint8 or not rgb.is_cuda:
        raise TypeError("rgb must be an H x W x 3 uint8 CUDA tensor")
    if rgb.stride(2) != 1 or rgb.stride(1) != 3:
        raise ValueError("rgb pixels must be three consecutive bytes")
    H, W = int(rgb.shape[0]), int(rgb.shape[1])
    if out is None:
        out = torch.empty((H, W), dtype=torch.uint8, device=rgb.device)
    _, _, op = _img2d(out, (torch.uint8,), "out")
    _check(lib().mr_rgb2gray(rgb.data_ptr(), int(rgb.stride(0)), out.data_ptr(), op, H, W,
                             _stream_ptr(stream)))
    return out


def open_disk13(img: torch.Tensor, out=None, workspace=None, stream=None) -> torch.Tensor:
    """Opening of a uint8 image by the radius-6 disk (13 x 13 box)."""
    H, W, p = _img2d(img, (torch.uint8,))
    if out is None:
        out = torch.empty_strided((H, W), (p, 1), dtype=torch.uint8, device=img.device)
    if out.stride(0) != p:
        raise ValueError("out must have the input's row pitch")
    if workspace is None:
        workspace = _ws(_size(lib().mr_open_disk13_workspace_bytes(H, W, p)), img.device, stream)
    _check(lib().mr_open_disk13(img.data_ptr(), out.data_ptr(), H, W, p, workspace.data_ptr(),
                                workspace.numel(), _stream_ptr(stream)))
    return out


def disk13(op: int, img: torch.Tensor, out=None, stream=None) -> torch.Tensor:
    """Flat erosion (MR_DISK_ERODE) or dilation (MR_DISK_DILATE) by the disk."""
    H, W, p = _img2d(img, (torch.uint8,))
    if out is None:
        out = torch.empty_strided((H, W), (p, 1), dtype=torch.uint8, device=img.device)
    if out.stride(0) != p:
        raise ValueError("out must have the input's row pitch")
    _check(lib().mr_disk13(int(op), img.data_ptr(), out.data_ptr(), H, W, p,
                           _stream_ptr(stream)))
    return out


def distance_transform(img: torch.Tensor, conn: int = 8, out=None, workspace=None,
                       stream=None) -> torch.Tensor:
    """int32 distance (G-steps) of every pixel to the nearest zero pixel of
    the uint8 ``img``; -1 everywhere if there is none. Waits for ``stream``
    between batches of rounds."""
    H, W, p = _img2d(img, (torch.uint8,))
    if out is None:
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _, _, dp = _img2d(out, (torch.int32,), "out")
    if workspace is None:
        workspace = _ws(_size(lib().mr_distance_transform_workspace_bytes(H, W, conn)),
                        img.device, stream)
    _check(lib().mr_distance_transform(img.data_ptr(), out.data_ptr(), H, W, p, dp, conn,
                                       workspace.data_ptr(), workspace.numel(),
                                       _stream_ptr(stream)))
    return out


def ccl(img: torch.Tensor, conn: int = 8, out=None, workspace=None, stream=None):
    """int32 labels of the nonzero pixels' components (smallest linear index
    + 1; background 0)."""
    H, W, p = _img2d(img, (torch.uint8,))
    if out is None:
        out = torch.empty((H, W), dtype=torch.int32, device=img.device)
    _, _, lp = _img2d(out, (torch.int32,), "out")
    if workspace is None:
        workspace = _ws(_size(lib().mr_ccl_workspace_bytes(H, W)), img.device, stream)
    _check(lib().mr_ccl(img.data_ptr(), out.data_ptr(), H, W, p, lp, conn, workspace.data_ptr(),
                        workspace.numel(), _stream_ptr(stream)))
    return out


def area_threshold(labels: torch.Tensor, min_area: int, max_area: int, workspace=None,
                   stream=None):
    """In place: zero every label whose pixel count is outside
    [min_area, max_area]. Returns (labels, workspace); the workspace's first
    H * W + 1 int32 hold the per-label areas."""
    H, W, p = _img2d(labels, (torch.int32,), "labels")
    if workspace is None:
        workspace = _ws(_size(lib().mr_area_threshold_workspace_bytes(H, W)), labels.device,
                        stream)
    _check(lib().mr_area_threshold(labels.data_ptr(), H, W, p, int(min_area), int(max_area),
                                   workspace.data_ptr(), workspace.numel(), _stream_ptr(stream)))
    return labels, workspace
