"""Helpers shared by the GPU tests: move arrays through the HIP path."""
from __future__ import annotations

import numpy as np
import torch

from paper_1311_0378_amd import mrecon

DEV = "cuda:0"
_TORCH = {np.dtype(np.uint8): torch.uint8, np.dtype(np.int32): torch.int32}


def to_dev(a: np.ndarray, pad: int = 0) -> torch.Tensor:
    """Copy to the GPU; with ``pad`` > 0 the rows get a larger pitch."""
    t = torch.from_numpy(np.ascontiguousarray(a))
    if pad:
        H, W = a.shape
        big = torch.zeros((H, W + pad), dtype=t.dtype)
        big[:, :W] = t
        return big.to(DEV)[:, :W]
    return t.to(DEV)


def gpu_recon(marker: np.ndarray, mask: np.ndarray, conn: int, tune=None, pad: int = 0,
              counters: bool = False):
    m = to_dev(marker, pad)
    k = to_dev(mask, pad)
    ws = mrecon.alloc_workspace(
        mrecon.workspace_bytes(mrecon.MR_OP_RECON, *marker.shape, m.dtype, conn, tune), m.device)
    print(f"[gpu] recon {marker.shape} {marker.dtype} conn{conn} tune={tune} pad={pad}", flush=True)
    mrecon.recon_dilate(m, k, conn, tune=tune, workspace=ws)
    c = mrecon.read_counters(ws)
    out = m.cpu().numpy()
    return (out, c) if counters else out


def gpu_fill(img: np.ndarray, conn: int, tune=None, pad: int = 0, counters: bool = False):
    f = to_dev(img, pad)
    ws = mrecon.alloc_workspace(
        mrecon.workspace_bytes(mrecon.MR_OP_FILL, *img.shape, f.dtype, conn, tune), f.device)
    print(f"[gpu] fill {img.shape} {img.dtype} conn{conn} tune={tune} pad={pad}", flush=True)
    mrecon.fill_holes(f, conn, tune=tune, workspace=ws)
    c = mrecon.read_counters(ws)
    out = f.cpu().numpy()
    return (out, c) if counters else out


def first_mismatch(got: np.ndarray, want: np.ndarray) -> str:
    bad = np.argwhere(got != want)
    if not len(bad):
        return "equal"
    y, x = bad[0]
    return (f"{len(bad)} pixels differ; first at ({y},{x}): got {got[y, x]} want {want[y, x]}")
