"""The allocation-free reconstruction entry point (mr_recon_dilate_noalloc)
against the workspace entry point (mr_recon_dilate), called through the C
ABI: two calls in a row on the library's per-GPU scratch, the second on a
smaller image, each compared element by element with the result of
mr_recon_dilate on the same input (integer data: tolerance 0). Also the
size limit and the schedule restriction, which fail before anything runs."""
import ctypes

import numpy as np
import pytest

from paper_1311_0378_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from gpu_util import DEV, first_mismatch  # noqa: E402
from paper_1311_0378_amd import mrecon  # noqa: E402


def _with_workspace(marker, mask, conn, tune):
    L = mrecon.lib()
    m = marker.clone()
    H, W = m.shape
    t = mrecon._DTYPES[m.dtype]
    nb = mrecon.workspace_bytes(mrecon.MR_OP_RECON, H, W, m.dtype, conn, tune)
    ws = mrecon.alloc_workspace(nb, DEV)
    rc = L.mr_recon_dilate(m.data_ptr(), mask.data_ptr(), H, W, m.stride(0), t, conn,
                           ws.data_ptr(), nb, mrecon._tune_ptr(tune), None)
    assert rc == mrecon.MR_OK, L.mr_last_error()
    torch.cuda.synchronize()
    return m


def _noalloc(marker, mask, conn, tune):
    L = mrecon.lib()
    m = marker.clone()
    H, W = m.shape
    t = mrecon._DTYPES[m.dtype]
    torch.cuda.synchronize()
    rc = L.mr_recon_dilate_noalloc(m.data_ptr(), mask.data_ptr(), H, W, m.stride(0), t, conn,
                                   mrecon._tune_ptr(tune), None)
    assert rc == mrecon.MR_OK, L.mr_last_error()
    torch.cuda.synchronize()
    return m


CASES = [
    ("u8", 8, None),
    ("u8", 4, dict(sweep_rounds=2, max_sweeps=3)),
    ("i32", 8, dict(sweep_rounds=-1, tail_rounds=2)),
]


@pytest.mark.parametrize("dt,conn,tune", CASES, ids=lambda c: str(c))
def test_noalloc_matches_workspace_entry_two_calls(dt, conn, tune):
    # first a large image (it fills most of the scratch), then a smaller one
    # on the scratch the first call left behind
    for (H, W, n, seed) in [(2900, 3100, 1700, 31), (257, 389, 20, 32)]:
        mk, ms = synth.make_tile(H, W, n, seed, dt, 0.05)
        marker = torch.from_numpy(mk).to(DEV)
        mask = torch.from_numpy(ms).to(DEV)
        print(f"[gpu] noalloc {dt} conn{conn} tune={tune} {H}x{W}", flush=True)
        want = _with_workspace(marker, mask, conn, tune).cpu().numpy()
        got = _noalloc(marker, mask, conn, tune).cpu().numpy()
        assert np.array_equal(got, want), f"{H}x{W}: " + first_mismatch(got, want)


def test_noalloc_full_size_16384():
    # the largest image class the scratch is stated to hold
    mk, ms = synth.single_16384("u8")
    marker = torch.from_numpy(mk).to(DEV)
    mask = torch.from_numpy(ms).to(DEV)
    print("[gpu] noalloc 16384x16384 u8 conn8", flush=True)
    want = _with_workspace(marker, mask, 8, None)
    got = _noalloc(marker, mask, 8, None)
    assert torch.equal(got, want)


def test_noalloc_rejects_before_running():
    L = mrecon.lib()
    x = torch.zeros((64, 64), dtype=torch.uint8, device=DEV)
    # converge mode polls through host words it allocates
    tune = mrecon.make_tune(sweep_rounds=-1, tail_rounds=0)
    rc = L.mr_recon_dilate_noalloc(x.data_ptr(), x.data_ptr(), 64, 64, 64, 1, 8,
                                   ctypes.byref(tune), None)
    assert rc == mrecon.MR_EINVAL and b"converge" in L.mr_last_error()
    # an image whose workspace exceeds the scratch (never dereferenced)
    rc = L.mr_recon_dilate_noalloc(x.data_ptr(), x.data_ptr(), 40000, 40000, 40000, 1, 8, None,
                                   None)
    assert rc == mrecon.MR_ENOMEM and b"scratch" in L.mr_last_error()
    assert bool((x == 0).all())
