"""The C ABI on the host: the library loads, exports what include/mr.h
declares, and rejects bad arguments before touching the device."""
import ctypes

import pytest

from paper_1311_0378_amd import mrecon


@pytest.fixture(scope="module")
def L():
    return mrecon.lib()


def test_exports_every_declared_function(L):
    names = mrecon.header_functions()
    assert "mr_recon_dilate" in names and "mr_fill_holes" in names
    for n in names:
        assert hasattr(L, n), f"{n} is declared in include/mr.h but not exported"


def test_abi_version(L):
    assert L.mr_abi_version() == mrecon.ABI_VERSION == 4


def test_default_tune():
    t = mrecon.default_tune()
    assert t.sweep_rounds != 0 and 1 <= t.max_sweeps <= 1024 and t.converge_rounds == 0
    assert 0 <= t.tail_rounds <= 1000 and 1 <= t.first_sweeps <= 1024


def test_workspace_bytes_grows_with_size():
    import torch
    a = mrecon.workspace_bytes(mrecon.MR_OP_RECON, 100, 100, torch.uint8, 8)
    b = mrecon.workspace_bytes(mrecon.MR_OP_RECON, 1000, 1000, torch.uint8, 8)
    f = mrecon.workspace_bytes(mrecon.MR_OP_FILL, 1000, 1000, torch.uint8, 8)
    f32 = mrecon.workspace_bytes(mrecon.MR_OP_FILL, 1000, 1000, torch.int32, 8)
    assert 0 < a < b < f < f32
    assert f - b >= 1000 * 1000  # the fill-holes working plane


@pytest.mark.parametrize("args", [
    (0, 0, 10, 10, 8),      # op, dtype ok ... H/W ok: baseline valid (checked separately)
])
def test_workspace_bytes_valid(L, args):
    op, _, H, W, conn = args
    assert L.mr_workspace_bytes(op, H, W, 1, conn, None) > 0


@pytest.mark.parametrize("op,H,W,t,conn", [
    (2, 10, 10, 1, 8), (0, 0, 10, 1, 8), (0, 10, -1, 1, 8), (0, 10, 10, 2, 8),
    (0, 10, 10, 1, 6), (0, 1 << 20, 1 << 14, 1, 8)])
def test_workspace_bytes_invalid(L, op, H, W, t, conn):
    assert L.mr_workspace_bytes(op, H, W, t, conn, None) == 0
    assert L.mr_last_error()


FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation


def _recon(L, marker=FAKE, mask=FAKE, H=8, W=8, pitch=0, t=1, conn=8, ws=FAKE,
           ws_bytes=1 << 30, tune=None):
    return L.mr_recon_dilate(ctypes.c_void_p(marker), ctypes.c_void_p(mask), H, W, pitch, t,
                             conn, ctypes.c_void_p(ws), ws_bytes, tune, None)


@pytest.mark.parametrize("kw,code", [
    (dict(marker=0), mrecon.MR_EINVAL), (dict(mask=0), mrecon.MR_EINVAL),
    (dict(ws=0), mrecon.MR_EINVAL), (dict(H=0), mrecon.MR_EINVAL), (dict(W=-3), mrecon.MR_EINVAL),
    (dict(pitch=4), mrecon.MR_EINVAL), (dict(conn=6), mrecon.MR_EINVAL),
    (dict(t=2), mrecon.MR_EINVAL), (dict(ws=FAKE + 8), mrecon.MR_EINVAL),
    (dict(t=4, marker=FAKE + 2), mrecon.MR_EINVAL), (dict(ws_bytes=100), mrecon.MR_ENOMEM),
])
def test_recon_rejects(L, kw, code):
    assert _recon(L, **kw) == code
    assert L.mr_last_error()


@pytest.mark.parametrize("field,value", [("sweep_rounds", 0), ("max_sweeps", 0),
                                         ("max_sweeps", 5000), ("persistent_blocks", -1),
                                         ("converge_rounds", -1),
                                         ("converge_rounds", 1001), ("tail_rounds", -1),
                                         ("tail_rounds", 1001), ("first_sweeps", 0),
                                         ("first_sweeps", 1025)])
def test_recon_rejects_bad_tune(L, field, value):
    t = mrecon.default_tune()
    setattr(t, field, value)
    assert _recon(L, tune=ctypes.byref(t)) == mrecon.MR_EINVAL


def test_fill_rejects(L):
    rc = L.mr_fill_holes(ctypes.c_void_p(0), 8, 8, 0, 1, 8, ctypes.c_void_p(FAKE), 1 << 30, None,
                         None)
    assert rc == mrecon.MR_EINVAL
    rc = L.mr_fill_holes(ctypes.c_void_p(FAKE), 8, 8, 0, 1, 8, ctypes.c_void_p(FAKE), 64, None,
                         None)
    assert rc == mrecon.MR_ENOMEM


def test_read_counters_rejects_null(L):
    assert L.mr_read_counters(None, None, None) == mrecon.MR_EINVAL


def _tiles(specs):
    arr = (mrecon.Tile * len(specs))()
    for i, (data, mask, H, W, pitch, op, res) in enumerate(specs):
        arr[i] = mrecon.Tile(data, mask, H, W, pitch, op, res)
    return arr


@pytest.mark.parametrize("spec", [
    (FAKE, 0, 8, 8, 0, 0, 0),        # recon without a mask
    (0, FAKE, 8, 8, 0, 0, 0),        # null data
    (FAKE, FAKE, 0, 8, 0, 0, 0),     # empty image
    (FAKE, FAKE, 8, 8, 4, 0, 0),     # pitch < W
    (FAKE, FAKE, 8, 8, 0, 3, 0),     # unknown op
    (FAKE, FAKE, 8, 8, 0, 0, 1),     # reserved set
])
def test_batch_rejects(L, spec):
    arr = _tiles([(FAKE, FAKE, 16, 16, 0, 0, 0), spec])
    assert L.mr_batch_workspace_bytes(arr, 2, 1, 8, None) == 0
    assert b"tile 1" in L.mr_last_error()
    rc = L.mr_batch(arr, 2, 1, 8, ctypes.c_void_p(FAKE), 1 << 40, None, None)
    assert rc == mrecon.MR_EINVAL


def test_batch_workspace_sizes(L):
    one = _tiles([(FAKE, FAKE, 300, 200, 0, 0, 0)])
    two = _tiles([(FAKE, FAKE, 300, 200, 0, 0, 0), (FAKE, 0, 100, 90, 0, 1, 0)])
    a = L.mr_batch_workspace_bytes(one, 1, 1, 8, None)
    b = L.mr_batch_workspace_bytes(two, 2, 1, 8, None)
    assert 0 < a < b
    assert b - a >= 100 * 128  # the fill image's working plane
    assert L.mr_batch_workspace_bytes(one, 0, 1, 8, None) == 0
    assert L.mr_autotune_workspace_bytes(one, 1, 1, 8) >= a + 300 * 200
    rc = L.mr_batch(one, 1, 1, 8, ctypes.c_void_p(FAKE), a - 256, None, None)
    assert rc == mrecon.MR_ENOMEM


def test_graph_needs_fixed_rounds(L):
    one = _tiles([(FAKE, FAKE, 30, 20, 0, 0, 0)])
    h = ctypes.c_void_p()
    t = mrecon.default_tune()
    t.sweep_rounds = -1
    t.tail_rounds = 0
    rc = L.mr_batch_graph_create(one, 1, 1, 8, ctypes.c_void_p(FAKE), 1 << 30, ctypes.byref(t),
                                 ctypes.byref(h))
    assert rc == mrecon.MR_EINVAL and not h.value


@pytest.mark.parametrize("kw", [dict(arena=0), dict(arena=FAKE + 4), dict(max_jobs=0),
                                dict(t=3), dict(conn=5)])
def test_server_create_rejects(L, kw):
    args = dict(arena=FAKE, size=1 << 30, max_jobs=8, t=1, conn=8)
    args.update(kw)
    h = ctypes.c_void_p()
    rc = L.mr_server_create(ctypes.c_void_p(args["arena"]), args["size"], args["max_jobs"],
                            args["t"], args["conn"], None, ctypes.byref(h))
    assert rc == mrecon.MR_EINVAL and not h.value
    assert L.mr_last_error()


def test_plane_limit(L):
    # H * pitch must stay below 2^32 elements: 65535 x 65535 is accepted,
    # 65536 x 65536 is refused
    n = L.mr_workspace_bytes(mrecon.MR_OP_RECON, 65535, 65535, mrecon.MR_U8, 8, None)
    assert n > 0
    assert L.mr_workspace_bytes(mrecon.MR_OP_RECON, 65536, 65536, mrecon.MR_U8, 8, None) == 0
    assert b"2^32" in L.mr_last_error()


def test_server_rounds_per_step_validation(L):
    assert L.mr_server_set_rounds_per_step(None, 4) == mrecon.MR_EINVAL


@pytest.mark.parametrize("words,n,kind,per_lane,waves", [
    (0, 1 << 16, 0, 1, 1), (FAKE + 2, 1 << 16, 0, 1, 1), (FAKE, 1000, 0, 1, 1),
    (FAKE, 32, 1, 1, 1), (FAKE, (1 << 32) * 2, 0, 1, 1), (FAKE, 1 << 16, 2, 1, 1),
    (FAKE, 1 << 16, 0, 0, 1), (FAKE, 1 << 16, 1, 1 << 17, 1), (FAKE, 1 << 16, 0, 1, 0),
    (FAKE, 1 << 16, 1, 1, (1 << 20) + 1)])
def test_probe_atomics_rejects(L, words, n, kind, per_lane, waves):
    assert L.mr_probe_atomics(ctypes.c_void_p(words), n, kind, per_lane, waves, 0, None) \
        == mrecon.MR_EINVAL
    assert L.mr_last_error().startswith(b"probe:")


@pytest.mark.parametrize("words,n,idx,n_ops,kind,waves,sums", [
    (0, 1 << 16, FAKE, 10, 0, 1, FAKE), (FAKE + 2, 1 << 16, FAKE, 10, 0, 1, FAKE),
    (FAKE, 1000, FAKE, 10, 0, 1, FAKE), (FAKE, 32, FAKE, 10, 1, 1, 0),
    (FAKE, 1 << 16, FAKE, 10, 2, 1, FAKE), (FAKE, 1 << 16, 0, 10, 1, 1, 0),
    (FAKE, 1 << 16, FAKE + 1, 10, 1, 1, 0), (FAKE, 1 << 16, FAKE, 0, 0, 1, FAKE),
    (FAKE, 1 << 16, FAKE, (1 << 34) + 1, 1, 1, 0), (FAKE, 1 << 16, FAKE, 10, 1, 0, 0),
    (FAKE, 1 << 16, FAKE, 10, 0, (1 << 20) + 1, FAKE), (FAKE, 1 << 16, FAKE, 10, 0, 1, 0),
    (FAKE, 1 << 16, FAKE, 10, 0, 1, FAKE + 2)])
def test_probe_random_rejects(L, words, n, idx, n_ops, kind, waves, sums):
    assert L.mr_probe_random(ctypes.c_void_p(words), n, ctypes.c_void_p(idx), n_ops, kind, waves,
                             ctypes.c_void_p(sums), None) == mrecon.MR_EINVAL
    assert L.mr_last_error().startswith(b"probe:")


def test_erode_workspace_bytes():
    import torch
    r = mrecon.workspace_bytes(mrecon.MR_OP_RECON, 100, 100, torch.uint8, 8)
    e = mrecon.erode_workspace_bytes(100, 100, 0, torch.uint8, 8)
    e_pitched = mrecon.erode_workspace_bytes(100, 100, 160, torch.uint8, 8)
    e32 = mrecon.erode_workspace_bytes(100, 100, 0, torch.int32, 8)
    assert e >= r + 100 * 100 and e_pitched >= r + 100 * 160 and e32 >= r + 4 * 100 * 100


@pytest.mark.parametrize("H,W,pitch,t,conn", [
    (0, 10, 0, 1, 8), (10, 10, 5, 1, 8), (10, 10, 0, 2, 8), (10, 10, 0, 1, 6),
    (1 << 20, 1 << 14, 0, 1, 8)])
def test_erode_workspace_bytes_invalid(L, H, W, pitch, t, conn):
    assert L.mr_recon_erode_workspace_bytes(H, W, pitch, t, conn, None) == 0
    assert L.mr_last_error()


def _erode(L, marker=FAKE, mask=FAKE, H=8, W=8, pitch=0, t=1, conn=8, ws=FAKE,
           ws_bytes=1 << 30, tune=None):
    return L.mr_recon_erode(ctypes.c_void_p(marker), ctypes.c_void_p(mask), H, W, pitch, t,
                            conn, ctypes.c_void_p(ws), ws_bytes, tune, None)


@pytest.mark.parametrize("kw,code", [
    (dict(marker=0), mrecon.MR_EINVAL), (dict(mask=0), mrecon.MR_EINVAL),
    (dict(ws=0), mrecon.MR_EINVAL), (dict(H=0), mrecon.MR_EINVAL), (dict(W=-3), mrecon.MR_EINVAL),
    (dict(pitch=4), mrecon.MR_EINVAL), (dict(conn=6), mrecon.MR_EINVAL),
    (dict(t=2), mrecon.MR_EINVAL), (dict(ws=FAKE + 8), mrecon.MR_EINVAL),
    (dict(t=4, marker=FAKE + 2), mrecon.MR_EINVAL), (dict(t=4, mask=FAKE + 1), mrecon.MR_EINVAL),
    (dict(ws_bytes=100), mrecon.MR_ENOMEM),
])
def test_erode_rejects(L, kw, code):
    assert _erode(L, **kw) == code
    assert L.mr_last_error()


def test_status_rejects_null(L):
    assert L.mr_status(None, None) == mrecon.MR_EINVAL
    assert b"null" in L.mr_last_error()


def test_job_struct_layout():
    # mr_job: three pointers, four int64, two int32 (flags last)
    assert ctypes.sizeof(mrecon.Job) == 3 * 8 + 4 * 8 + 2 * 4
    assert mrecon.Job.flags.offset == 3 * 8 + 4 * 8 + 4
    assert mrecon.MR_JOB_DEVICE == 1


def test_default_tune_environment_overrides(monkeypatch):
    base = mrecon.default_tune()
    monkeypatch.setenv("MR_TUNE_TAIL_ROUNDS", "5")
    monkeypatch.setenv("MR_TUNE_FIRST_SWEEPS", "16")
    monkeypatch.setenv("MR_TUNE_MAX_SWEEPS", "0")        # out of range: ignored
    monkeypatch.setenv("MR_TUNE_SWEEP_ROUNDS", "3x")     # not a number: ignored
    t = mrecon.default_tune()
    assert t.tail_rounds == 5 and t.first_sweeps == 16
    assert t.max_sweeps == base.max_sweeps and t.sweep_rounds == base.sweep_rounds
    monkeypatch.delenv("MR_TUNE_TAIL_ROUNDS")
    monkeypatch.delenv("MR_TUNE_FIRST_SWEEPS")
    assert mrecon.default_tune().tail_rounds == base.tail_rounds


def test_autotune_cache_hit_times_nothing(tmp_path):
    # a batch whose key is in the cache takes the stored tune without any
    # device work (these tensors are on the host, which the timing path
    # would reject)
    import json
    import torch
    items = [(torch.zeros(70, 90, dtype=torch.uint8), torch.zeros(70, 90, dtype=torch.uint8),
              mrecon.MR_OP_RECON)] * 3
    key = mrecon.tune_cache_key(items, 8)
    assert key == mrecon.tune_cache_key(items, 8) != mrecon.tune_cache_key(items, 4)
    assert key.startswith(f"abi{mrecon.ABI_VERSION}-u8-conn8-")
    path = tmp_path / "tunes.json"
    path.write_text(json.dumps({key: {"sweep_rounds": -1, "max_sweeps": 3, "tail_rounds": 6,
                                      "first_sweeps": 16}}))
    t = mrecon.autotune(items, 8, cache=str(path))
    assert (t.sweep_rounds, t.max_sweeps, t.tail_rounds, t.first_sweeps) == (-1, 3, 6, 16)
