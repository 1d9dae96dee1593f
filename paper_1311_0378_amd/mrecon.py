"""ctypes binding of libmrecon (include/mr.h). Argument marshalling only.

Every function takes and returns torch CUDA tensors; PyTorch provides the
device memory and the stream, and all of the computation runs in the HIP
kernels of ``libmrecon.so``. There is no fallback: if the library is missing
the first call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrecon.so")
ABI_VERSION = 4  # the layout of the structs below (include/mr.h MR_ABI_VERSION)
HEADER = os.path.join(HERE, "..", "include", "mr.h")

MR_U8, MR_I32 = 1, 4
MR_OK, MR_EINVAL, MR_ENOMEM, MR_EHIP, MR_EAGAIN = 0, -1, -2, -3, -4
MR_OP_RECON, MR_OP_FILL = 0, 1
MR_PROBE_ADD, MR_PROBE_CAS = 0, 1
MR_RANDOM_READ, MR_RANDOM_WRITE = 0, 1
MR_JOB_DEVICE = 1

_DTYPES = {torch.uint8: MR_U8, torch.int32: MR_I32}


class MrError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmrecon error {code}: {msg}")
        self.code = code


class Tune(ctypes.Structure):
    _fields_ = [("sweep_rounds", ctypes.c_int32), ("max_sweeps", ctypes.c_int32),
                ("persistent_blocks", ctypes.c_int32), ("converge_rounds", ctypes.c_int32),
                ("tail_rounds", ctypes.c_int32), ("first_sweeps", ctypes.c_int32)]


class Tile(ctypes.Structure):
    _fields_ = [("data_inout", ctypes.c_void_p), ("mask", ctypes.c_void_p),
                ("H", ctypes.c_int64), ("W", ctypes.c_int64), ("pitch", ctypes.c_int64),
                ("op", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("mask", ctypes.c_void_p), ("result", ctypes.c_void_p),
                ("H", ctypes.c_int64), ("W", ctypes.c_int64), ("ld", ctypes.c_int64),
                ("ld_result", ctypes.c_int64), ("op", ctypes.c_int32),
                ("flags", ctypes.c_int32)]


class LaunchTime(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("round", ctypes.c_int32), ("launches", ctypes.c_int32),
                ("ms", ctypes.c_float)]


KIND_NAMES = {0: "tile_round", 1: "seed", 2: "queue", 3: "tile_queue"}


class Counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in
                ("rounds", "tiles", "seeds", "pops", "pushes", "cas_retries", "overflows",
                 "sweeps")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1311_0378_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
        c_int = ctypes.c_int
        L.mr_default_tune.argtypes = [ctypes.POINTER(Tune)]
        L.mr_default_tune.restype = None
        L.mr_workspace_bytes.argtypes = [c_int, i64, i64, c_int, c_int, ctypes.POINTER(Tune)]
        L.mr_workspace_bytes.restype = sz
        L.mr_recon_dilate.argtypes = [vp, vp, i64, i64, i64, c_int, c_int, vp, sz,
                                      ctypes.POINTER(Tune), vp]
        L.mr_recon_dilate.restype = c_int
        L.mr_fill_holes.argtypes = [vp, i64, i64, i64, c_int, c_int, vp, sz,
                                    ctypes.POINTER(Tune), vp]
        L.mr_fill_holes.restype = c_int
        L.mr_recon_dilate_noalloc.argtypes = [vp, vp, i64, i64, i64, c_int, c_int,
                                              ctypes.POINTER(Tune), vp]
        L.mr_recon_dilate_noalloc.restype = c_int
        L.mr_recon_erode_workspace_bytes.argtypes = [i64, i64, i64, c_int, c_int,
                                                     ctypes.POINTER(Tune)]
        L.mr_recon_erode_workspace_bytes.restype = sz
        L.mr_recon_erode.argtypes = [vp, vp, i64, i64, i64, c_int, c_int, vp, sz,
                                     ctypes.POINTER(Tune), vp]
        L.mr_recon_erode.restype = c_int
        L.mr_read_counters.argtypes = [vp, ctypes.POINTER(Counters), vp]
        L.mr_read_counters.restype = c_int
        L.mr_status.argtypes = [vp, vp]
        L.mr_status.restype = c_int
        L.mr_read_round_tiles.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), i32,
                                          ctypes.POINTER(i32), vp]
        L.mr_read_round_tiles.restype = c_int
        TP = ctypes.POINTER(Tile)
        L.mr_batch_workspace_bytes.argtypes = [TP, i32, c_int, c_int, ctypes.POINTER(Tune)]
        L.mr_batch_workspace_bytes.restype = sz
        L.mr_batch.argtypes = [TP, i32, c_int, c_int, vp, sz, ctypes.POINTER(Tune), vp]
        L.mr_batch.restype = c_int
        L.mr_batch_graph_create.argtypes = [TP, i32, c_int, c_int, vp, sz, ctypes.POINTER(Tune),
                                            ctypes.POINTER(vp)]
        L.mr_batch_graph_create.restype = c_int
        L.mr_graph_launch.argtypes = [vp, vp]
        L.mr_graph_launch.restype = c_int
        L.mr_graph_destroy.argtypes = [vp]
        L.mr_graph_destroy.restype = None
        L.mr_autotune_workspace_bytes.argtypes = [TP, i32, c_int, c_int]
        L.mr_autotune_workspace_bytes.restype = sz
        L.mr_autotune.argtypes = [TP, i32, c_int, c_int, vp, sz, vp, ctypes.POINTER(Tune)]
        L.mr_autotune.restype = c_int
        L.mr_server_create.argtypes = [vp, sz, i32, c_int, c_int, vp, ctypes.POINTER(vp)]
        L.mr_server_create.restype = c_int
        L.mr_server_submit.argtypes = [vp, ctypes.POINTER(Job), ctypes.POINTER(ctypes.c_uint64)]
        L.mr_server_submit.restype = c_int
        L.mr_server_step.argtypes = [vp]
        L.mr_server_step.restype = c_int
        L.mr_server_set_rounds_per_step.argtypes = [vp, i32]
        L.mr_server_set_rounds_per_step.restype = c_int
        L.mr_server_poll.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64), i32, ctypes.POINTER(i32)]
        L.mr_server_poll.restype = c_int
        L.mr_server_drain.argtypes = [vp]
        L.mr_server_drain.restype = c_int
        L.mr_server_stats.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(sz)]
        L.mr_server_stats.restype = c_int
        L.mr_server_destroy.argtypes = [vp]
        L.mr_server_destroy.restype = None
        L.mr_timing_enable.argtypes = [c_int]
        L.mr_timing_enable.restype = c_int
        L.mr_timing_collect.argtypes = [ctypes.POINTER(LaunchTime), i32, ctypes.POINTER(i32)]
        L.mr_timing_collect.restype = c_int
        L.mr_probe_atomics.argtypes = [vp, sz, c_int, i32, i32, ctypes.c_uint32, vp]
        L.mr_probe_atomics.restype = c_int
        L.mr_probe_random.argtypes = [vp, sz, vp, sz, c_int, i32, vp, vp]
        L.mr_probe_random.restype = c_int
        L.mr_last_error.argtypes = []
        L.mr_last_error.restype = ctypes.c_char_p
        L.mr_abi_version.argtypes = []
        L.mr_abi_version.restype = c_int
        if L.mr_abi_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {L.mr_abi_version()}, this binding "
                               f"needs {ABI_VERSION}: rebuild with python -m "
                               "paper_1311_0378_amd.build")
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/*.h (mr.h and mr_ops.h)."""
    import glob
    names = set()
    for path in sorted(glob.glob(os.path.join(os.path.dirname(HEADER), "*.h"))):
        text = re.sub(r"/\*.*?\*/", "", open(path).read(), flags=re.S)
        names.update(re.findall(r"\b(mr_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def _check(rc: int):
    if rc != MR_OK:
        raise MrError(rc, lib().mr_last_error().decode())


def default_tune() -> Tune:
    t = Tune()
    lib().mr_default_tune(ctypes.byref(t))
    return t


def make_tune(**kw) -> Tune:
    t = default_tune()
    for k, v in kw.items():
        setattr(t, k, int(v))
    return t


def _tune_ptr(tune):
    if tune is None:
        return None
    if isinstance(tune, dict):
        tune = make_tune(**tune)
    return ctypes.byref(tune)


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _image_args(t: torch.Tensor):
    if t.dim() != 2:
        raise ValueError("images must be 2-D")
    if t.dtype not in _DTYPES:
        raise TypeError(f"pixel type must be uint8 or int32, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError("images must be CUDA (HIP) tensors")
    if t.stride(1) != 1:
        raise ValueError("image rows must be contiguous (stride(1) == 1)")
    H, W = t.shape
    return int(H), int(W), int(t.stride(0)), _DTYPES[t.dtype]


def workspace_bytes(op: int, H: int, W: int, dtype: torch.dtype, conn: int, tune=None) -> int:
    n = lib().mr_workspace_bytes(op, H, W, _DTYPES[dtype], conn, _tune_ptr(tune))
    if n == 0:
        raise MrError(MR_EINVAL, lib().mr_last_error().decode())
    return int(n)


def alloc_workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _call_workspace(nbytes: int, device, stream) -> torch.Tensor:
    """A workspace for one call, made by the binding. It is allocated on the
    current stream; when the call runs on another stream, the caching
    allocator is told so (record_stream) and will not hand the block out
    again until that stream's work on it has finished."""
    ws = alloc_workspace(nbytes, device)
    if stream is not None:
        ws.record_stream(stream)
    return ws


def recon_dilate(marker: torch.Tensor, mask: torch.Tensor, conn: int = 8, tune=None,
                 workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Reconstruction by dilation of ``marker`` under ``mask``, in place in
    ``marker`` (returned). Enqueued on ``stream`` (default: current)."""
    H, W, pitch, t = _image_args(marker)
    if mask.shape != marker.shape or mask.dtype != marker.dtype or mask.stride() != marker.stride():
        raise ValueError("mask must match the marker's shape, dtype and strides")
    if workspace is None:
        workspace = _call_workspace(workspace_bytes(MR_OP_RECON, H, W, marker.dtype, conn, tune),
                                    marker.device, stream)
    _check(lib().mr_recon_dilate(marker.data_ptr(), mask.data_ptr(), H, W, pitch, t, conn,
                                 workspace.data_ptr(), workspace.numel(), _tune_ptr(tune),
                                 _stream_ptr(stream)))
    return marker


def recon_dilate_noalloc(marker: torch.Tensor, mask: torch.Tensor, conn: int = 8, tune=None,
                         stream=None) -> torch.Tensor:
    """Reconstruction by dilation in place in ``marker`` without a workspace:
    the library's per-GPU scratch array serves instead (calls on one GPU must
    not overlap). Nothing is allocated."""
    H, W, pitch, t = _image_args(marker)
    if mask.shape != marker.shape or mask.dtype != marker.dtype or mask.stride() != marker.stride():
        raise ValueError("mask must match the marker's shape, dtype and strides")
    _check(lib().mr_recon_dilate_noalloc(marker.data_ptr(), mask.data_ptr(), H, W, pitch, t, conn,
                                         _tune_ptr(tune), _stream_ptr(stream)))
    return marker


def erode_workspace_bytes(H: int, W: int, pitch: int, dtype: torch.dtype, conn: int,
                          tune=None) -> int:
    n = lib().mr_recon_erode_workspace_bytes(H, W, pitch, _DTYPES[dtype], conn, _tune_ptr(tune))
    if n == 0:
        raise MrError(MR_EINVAL, lib().mr_last_error().decode())
    return int(n)


def recon_erode(marker: torch.Tensor, mask: torch.Tensor, conn: int = 8, tune=None,
                workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Reconstruction by erosion of ``marker`` over ``mask``, in place in
    ``marker`` (returned). Enqueued on ``stream`` (default: current)."""
    H, W, pitch, t = _image_args(marker)
    if mask.shape != marker.shape or mask.dtype != marker.dtype or mask.stride() != marker.stride():
        raise ValueError("mask must match the marker's shape, dtype and strides")
    if workspace is None:
        workspace = _call_workspace(erode_workspace_bytes(H, W, pitch, marker.dtype, conn, tune),
                                    marker.device, stream)
    _check(lib().mr_recon_erode(marker.data_ptr(), mask.data_ptr(), H, W, pitch, t, conn,
                                workspace.data_ptr(), workspace.numel(), _tune_ptr(tune),
                                _stream_ptr(stream)))
    return marker


def fill_holes(img: torch.Tensor, conn: int = 8, tune=None,
               workspace: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Fill-holes of ``img`` in place (returned)."""
    H, W, pitch, t = _image_args(img)
    if workspace is None:
        workspace = _call_workspace(workspace_bytes(MR_OP_FILL, H, W, img.dtype, conn, tune),
                                    img.device, stream)
    _check(lib().mr_fill_holes(img.data_ptr(), H, W, pitch, t, conn, workspace.data_ptr(),
                               workspace.numel(), _tune_ptr(tune), _stream_ptr(stream)))
    return img


def make_tiles(items):
    """``items``: sequence of ``(data, mask, op)`` with ``mask`` None for
    fill-holes. Returns ``(Tile array, n, pixel type, torch dtype)``."""
    items = list(items)
    if not items:
        raise ValueError("empty batch")
    arr = (Tile * len(items))()
    dtype = items[0][0].dtype
    for i, (data, mask, op) in enumerate(items):
        H, W, pitch, t = _image_args(data)
        if data.dtype != dtype:
            raise TypeError("all images of a batch share one pixel type")
        if mask is not None and (mask.shape != data.shape or mask.stride() != data.stride()
                                 or mask.dtype != dtype):
            raise ValueError(f"image {i}: mask must match the data's shape, dtype and strides")
        arr[i] = Tile(data.data_ptr(), mask.data_ptr() if mask is not None else None,
                      H, W, pitch, int(op), 0)
    return arr, len(items), _DTYPES[dtype], dtype


def batch_workspace_bytes(items, conn: int = 8, tune=None) -> int:
    arr, n, t, _ = make_tiles(items)
    nb = lib().mr_batch_workspace_bytes(arr, n, t, conn, _tune_ptr(tune))
    if nb == 0:
        raise MrError(MR_EINVAL, lib().mr_last_error().decode())
    return int(nb)


def batch(items, conn: int = 8, tune=None, workspace: torch.Tensor | None = None, stream=None):
    """Reconstruction / fill-holes of every ``(data, mask, op)`` item in one
    launch sequence; results replace each ``data`` in place."""
    arr, n, t, _ = make_tiles(items)
    dev = items[0][0].device
    if workspace is None:
        workspace = _call_workspace(batch_workspace_bytes(items, conn, tune), dev, stream)
    _check(lib().mr_batch(arr, n, t, conn, workspace.data_ptr(), workspace.numel(),
                          _tune_ptr(tune), _stream_ptr(stream)))
    return workspace


class BatchGraph:
    """A batch captured into a HIP graph; ``launch()`` replays it on the same
    buffers. Needs a tune with sweep_rounds > 0, or with tail_rounds > 0."""

    def __init__(self, items, conn: int = 8, tune=None, workspace: torch.Tensor | None = None):
        arr, n, t, _ = make_tiles(items)
        self.items = list(items)  # keep the tensors alive
        if workspace is None:
            workspace = alloc_workspace(batch_workspace_bytes(items, conn, tune),
                                        items[0][0].device)
        self.workspace = workspace
        h = ctypes.c_void_p()
        _check(lib().mr_batch_graph_create(arr, n, t, conn, workspace.data_ptr(),
                                           workspace.numel(), _tune_ptr(tune), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib().mr_graph_launch(self._h, _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().mr_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_cache_key(items, conn: int) -> str:
    """The autotuner cache's key for a batch: the ABI version (a tune stored by
    a library whose mr_tune differs is not reused), pixel type, connectivity,
    the number of images and the total pixel count, each bucketed to a power
    of 2."""
    dt = "u8" if items[0][0].dtype == torch.uint8 else "i32"
    px = sum(int(a.shape[0]) * int(a.shape[1]) for a, *_ in items)
    return (f"abi{ABI_VERSION}-{dt}-conn{conn}-n{max(len(items), 1).bit_length()}"
            f"-px{max(px, 1).bit_length()}")


def autotune(items, conn: int = 8, stream=None, cache=None) -> Tune:
    """Time candidate tunings of ``batch`` on these items (their data are
    restored) and return the fastest.

    ``cache`` (default: the MR_TUNE_CACHE environment variable, if set) names
    a JSON file of tunes keyed by tune_cache_key: a batch whose key is in it
    takes the stored tune without timing anything, and a newly timed tune is
    added to it."""
    import json
    cache = cache if cache is not None else os.environ.get("MR_TUNE_CACHE")
    key = tune_cache_key(items, conn)
    if cache and os.path.exists(cache):
        with open(cache) as f:
            stored = json.load(f).get(key)
        if stored is not None:
            return make_tune(**stored)
    arr, n, t, _ = make_tiles(items)
    nb = lib().mr_autotune_workspace_bytes(arr, n, t, conn)
    if nb == 0:
        raise MrError(MR_EINVAL, lib().mr_last_error().decode())
    ws = alloc_workspace(int(nb), items[0][0].device)
    out = Tune()
    _check(lib().mr_autotune(arr, n, t, conn, ws.data_ptr(), ws.numel(), _stream_ptr(stream),
                             ctypes.byref(out)))
    if cache:
        entries = {}
        if os.path.exists(cache):
            with open(cache) as f:
                entries = json.load(f)
        entries[key] = {k: int(getattr(out, k)) for k, _ in Tune._fields_}
        tmp = f"{cache}.tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(entries, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return out


def _host_rows(a, dtype):
    """A 2-D host tensor whose rows are unit-stride (a window of a larger
    image is fine), pinned if it is not already."""
    t = torch.as_tensor(a)
    if t.device.type != "cpu" or t.dim() != 2 or t.dtype != dtype:
        raise TypeError(f"job images must be 2-D host arrays of {dtype}")
    if t.stride(1) != 1 or t.stride(0) < t.shape[1]:
        t = t.contiguous()
    if not t.is_pinned():
        t = t.contiguous().pin_memory()
    return t


class Server:
    """Continuous-batching server over a device arena of ``arena_bytes``.

    ``submit`` admits a job from host memory or returns None when it cannot
    be admitted yet; ``step`` launches one tile round over every resident job
    and retires what the round before finished; ``poll`` returns the jobs
    whose results have arrived in host memory."""

    def __init__(self, arena_bytes: int, max_jobs: int = 64, dtype=torch.uint8, conn: int = 8,
                 device="cuda:0", stream=None, rounds_per_step: int | None = None):
        self.dtype = dtype
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        _check(lib().mr_server_create(self.arena.data_ptr(), self.arena.numel(), int(max_jobs),
                                      _DTYPES[dtype], int(conn), _stream_ptr(stream),
                                      ctypes.byref(h)))
        self._h = h
        self.jobs = {}  # id -> (buffers kept alive until done, result)
        if rounds_per_step is not None:
            _check(lib().mr_server_set_rounds_per_step(self._h, int(rounds_per_step)))

    def submit(self, data, mask=None, op=None, out=None):
        """Admit ``data`` (the marker, or for fill-holes the image when
        ``mask`` is None). Host arrays make a host job: ``out`` (pinned host
        memory of the job's shape, unit-stride rows) receives the result; by
        default a pinned buffer is allocated. CUDA tensors make a device job
        (MR_JOB_DEVICE): the result goes to ``out``, a device tensor (by
        default a new one). Returns the job id, or None if there is no room
        right now."""
        if op is None:
            op = MR_OP_RECON if mask is not None else MR_OP_FILL
        if isinstance(data, torch.Tensor) and data.is_cuda:
            return self._submit_device(data, mask, op, out)
        d = _host_rows(data, self.dtype)
        m = _host_rows(mask, self.dtype) if mask is not None else None
        if m is not None and m.shape != d.shape:
            raise ValueError("marker and mask shapes differ")
        if m is not None and m.stride(0) != d.stride(0):  # one row pitch for both
            d, m = (_host_rows(x.contiguous(), self.dtype) for x in (d, m))
        H, W = d.shape
        if out is None:
            out = torch.empty((H, W), dtype=self.dtype, pin_memory=True)
        elif (tuple(out.shape) != (H, W) or out.dtype != self.dtype or out.stride(1) != 1
              or out.stride(0) < W or not out.is_pinned()):
            raise ValueError("out must be pinned, of the job's shape and type, rows unit-stride")
        job = Job(d.data_ptr(), m.data_ptr() if m is not None else None, out.data_ptr(),
                  H, W, d.stride(0), out.stride(0), int(op), 0)
        jid = ctypes.c_uint64()
        rc = lib().mr_server_submit(self._h, ctypes.byref(job), ctypes.byref(jid))
        if rc == MR_EAGAIN:
            return None
        _check(rc)
        self.jobs[jid.value] = (d, m, out)
        return jid.value

    def _submit_device(self, d, m, op, out):
        for x in (d, m, out):
            if x is not None and (not x.is_cuda or x.dim() != 2 or x.dtype != self.dtype
                                  or x.stride(1) != 1 or x.stride(0) < x.shape[1]):
                raise ValueError("device jobs take 2-D CUDA tensors of the server's pixel type "
                                 "with unit-stride rows")
        if m is not None and (m.shape != d.shape or m.stride(0) != d.stride(0)):
            raise ValueError("marker and mask must share shape and row pitch")
        H, W = d.shape
        if out is None:
            out = torch.empty((H, W), dtype=self.dtype, device=d.device)
        elif tuple(out.shape) != (H, W):
            raise ValueError("out must have the job's shape")
        job = Job(d.data_ptr(), m.data_ptr() if m is not None else None, out.data_ptr(),
                  H, W, d.stride(0), out.stride(0), int(op), MR_JOB_DEVICE)
        jid = ctypes.c_uint64()
        rc = lib().mr_server_submit(self._h, ctypes.byref(job), ctypes.byref(jid))
        if rc == MR_EAGAIN:
            return None
        _check(rc)
        self.jobs[jid.value] = (d, m, out)
        return jid.value

    def step(self):
        _check(lib().mr_server_step(self._h))

    def poll(self):
        """[(job id, result tensor)] for the jobs whose results have arrived
        since the last poll."""
        cap = 4096
        buf = (ctypes.c_uint64 * cap)()
        n = ctypes.c_int32()
        _check(lib().mr_server_poll(self._h, buf, cap, ctypes.byref(n)))
        return [(int(buf[i]), self.jobs.pop(int(buf[i]))[2]) for i in range(n.value)]

    def drain(self):
        _check(lib().mr_server_drain(self._h))

    def stats(self):
        r = ctypes.c_int32()
        rounds = ctypes.c_uint64()
        fb = ctypes.c_size_t()
        _check(lib().mr_server_stats(self._h, ctypes.byref(r), ctypes.byref(rounds),
                                     ctypes.byref(fb)))
        return {"resident": r.value, "rounds": rounds.value, "largest_free": fb.value}

    def close(self):
        if self._h:
            lib().mr_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def read_round_tiles(workspace: torch.Tensor, stream=None) -> list:
    """Tile visits per round of the last call that used ``workspace``; the
    last entry is the number of tiles the seed pass started from."""
    cap = 1001
    buf = (ctypes.c_uint32 * cap)()
    n = ctypes.c_int32()
    _check(lib().mr_read_round_tiles(workspace.data_ptr(), buf, cap, ctypes.byref(n),
                                     _stream_ptr(stream)))
    return [int(buf[i]) for i in range(min(cap, n.value + 1))]


TIMING_MODES = {False: 0, True: 1, "launches": 1, "spans": 2}


def timing_enable(on=True) -> None:
    """Time this thread's launches with HIP events on each call's stream:
    ``True``/``"launches"`` brackets every tile-round, seed, queue and
    tile-queue launch; ``"spans"`` brackets each run of consecutive tile rounds
    (no host wait between them) with one pair of events instead; ``False``
    turns timing off."""
    _check(lib().mr_timing_enable(TIMING_MODES[on]))


def timing_collect() -> list:
    """Wait for and return the records as ``(kind, round, ms, launches)``:
    ``round`` is the first tile round a record covers (0 for other kinds) and
    ``launches`` the number of launches it covers."""
    n = ctypes.c_int32()
    cap = 1 << 16
    buf = (LaunchTime * cap)()
    _check(lib().mr_timing_collect(buf, cap, ctypes.byref(n)))
    return [(KIND_NAMES.get(buf[i].kind, str(buf[i].kind)), int(buf[i].round), float(buf[i].ms),
             int(buf[i].launches)) for i in range(min(cap, n.value))]


def status(workspace: torch.Tensor, stream=None) -> None:
    """Wait for ``stream`` and raise MrError (MR_EHIP) if the last call that
    used ``workspace`` gave up before its fixed point (watchdog or ring
    guard); its result is then incomplete."""
    _check(lib().mr_status(workspace.data_ptr(), _stream_ptr(stream)))


def read_counters(workspace: torch.Tensor, stream=None) -> dict:
    """Work counters of the last call that used ``workspace`` (waits for it)."""
    c = Counters()
    _check(lib().mr_read_counters(workspace.data_ptr(), ctypes.byref(c), _stream_ptr(stream)))
    return c.as_dict()


def probe_atomics(words: torch.Tensor, kind: int, per_lane: int, waves: int, seed: int = 0,
                  stream=None) -> None:
    """Enqueue the device atomic-rate probe on ``words`` (a contiguous 32-bit
    device tensor whose length is a power of two): ``waves`` 64-lane waves,
    ``per_lane`` atomics per lane of kind ``MR_PROBE_ADD`` or ``MR_PROBE_CAS``.
    The sum of ``words`` grows by ``waves * 64 * per_lane``."""
    if (words.dtype not in (torch.int32, torch.uint32) or not words.is_contiguous()
            or not words.is_cuda):
        raise TypeError("words must be a contiguous int32 or uint32 device tensor")
    _check(lib().mr_probe_atomics(words.data_ptr(), words.numel(), int(kind), int(per_lane),
                                  int(waves), int(seed) & 0xFFFFFFFF, _stream_ptr(stream)))


def probe_random(words: torch.Tensor, indices: torch.Tensor, kind: int, waves: int,
                 sums: torch.Tensor | None = None, stream=None) -> None:
    """Enqueue the random-access probe: ``indices.numel()`` plain reads
    (``MR_RANDOM_READ``, per-lane wrapping sums into ``sums``, ``waves * 64``
    32-bit words) or writes (``MR_RANDOM_WRITE``, operation i stores i) of
    ``words`` (a contiguous 32-bit device tensor whose length is a power of
    two) at the positions ``indices`` (contiguous 32-bit device tensor) holds,
    taken modulo ``words.numel()``."""
    for name, t in (("words", words), ("indices", indices)) + ((("sums", sums),)
                                                               if sums is not None else ()):
        if (t.dtype not in (torch.int32, torch.uint32) or not t.is_contiguous()
                or not t.is_cuda):
            raise TypeError(f"{name} must be a contiguous int32 or uint32 device tensor")
    if sums is not None and sums.numel() < int(waves) * 64:
        raise ValueError(f"sums holds {sums.numel()} words; the launch writes {int(waves) * 64}")
    _check(lib().mr_probe_random(words.data_ptr(), words.numel(), indices.data_ptr(),
                                 indices.numel(), int(kind), int(waves),
                                 sums.data_ptr() if sums is not None else None,
                                 _stream_ptr(stream)))
