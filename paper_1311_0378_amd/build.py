"""Build libmrecon.so (gfx950) in place with hipcc.

Every source compiles to its own object in parallel, then hipcc links them.
Usage: ``python -m paper_1311_0378_amd.build [--verbose]``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmrecon.so")
SOURCES = ["mr_kernels.hip", "mr_api.hip", "mr_server.hip", "mr_probe.hip", "mr_erode.hip",
           "mr_ops.hip", "mr_ccl.hip", "mr_dt.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    # packed fp32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}: {' '.join(cmd[-3:])}")
    if verbose and res.stderr:
        sys.stderr.write(res.stderr)


def build(verbose: bool = False, extra=()) -> str:
    """Compile every HIP source into ``libmrecon.so`` next to this file."""
    srcs = list(SOURCES)
    with tempfile.TemporaryDirectory(prefix="mrecon_build_") as tmpd:
        objs = [os.path.join(tmpd, s.replace(".hip", ".o")) for s in srcs]
        cmds = [[HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, s), "-o", o]
                for s, o in zip(srcs, objs)]
        jobs = min(len(cmds), max(1, min(8, os.cpu_count() or 1)))
        with ThreadPoolExecutor(jobs) as ex:
            list(ex.map(lambda c: _run(c, verbose), cmds))
        tmp = f"{LIB}.tmp{os.getpid()}"
        _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


def sources_newer_than_lib() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    deps += [os.path.join(HERE, "..", "include", h) for h in ("mr.h", "mr_ops.h")]
    return any(os.path.getmtime(p) > t for p in deps if os.path.exists(p))


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
