"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU): oracle/sanitize_check.c runs every entry point on seeded random images
of many shapes, down to 1 x 1, with both connectivities; any out-of-bounds
access, use after free, leak, signed overflow or bad shift aborts the run."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_check")
    srcs = [os.path.join(ORACLE, f) for f in ("mro.c", "mro_ops.c", "sanitize_check.c")]
    flags = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    build = subprocess.run(["gcc", *flags, *srcs, "-o", exe], capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("the sanitizer runtimes are not installed")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ok" in run.stdout
