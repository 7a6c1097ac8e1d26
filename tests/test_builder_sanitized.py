"""Host-side memory and undefined-behaviour check of the network builders:
tests/native/builder_check.cpp is compiled with g++ together with the
library's builder.cpp under AddressSanitizer and UndefinedBehaviorSanitizer
and run (every family at several sizes, the DEM front end, invalid inputs).
No device code is involved."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_builders_under_sanitizers(tmp_path):
    exe = str(tmp_path / "builder_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           os.path.join(ROOT, "tests", "native", "builder_check.cpp"),
           os.path.join(ROOT, "paper_2310_10722_amd", "csrc", "builder.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, (run.stdout + run.stderr)[-3000:]
    assert "builder checks passed" in run.stdout
