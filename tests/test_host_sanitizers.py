"""Host-side code built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on
the CPU: the serving loop's bookkeeping (image arena, in-order admission) driven by a stub executor
(tests/host/arena_admission_test.cpp), and the curve kernel's column arithmetic, checked for every
width to read only columns inside the row (tests/host/columns_test.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
@pytest.mark.parametrize("name", ["arena_admission_test", "columns_test"])
def test_host_code_under_sanitizers(tmp_path, name):
    exe = tmp_path / name
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "paper_1707_05062_amd", "csrc"),
           os.path.join(HERE, "host", name + ".cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "ok" in out.stdout
