"""The library's host planning code (binomial checkpointing schedule and the
snapshot map of its first sweep, stencil z chunking, receiver buckets) built
with g++ under AddressSanitizer and UndefinedBehaviorSanitizer and run on the
CPU. Any out-of-bounds access, use after free, leak, signed overflow or
misaligned access ends the run with an error; tests/host/test_plan.cpp then
checks the plans themselves (schedules executed on symbolic states against a
brute-force minimum, chunk cover, bucket contents and order)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2304_04781_amd", "csrc")
SANITIZE = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
            "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def gxx():
    g = shutil.which("g++")
    if g is None:
        pytest.skip("g++ not available")
    return g


def build(srcs, exe):
    r = subprocess.run([gxx()] + SANITIZE + ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + srcs + ["-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return exe


def test_sanitizers_are_live(tmp_path):
    """A read one element past a vector's end must be reported, so a clean run of
    the planning tests below means something."""
    src = tmp_path / "oob.cpp"
    src.write_text("#include <vector>\nint main(int argc, char**) { std::vector<int> v(4); return v.data()[argc + 3]; }\n")
    exe = build([str(src)], str(tmp_path / "oob"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60, env=ENV)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_host_planning_under_sanitizers(tmp_path):
    srcs = [os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "revolve.cpp"),
            os.path.join(ROOT, "tests", "host", "test_plan.cpp")]
    exe = build(srcs, str(tmp_path / "test_plan"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host planning: ok" in r.stdout
