"""The GEMM dispatcher's host-side launch guards, on the CPU.

A small C++ program (tests/host/launch_guards.cpp) links the in-tree library
and calls its dispatcher with a split-K partial-sum buffer smaller than the
launch needs, with more slices than the buffer was sized for, with a shape
the kernel cannot run and without scale bookkeeping: each must be refused
with TNC_EINVAL before anything is launched (no GPU is needed or used)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2407_00769_amd")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(os.path.join(PKG, "libtnc.so")), reason="libtnc.so not built")
def test_launch_guards_fire_before_any_launch(tmp_path):
    exe = str(tmp_path / "launch_guards")
    cmd = [HIPCC, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", "-Wno-unused-result",
           "-I", os.path.join(PKG, "csrc"), os.path.join(ROOT, "tests", "host", "launch_guards.cpp"),
           "-L", PKG, "-ltnc", "-Wl,-rpath," + PKG, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        pytest.skip("could not build the guard program: " + r.stderr[-400:])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count("ok ") == 4, r.stdout
