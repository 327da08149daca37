"""Build libtnc.so for gfx950 with hipcc (in-tree, no JIT cache)."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libtnc.so")
SOURCES = ["kernels.hip", "gemm.hip", "mlp.hip", "codec.hip", "planner.cpp", "simplify.cpp", "engine.cpp", "contract.cpp",
           "search.cpp", "codec.cpp", "postselect.hip", "postselect.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # never form packed FP32 ops (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


# the codec takes its integer decisions, and the post-selection its
# probabilities, with every operation rounded on its own: no contraction into
# fused multiply-adds there
EXTRA = {"codec.hip": ["-ffp-contract=off"], "postselect.hip": ["-ffp-contract=off"]}


def _compile(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(BUILD, src + ".o")
    lang = [] if src.endswith(".hip") else ["-x", "hip"]
    cmd = [HIPCC] + FLAGS + EXTRA.get(src, []) + lang + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, LIB)
    return LIB


# Host-code sanitizer build (address + undefined behaviour) for the CPU tests:
# host objects only (--offload-host-only: no device code, so nothing in it can
# launch a kernel), each sanitizer flag bound to the host compiler.
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_DIR = os.path.join(BUILD, "sanitize")
SAN_LIB = os.path.join(SAN_DIR, "libtnc_san.so")


def _compile_san(src: str) -> str:
    path = os.path.join(CSRC, src)
    obj = os.path.join(SAN_DIR, src + ".o")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Wno-unused-result", "-Wno-unused-value"]
    cmd = [HIPCC] + flags + SAN + EXTRA.get(src, []) + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"sanitizer build failed on {src}")
    return obj


def build_sanitized(jobs: int = 8) -> str:
    """libtnc_san.so: the host code under AddressSanitizer and UBSan, for
    running the host-only entry points (network, search, analysis) on the
    CPU with the sanitizer runtime preloaded."""
    os.makedirs(SAN_DIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(jobs, len(SOURCES))) as ex:
        objs = list(ex.map(_compile_san, SOURCES))
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + SAN + ["-Xarch_host", "-shared-libsan", "-o",
                                                                       SAN_LIB] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("sanitizer link failed")
    return SAN_LIB


def sanitizer_runtime() -> str:
    """Path of the clang AddressSanitizer runtime that must be preloaded."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "sanitize":
        print(build_sanitized())
    else:
        print(build())
