"""Build the gfx950 HIP library libusv.so in-tree with hipcc.

Flags: -O3, -ffp-contract=off (the nearest-voxel path must evaluate every FP32/FP64
expression in the order written, host and device alike), packed FP32 instructions
disabled for device code, code object for gfx950 only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libusv.so")
SOURCES = ["runtime.hip", "ingest.hip", "finalize.hip", "segment.hip", "cut.hip", "vnn.hip", "export.hip", "fill.hip", "splat.hip", "pipeline.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-fno-gpu-rdc", "-Wall", "-Wno-unused-function",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + srcs
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass does not know the packed-fp32 target feature and says so; harmless
    noise = ("packed-fp32-ops", "is not a recognized feature", "warning generated", "warnings generated")
    msgs = [ln for ln in (r.stdout + r.stderr).splitlines() if not any(n in ln for n in noise)]
    if r.returncode != 0:
        sys.stderr.write("\n".join(msgs) + "\n")
        raise RuntimeError("hipcc failed building libusv.so")
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    return LIB


def build_host_sanitized(out_path: str) -> str:
    """libusv.so with its host code built with AddressSanitizer and UndefinedBehaviorSanitizer
    (each -fsanitize= applies to the host pass only; the gfx950 code is built as usual):
    for checking the host runtime (argument validation, pose fold, boxes, tables) in a
    process started with clang's sanitizer runtime preloaded."""
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
            "-shared-libasan", "-g"]
    flags = [f if f != "-O3" else "-O1" for f in FLAGS]
    cmd = [HIPCC] + flags + host + ["-o", out_path] + [os.path.join(CSRC, s) for s in SOURCES]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building the sanitized libusv.so")
    return out_path


def asan_runtime() -> str:
    """clang's AddressSanitizer runtime that the sanitized library links against."""
    import glob
    base = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(HIPCC))), "llvm", "lib", "clang")
    hits = sorted(glob.glob(os.path.join(base, "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    if not hits:
        hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("libclang_rt.asan-x86_64.so")
    return hits[-1]


if __name__ == "__main__":
    print(build(verbose=True))
