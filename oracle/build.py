"""Compile the C oracle (test infrastructure) into oracle/_build/liborc.so with gcc.

Flags: -O2 -ffp-contract=off -fno-fast-math so that every floating-point expression
is evaluated in the order written (no FMA contraction); -fopenmp for the multi-thread
schedule of the N-core CPU baseline (the single-thread functions use no threads).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "usv_oracle.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liborc.so")


def build(force: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True))


def build_sanitized(out_path: str) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer (gcc): every
    out-of-bounds access, use after free or undefined operation aborts.  Loaded by a
    process started with the sanitizer runtime preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
           "-fopenmp", "-fPIC", "-shared", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-o", out_path, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path
