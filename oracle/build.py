"""Build the CPU oracle shared library with the host compiler.

Test infrastructure only (see oracle.cpp). The flags fix the floating-point
semantics the oracle relies on: no FMA contraction, no fast-math, SSE2
binary64 (the x86-64 default, never x87).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

CXXFLAGS = ["-O2", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-Wall", "-Wextra"]


def build(src=None, out=None, quiet=True):
    """Compile ``src`` (default: oracle.cpp) into ``out`` (default: liboracle.so)."""
    src = src or os.path.join(HERE, "oracle.cpp")
    out = out or LIB
    cmd = ["g++", *CXXFLAGS, "-I", HERE, src, "-o", out + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + " ".join(cmd) + "\n" + res.stderr)
    os.replace(out + ".tmp", out)
    if not quiet:
        print("built", out)
    return out


if __name__ == "__main__":
    build(quiet=False)
    sys.exit(0)
