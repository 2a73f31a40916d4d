"""Builds the oracle's C part (``oracle/_direct.so``) with gcc and OpenMP."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(_HERE, "direct.c")
    out = os.path.join(_HERE, "_direct.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
           "-std=c99", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build_asan() -> str:
    """The direct sum and its driver (``asan_check.c``) built with AddressSanitizer
    and UndefinedBehaviorSanitizer into the executable ``_direct_asan``."""
    out = os.path.join(_HERE, "_direct_asan")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-std=c99", "-o", tmp,
           os.path.join(_HERE, "direct.c"), os.path.join(_HERE, "asan_check.c"), "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
