"""Builds ``libvmfmm.so`` (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: ``python -m paper_1110_2921_amd.build``.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libvmfmm.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]
SOURCES = ["kernels_tree.hip", "kernels_fmm.hip", "kernels_p2p.hip", "kernels_step.hip", "kernels_adjoint.hip",
           "kernels_adaptive.hip", "kernels_m2l_sym.hip",
           "kernels_rbf.hip", "kernels_spectrum.hip",
           "operators.cpp",
           "vmfmm.cpp"]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        objs.append(obj)
        cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # the host pass does not know the device-only feature flag
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln]
        if p.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-L/opt/rocm/lib", "-lhipfft"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def build_host_check() -> str:
    """The host layer (the C ABI driver and the operator generation) built with
    AddressSanitizer, linked with the kernels' objects of the last build() and
    the driver csrc/host_check.cpp, into the executable _build/host_check."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    san = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs, procs = [], []
    for src in ("operators.cpp", "vmfmm.cpp", "host_check.cpp"):
        obj = os.path.join(BUILD_DIR, src + ".asan.o")
        objs.append(obj)
        cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + san + \
              ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed for " + src + ":\n" + out.decode(errors="replace"))
    kernels = [os.path.join(BUILD_DIR, s + ".o") for s in SOURCES if s.endswith(".hip")]
    if not all(os.path.exists(k) for k in kernels):
        build()
    exe = os.path.join(BUILD_DIR, "host_check")
    cmd = [HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-o", exe] + objs + kernels + \
          ["-L/opt/rocm/lib", "-lhipfft"]
    subprocess.run(cmd, check=True)
    return exe


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
