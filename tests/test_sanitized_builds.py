"""AddressSanitizer builds of the host code (no GPU).

* The oracle's C direct sum with its driver (``oracle/asan_check.c``),
  AddressSanitizer + UndefinedBehaviorSanitizer: free space and image blocks,
  with and without leaf coordinates, coincident particles, empty target and
  source sets, invalid arguments.
* The library's host layer (``csrc/vmfmm.cpp``, ``csrc/operators.cpp``) with
  AddressSanitizer on the host side only, driven by ``csrc/host_check.cpp``:
  the context-free entry points (offset table, M2L lists of every cell of
  levels up to 4, operators of every degree) and the argument checks of every
  entry point on a null context.

Each executable prints OK and exits 0 when every call behaved; any
sanitizer report aborts it with a non-zero status.
"""
import os
import subprocess

from oracle import build as oracle_build
from paper_1110_2921_amd import build as lib_build

ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1", OMP_NUM_THREADS="2",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


def test_oracle_direct_sum_under_asan_and_ubsan():
    _run(oracle_build.build_asan())


def test_host_layer_under_asan():
    _run(lib_build.build_host_check())
