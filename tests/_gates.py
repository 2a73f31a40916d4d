"""Error measures and gates of the parity tests.

``rel``    relative L2 error over all particles and components;
``worst``  the largest per-particle error (Euclidean norm over that particle's
           components) divided by the largest per-particle reference norm.
           One wrong leaf among thousands barely moves the L2 norm at full
           size but shows here at its own magnitude.
``close``  asserts both, printing the measured values next to their gates.

Gates shared by the FMM parity tests:
* FP64 GPU against the oracle FMM of the same definition: 1e-10 in both
  measures (the two differ by round-off, measured 1e-15 .. 1e-13);
* mixed (FP32 near field with compensated sums, FP32 MFMA expansions)
  against FP64: u 1e-5 L2 / 4e-5 worst; J and dalpha/dt 1e-4 / 4e-4.
"""
import numpy as np

FP64 = (1e-10, 1e-10)
MIXED_U = (1e-5, 4e-5)
MIXED_J = (1e-4, 4e-4)


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def worst(a, b):
    a = np.asarray(a, np.float64).reshape(len(a), -1)
    b = np.asarray(b, np.float64).reshape(len(b), -1)
    return float(np.linalg.norm(a - b, axis=1).max() / np.linalg.norm(b, axis=1).max())


def close(a, b, gates, what=""):
    l2, mx = gates
    e, m = rel(a, b), worst(a, b)
    print(f"[parity] {what}: rel-L2 {e:.2e} (gate {l2:.0e}), worst particle {m:.2e} (gate {mx:.0e})", flush=True)
    assert e < l2 and m < mx, (what, e, m)
