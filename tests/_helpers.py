"""Shared helpers for the GPU parity tests."""
import sys

import numpy as np


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    n = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((got - ref).ravel()) / (n if n > 0 else 1.0))


def say(*a):
    """Name the case before a GPU step (flushed, so it survives a crash of the process)."""
    print(*a, file=sys.stderr, flush=True)


# Parity bars: FP32 projections 1e-5 relative L2, FP32 backprojections 1e-4 (vs the FP64 oracle).
TOL_PROJ = 1e-5
TOL_BP = 1e-4
