"""Helpers shared by the GPU tests (not the oracle, not the library)."""
import sys

import numpy as np


def announce(msg):
    """Name the case before a GPU step, so a fault can be traced to it."""
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


def rel_max(a, b, scale=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / s) if s > 0 else float(np.abs(a - b).max())


def rms(a):
    a = np.asarray(a, dtype=np.float64)
    return float(np.sqrt(np.mean(a * a)))
