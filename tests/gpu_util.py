"""Helpers for the GPU parity tests (run through the C ABI)."""
import sys

import numpy as np
import pytest


def require_gpu():
    try:
        import torch
    except Exception:  # pragma: no cover
        pytest.skip("torch missing")
    if not torch.cuda.is_available():
        pytest.fail("GPU test selected but no GPU is visible")


def announce(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def rel_l2(x, ref):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    d = np.linalg.norm(ref)
    return float(np.linalg.norm(x - ref) / (d if d > 0 else 1.0))


def interior_rel_l2(x, ref, band):
    """rel-L2 over nodes at least `band` nodes from every grid end."""
    sl = tuple(slice(band, n - band) for n in np.shape(ref))
    return rel_l2(np.asarray(x)[sl], np.asarray(ref)[sl])
