"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import numpy as np


def state_error(gpu_state, oracle_g, oracle_h):
    """max|g_gpu - g_orc| / max|g_orc| over all cells (and the same for h);
    infinite when either side holds a NaN."""
    for a, b, c in zip(gpu_state, oracle_g, oracle_h):
        if not (np.all(np.isfinite(a[0])) and np.all(np.isfinite(a[1])) and np.all(np.isfinite(b))
                and np.all(np.isfinite(c))):
            return float("inf"), float("inf")
    eg = max(float(np.max(np.abs(a[0] - b))) for a, b in zip(gpu_state, oracle_g))
    eh = max(float(np.max(np.abs(a[1] - b))) for a, b in zip(gpu_state, oracle_h))
    sg = max(float(np.max(np.abs(b))) for b in oracle_g)
    sh = max(float(np.max(np.abs(b))) for b in oracle_h)
    return eg / sg, eh / sh


def rel_l2(a, b, vol):
    """Volume-weighted relative L2 difference."""
    return float(np.sqrt(np.sum(vol * (a - b) ** 2) / np.sum(vol * b ** 2)))
