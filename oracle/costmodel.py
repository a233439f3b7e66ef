"""Cost accounting of Sec. 3.5 and the empirical runtime model of Sec. 4.6.

compression ratio   C_xi = N_uvs / Nbar_xi                (Eq. cost-compression)
workload index      I = Nbar/N_uvs + l_cross N_cross/N_int + l_upd N_upd/N_cell
                                                      (Eq. composite_workload_index)
runtime model       t_rel ~ r + l_cross f + c          (Eq. empirical_runtime_model)
with r = Nbar/N_uvs, f = N_cross/N_int (Eq. normalized_performance_quantities);
the fit is an ordinary least-squares line of t_rel - r against f.
"""
from __future__ import annotations

import numpy as np


def compression_ratio(n_uvs, nbar):
    return n_uvs / nbar


def workload_index(nbar, n_uvs, n_cross, n_int, n_upd=0.0, n_cell=1.0, l_cross=0.0, l_upd=0.0):
    return nbar / n_uvs + l_cross * n_cross / n_int + l_upd * n_upd / n_cell


def fit_runtime_model(nbar, n_cross, t, n_uvs, n_int, t_uvs):
    """Least-squares (l_cross, c, R^2) of t/t_uvs - r = l_cross f + c."""
    r = np.asarray(nbar, float) / n_uvs
    f = np.asarray(n_cross, float) / n_int
    y = np.asarray(t, float) / t_uvs - r
    A = np.column_stack([f, np.ones_like(f)])
    (lam, c), *_ = np.linalg.lstsq(A, y, rcond=None)
    pred = lam * f + c
    ss_res = np.sum((y - pred) ** 2)
    ss_tot = np.sum((y - y.mean()) ** 2)
    return float(lam), float(c), float(1.0 - ss_res / ss_tot)


def model_time(nbar, n_cross, n_uvs, n_int, t_uvs, l_cross, c):
    return (np.asarray(nbar, float) / n_uvs + l_cross * np.asarray(n_cross, float) / n_int + c) * t_uvs


def multilevel_wins(r, r_global, f, l_cross):
    """Eq. multilevel_runtime_criterion: f < (r_global - r) / l_cross."""
    return f < (r_global - r) / l_cross, (r_global - r) / l_cross
