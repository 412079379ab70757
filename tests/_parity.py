"""Per-cell parity metric of the GPU path against the oracle.

err = |x - y| / max(|y|, 1e-3 * max_cells |y_var|) per cell and variable (0 when both are 0):
relative where a variable is not small compared with its own range, absolute at 1e-3 of that
range otherwise (floors and the atmosphere hold values many decades below the torus)."""
import numpy as np


def rel_err(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    nv = y.shape[0]
    scale = np.abs(y).reshape(nv, -1).max(axis=1)
    den = np.maximum(np.abs(y), 1e-3 * scale.reshape((nv,) + (1,) * (y.ndim - 1)))
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.where(den > 0, np.abs(x - y) / np.where(den > 0, den, 1.0), np.where(x == y, 0.0, np.inf))
    return e


def max_rel_err(x, y):
    return float(rel_err(x, y).max())
