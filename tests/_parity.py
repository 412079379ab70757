"""Per-cell parity metric of the GPU path against the oracle.

For primitive states P = (rho, u, u~1, u~2, u~3, B1, B2, B3):

    err = |x - y| / max(|y|, 1e-3 * S_k)      (0 where x == y)

with S_k the scale of variable k: max|rho| over all cells for rho; for u, the larger of max|u|
over all cells and 10 rho, ten times the local rest-mass energy density (u is recovered from the
energy equation as the difference between the total energy and the rest mass, so its absolute
precision is ~eps rho times the cancellation of the Lax-Friedrichs flux, ~40 at the torus
surface, whatever the implementation: in the cold inner edge of a 256^3 torus, u/rho ~ 3e-4 to
3e-3, two independent FP64 codes differ there by up to ~3e-12 of u); the largest component of the field for every B^i (the
three components are one vector); and for every u~^i the largest velocity component but at least
1 (u~ is a spatial 4-velocity in units of c, so a few ulp of 1 is the rounding limit however
slow the local flow is).  Relative where a quantity is not tiny against its own scale, absolute
at 1e-3 of that scale otherwise: floors and the atmosphere hold values many decades below the
torus, where the inversion is ill-conditioned and no FP64 implementation can fix more digits.

For conserved vectors and fluxes each of the 9 components is its own scale."""
import numpy as np


def _scales(y):
    nv = y.shape[0]
    sc = np.abs(y).reshape(nv, -1).max(axis=1)
    if nv == 8:
        sc[2:5] = max(sc[2:5].max(), 1.0)
        sc[5:8] = sc[5:8].max()
    return sc


def rel_err(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    nv = y.shape[0]
    sc = _scales(y)
    den = np.maximum(np.abs(y), 1e-3 * sc.reshape((nv,) + (1,) * (y.ndim - 1)))
    if nv == 8:
        den[1] = np.maximum(den[1], 1e-2 * np.abs(y[0]))
    with np.errstate(invalid="ignore", divide="ignore"):
        e = np.where(den > 0, np.abs(x - y) / np.where(den > 0, den, 1.0), np.where(x == y, 0.0, np.inf))
    return e


def max_rel_err(x, y):
    return float(rel_err(x, y).max())


def scaled_abs_err(x, y):
    """max over cells of |x - y| / max|y_k| per component k (fluxes, conserved vectors)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    nv = y.shape[0]
    sc = np.abs(y).reshape(nv, -1).max(axis=1)
    # a component that vanishes identically (e.g. F^d(B^d)) is measured against the largest one
    sc = np.where(sc > 0, sc, sc.max())
    d = np.abs(x - y).reshape(nv, -1).max(axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        return float(np.where(sc > 0, d / np.where(sc > 0, sc, 1.0), np.where(d == 0, 0.0, np.inf)).max())


NAMES = ("rho", "u", "u~1", "u~2", "u~3", "B1", "B2", "B3")


def worst(x, y):
    """Description of the worst cell under rel_err (for assertion messages)."""
    e = rel_err(x, y)
    idx = np.unravel_index(int(np.argmax(e)), e.shape)
    var = NAMES[idx[0]] if y.shape[0] == 8 else str(idx[0])
    return (f"err {e[idx]:.3e} at {var}{tuple(int(v) for v in idx[1:])}: gpu {x[idx]!r} oracle {y[idx]!r}; "
            f"per-variable max {np.array2string(e.reshape(e.shape[0], -1).max(axis=1), precision=2)}")


def assert_parity(x, y, tol):
    err = max_rel_err(x, y)
    assert err < tol, worst(x, y)
