"""Pins of the oracle's hyper-exponential radial grid (Sec. 4.1: r = exp(X1) below x_b and
r = exp(X1 + (X1 - x_b)^n_X) beyond, x_b = ln 400, n_X = 4, outer edge 5000 M).

- The metric at points beyond x_b is the Boyer-Lindquist Kerr metric pulled back through
  Kerr-Schild time and the map, with dr/dX1 taken by Richardson-extrapolated central differences
  of r(X1) (not the oracle's analytic derivative).
- g g^-1 = I, sqrt(-g) = sqrt(-det g), and Gamma^l_{l mu} = d_mu ln sqrt(-g) there.
- r and dr/dX1 are continuous at x_b; the grid's outer X1 face sits at r = r_out.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from tests.test_oracle_geometry import _bl_metric

RNG = np.random.default_rng(2024)
R_BR, N_X = 400.0, 4


def _cfg(a=0.9375, n1=96):
    return orc.make_cfg(None, n1=n1, n2=64, n3=1, spin=a, h=0.3, r_out=5000.0, r_br=R_BR, n_x=N_X)


def _r(X1):
    xb = math.log(R_BR)
    return math.exp(X1) if X1 < xb else math.exp(X1 + (X1 - xb) ** N_X)


def _drdx(X1, h=1e-4):
    d = lambda e: (_r(X1 + e) - _r(X1 - e)) / (2 * e)
    return (4 * d(h / 2) - d(h)) / 3


def _points(n=20):
    xb = math.log(R_BR)
    for _ in range(n):
        yield RNG.uniform(-0.99, 0.99), RNG.uniform(xb + 0.05, xb + 1.2), RNG.uniform(0.03, 0.97)


def test_metric_beyond_the_break_is_the_pulled_back_kerr_metric():
    for a, X1, X2 in _points():
        h = 0.3
        th = math.pi * X2 + 0.5 * (1 - h) * math.sin(2 * math.pi * X2)
        J = np.diag([1.0, _drdx(X1), math.pi * (1 + (1 - h) * math.cos(2 * math.pi * X2)), 1.0])
        r = _r(X1)
        gcov, _, _, _ = orc.geom(_cfg(a), X1, X2)
        ks = np.linalg.inv(J).T @ gcov @ np.linalg.inv(J)
        dlt = r * r - 2 * r + a * a
        L = np.eye(4)
        L[0, 1] = -2 * r / dlt
        L[3, 1] = -a / dlt
        bl_from_ks = L.T @ _bl_metric(a, r, th) @ L
        assert np.allclose(ks, bl_from_ks, rtol=1e-8, atol=1e-8 * np.abs(ks).max()), (a, X1, X2)


def test_inverse_determinant_and_contracted_connection_beyond_the_break():
    for a, X1, X2 in _points(12):
        cfg = _cfg(a)
        gcov, gcon, gdet, conn = orc.geom(cfg, X1, X2)
        assert np.allclose(gcov @ gcon, np.eye(4), rtol=0, atol=1e-12)
        assert gdet == pytest.approx(math.sqrt(-np.linalg.det(gcov)), rel=1e-12)
        e = 1e-5
        for mu, (d1, d2) in ((1, (e, 0)), (2, (0, e))):
            f = lambda s: math.log(orc.geom(cfg, X1 + s * d1, X2 + s * d2)[2])
            d_e = (f(1) - f(-1)) / (2 * e)
            d_h = (f(0.5) - f(-0.5)) / e
            fd = (4 * d_h - d_e) / 3
            assert np.trace(conn[:, mu, :]) == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_map_is_continuous_at_the_break_and_reaches_r_out():
    cfg = _cfg()
    xb = math.log(R_BR)
    for s in (-1e-9, 1e-9):
        assert orc.geom(cfg, xb + s, 0.5)[2] == pytest.approx(orc.geom(cfg, xb, 0.5)[2], rel=1e-7)
    x1lo, dx1 = orc.grid_x1(cfg)
    assert x1lo == pytest.approx(math.log(cfg.r_in), rel=0, abs=0)
    assert _r(x1lo + cfg.n1 * dx1) == pytest.approx(5000.0, rel=1e-12)
    # without the break the same grid is plain exponential
    x1lo_p, dx1_p = orc.grid_x1(orc.make_cfg(None, n1=96, spin=0.9375, r_out=5000.0))
    assert dx1_p == pytest.approx((math.log(5000.0) - x1lo_p) / 96, rel=1e-15)
    assert dx1 < dx1_p
