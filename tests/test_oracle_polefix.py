"""Pins of the oracle's polar u~2 interpolation (Sec. 4.1: the polar velocity component of the two
cells next to each pole is interpolated to zero at the pole; reading: a straight line in X2 from
zero at the pole to the centre of the first cell left alone).

- A step too short to change anything else (dt = 1e-300: U + dt L rounds to U) leaves just the
  interpolation: u~2 of cell j < n_p is (j + 1/2)/(n_p + 1/2) times u~2 of cell n_p, mirrored at
  the other pole, to the inversion's round-off, and every other primitive keeps its value.
- With it on, an equatorially symmetric torus stays mirror symmetric over several steps (the
  upper pole is handled as the mirror image of the lower one) and differs from the run without it.
- It applies to MKS grids only and needs 2 n_p < n2.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import TorusConfig, make_torus


def _torus(**kw):
    base = dict(n1=24, n2=32, n3=1, r_out=40.0, delta=0.0, beta=100.0, beta_mode="min",
                rho_fl_coef=1e-4, rho_fl_pow=-1.5, u_fl_coef=1e-6, u_fl_pow=-2.5, cfl=0.8)
    base.update(kw)
    return TorusConfig(**base)


@pytest.mark.parametrize("npole", [2, 3])
def test_a_null_step_leaves_the_linear_interpolation_at_both_poles(npole):
    c = _torus(n3=4)
    P0 = make_torus(c)
    rng = np.random.default_rng(8)
    P0[3] = 0.05 * (0.5 + rng.random(P0[3].shape))         # a polar velocity everywhere
    cfg = orc.make_cfg(c, pole_fix=npole)
    P1, _, nfail, _ = orc.step(cfg, P0, 1, 1e-300)
    assert nfail == 0
    n2 = c.n2
    tol = 1e-9
    for j in range(npole):
        f = (j + 0.5) / (npole + 0.5)
        lo, hi = P1[3, :, j], P1[3, :, n2 - 1 - j]
        assert np.all(np.abs(lo - f * P0[3, :, npole]) <= tol * np.abs(P0[3, :, npole]))
        assert np.all(np.abs(hi - f * P0[3, :, n2 - 1 - npole]) <= tol * np.abs(P0[3, :, n2 - 1 - npole]))
    keep = np.ones(n2, bool)
    keep[:npole] = keep[n2 - npole:] = False
    assert np.all(np.abs(P1[3][:, keep] - P0[3][:, keep]) <= tol * np.abs(P0[3][:, keep]))
    for q in (0, 1, 2, 4, 5, 6, 7):
        scale = max(np.abs(P0[q]).max(), 1e-30)
        assert np.abs(P1[q] - P0[q]).max() <= tol * scale, q
    # without the option the same null step changes nothing
    Q1, _, _, _ = orc.step(orc.make_cfg(c), P0, 1, 1e-300)
    assert np.abs(Q1[3] - P0[3]).max() <= tol * np.abs(P0[3]).max()


def test_equatorially_symmetric_torus_stays_symmetric_with_the_polar_interpolation():
    c = _torus(n1=32)
    P0 = make_torus(c)
    cfg = orc.make_cfg(c, pole_fix=2)
    P1, _, _, _ = orc.step(cfg, P0, 6)
    M = P1[:, :, ::-1, :]
    sym = np.array([1, 1, 1, -1, 1, -1, 1, -1])  # rho, u, u~1, -u~2, u~3, -B1, B2, -B3
    scale = np.abs(P1).reshape(8, -1).max(axis=1)
    for q in range(8):
        assert np.abs(P1[q] - sym[q] * M[q]).max() <= 1e-12 * max(scale[q], 1e-30), q
    Q1, _, _, _ = orc.step(orc.make_cfg(c), P0, 6)
    assert np.abs(Q1[3] - P1[3]).max() > 0.0


def test_polar_interpolation_needs_an_mks_grid_with_room_for_both_poles():
    c = _torus(n2=8)
    P0 = make_torus(c)
    with pytest.raises(RuntimeError):
        orc.step(orc.make_cfg(c, pole_fix=4), P0, 1)
    orc.step(orc.make_cfg(c, pole_fix=3), P0, 1)
    P = np.zeros((8, 8, 8, 1))
    P[0] = P[1] = 1.0
    with pytest.raises(RuntimeError):
        orc.step(orc.make_cfg(None, coords="cart", n1=8, n2=8, n3=1, pole_fix=2), P, 1)
