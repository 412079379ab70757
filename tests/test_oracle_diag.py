"""Pins of the oracle's accretion diagnostics (Sec. 4.2: Eqs. diag_Mdot, diag_MAD,
angular_momentum_horizon, energy_flux_horizon, lin, lout) against states with a known answer.

- Marginally bound radial infall of cold dust in Schwarzschild (a = 0): the geodesic falling from
  rest at infinity has u_t = -1, so the energy flux equals the mass flux at every radius, and with
  no phi motion the angular-momentum fluxes vanish.  u^t and u^r are the closed forms
  u^r = -sqrt(2/r), u^t = (1 + x + x^2)/(1 + x), x = sqrt(2/r) (Kerr-Schild time).
- The same dust with u_phi = l in every cell: ldot_in(r) = l at every radius and Ldot = l Mdot.
- Reflection phi -> -phi at a = 0 (u~^3, B^3 -> -u~^3, -B^3): Mdot, phi_B and Edot unchanged,
  Ldot, ldot_in and ldot_out change sign.
- ldot_out is quadratic in the field.
- T^1_3 = (w + b^2) u^1 u_3 - b^1 b_3, so Ldot(r) = Mdot(r) (ldot_in - ldot_out) on any state.
"""
import math

import numpy as np

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import TorusConfig, make_torus


def _cfg(n1=24, n2=16, n3=1, spin=0.0):
    return orc.make_cfg(None, coords="mks", n1=n1, n2=n2, n3=n3, spin=spin, r_in_grid=1.6, r_out=30.0,
                        h=0.3, gam=4.0 / 3.0)


def _infall_dust(cfg, ell=None, seed=3):
    """Cold dust on the E = 1 radial geodesic (optionally with u_phi = ell), rho varying in theta/phi."""
    n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
    dx1 = (math.log(cfg.r_out) - math.log(cfg.r_in)) / n1
    rng = np.random.default_rng(seed)
    P = np.zeros((8, n1, n2, n3))
    P[0] = 0.5 + rng.random((n1, n2, n3))
    for i in range(n1):
        X1 = math.log(cfg.r_in) + (i + 0.5) * dx1
        r = math.exp(X1)
        x = math.sqrt(2.0 / r)
        ur = -x
        ut = (1.0 + x + x * x) / (1.0 + x)
        for j in range(n2):
            gcov, gcon, _, _ = orc.geom(cfg, X1, (j + 0.5) / n2)
            u1 = ur / r                       # X1 = ln r
            P[2, i, j, :] = u1 - ut * gcon[0, 1] / gcon[0, 0]
            if ell is not None:
                P[4, i, j, :] = ell / gcov[3, 3]   # a = 0: u^3 = u~^3 and u_3 = g_33 u^3
    return P


def test_marginally_bound_infall_energy_flux_equals_mass_flux():
    for n3 in (1, 6):
        cfg = _cfg(n3=n3)
        P = _infall_dust(cfg)
        hz, rad, ih = orc.diag_full(cfg, P)
        assert ih >= 0
        assert np.all(rad[0] < 0.0)                        # inflow everywhere
        assert np.allclose(rad[3], rad[0], rtol=1e-12, atol=0.0)
        assert np.all(rad[2] == 0.0) and np.all(rad[4] == 0.0) and np.all(rad[5] == 0.0)
        assert hz[3] == rad[3, ih] and hz[0] == rad[0, ih]
        assert hz[4] == hz[1] / math.sqrt(abs(hz[0]))


def test_uniform_specific_angular_momentum_gives_ldot_in_equal_to_it():
    ell = 2.7
    cfg = _cfg(n3=4)
    P = _infall_dust(cfg, ell=ell)
    hz, rad, ih = orc.diag_full(cfg, P)
    assert np.allclose(rad[4], ell, rtol=1e-13, atol=0.0)
    assert np.allclose(rad[2], ell * rad[0], rtol=1e-13, atol=0.0)
    assert hz[2] == rad[2, ih]
    assert np.all(rad[5] == 0.0)


def test_phi_reflection_at_zero_spin():
    c = TorusConfig(n1=32, n2=24, n3=1, spin=0.0, r_out=40.0, r_in=6.0, r_max=12.0, gam=13.0 / 9.0,
                    delta=0.04, seed=9, cfl=0.45)
    cfg = orc.make_cfg(c)
    P0 = make_torus(c)
    P, _, _, _ = orc.step(cfg, P0, 3)               # a state with inflow and sheared field
    P[7] += 0.3 * P[5]                              # give B^3 a share so b_3 is not trivial
    P[4] += 0.01
    R = P.copy()
    R[4] *= -1.0
    R[7] *= -1.0
    hz, rad, ih = orc.diag_full(cfg, P)
    hzr, radr, ihr = orc.diag_full(cfg, R)
    assert ih == ihr >= 0
    for q in (0, 1, 3):
        assert np.allclose(radr[q], rad[q], rtol=1e-13, atol=1e-300)
    for q in (2, 4, 5):
        assert np.allclose(radr[q], -rad[q], rtol=1e-12, atol=1e-300)
    assert np.abs(rad[2]).max() > 0.0 and np.abs(rad[5]).max() > 0.0


def test_outward_flux_is_quadratic_in_the_field():
    c = TorusConfig(n1=24, n2=16, n3=4, spin=0.9, r_out=40.0, r_in=6.0, r_max=12.0, gam=13.0 / 9.0,
                    delta=0.04, seed=10, cfl=0.45)
    cfg = orc.make_cfg(c)
    P = make_torus(c)
    P[7] = 0.2 * P[5] + 0.1 * P[6]
    Q = P.copy()
    Q[5:8] *= 3.0
    _, rad, _ = orc.diag_full(cfg, P)
    _, radq, _ = orc.diag_full(cfg, Q)
    assert np.allclose(radq[5], 9.0 * rad[5], rtol=1e-12, atol=1e-300)
    assert np.allclose(radq[0], rad[0], rtol=0, atol=0)       # the mass flux does not see B
    assert np.allclose(radq[1], 3.0 * rad[1], rtol=1e-14)


def test_horizon_row_matches_the_plain_horizon_diagnostic():
    c = TorusConfig(n1=24, n2=16, n3=1, spin=0.9375, r_out=40.0, delta=0.02, seed=1, cfl=0.8)
    cfg = orc.make_cfg(c)
    P = make_torus(c)
    hz, rad, ih = orc.diag_full(cfg, P)
    m, f, ih2 = orc.diag(cfg, P)
    assert ih == ih2
    assert hz[0] == m and hz[1] == f


def test_angular_momentum_flux_splits_into_inward_and_outward_parts():
    """T^1_3 = (w + b^2) u^1 u_3 - b^1 b_3 (delta^1_3 = 0): Ldot(r) = Mdot(r)(ldot_in - ldot_out),
    which ties the three sums together on a magnetised, spinning state."""
    c = TorusConfig(n1=24, n2=16, n3=4, spin=0.9, r_out=40.0, r_in=6.0, r_max=12.0, gam=13.0 / 9.0,
                    delta=0.04, seed=12, cfl=0.45)
    cfg = orc.make_cfg(c)
    P = make_torus(c)
    P[7] = 0.3 * P[5] - 0.2 * P[6]
    hz, rad, ih = orc.diag_full(cfg, P)
    assert np.abs(rad[5]).max() > 1e-3 * np.abs(rad[4]).max()   # the field term is not negligible
    scale = np.abs(rad[0] * rad[4]) + np.abs(rad[0] * rad[5])
    assert np.all(np.abs(rad[2] - rad[0] * (rad[4] - rad[5])) <= 1e-12 * scale)
