"""Pins of the oracle's HLL flux (Sec. 2.2, Eq. fluxes_HLL) against what its definition fixes,
independently of the formula as the oracle writes it.

The HLL flux weights the left and right physical fluxes by the fastest right- and left-going
signal speeds c_max and c_min (both clipped at zero).  Three limits follow from the definition:
- every wave of both states moves right (c_min = 0): the face flux is the left state's physical
  flux F(P_l), with no dissipation;
- every wave moves left (c_max = 0): it is the right state's flux F(P_r);
- c_max = c_min (a fluid at rest on both sides): it is the Lax-Friedrichs flux of the same face.
The expected fluxes come from the oracle's per-point flux vector of the reconstructed states (the
MC-limited PLM states, built here from the limiter alone) and from its LLF sweep; a swap of c_max
and c_min in the weights (planted below) turns the first limit into F(P_r) and fails.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from tests._planted import variant

N = 32


def _line(v, gam=5.0 / 3.0, bx=0.0, by=0.0):
    """A 1D flat periodic line (X1 active) with a smooth density and pressure wave carried at
    3-velocity v along X1, plus a weak field."""
    x = (np.arange(N) + 0.5) / N
    P = np.zeros((8, N, 1, 1))
    rho = 1.0 + 0.3 * np.sin(2 * math.pi * x) + 0.1 * np.cos(6 * math.pi * x)
    p = 1e-3 * (1.0 + 0.5 * np.cos(2 * math.pi * x))
    lor = 1.0 / math.sqrt(1.0 - v * v)
    P[0, :, 0, 0] = rho
    P[1, :, 0, 0] = p / (gam - 1.0)
    P[2, :, 0, 0] = lor * v
    P[5, :, 0, 0] = bx
    P[6, :, 0, 0] = by * (1.0 + 0.2 * np.sin(2 * math.pi * x))
    return P


def _cfg(riemann, gam=5.0 / 3.0):
    return orc.make_cfg(None, coords="cart", n1=N, n2=1, n3=1, gam=gam, riemann=riemann,
                        xmin=(0.0, 0.0, 0.0), xmax=(1.0, 1.0, 1.0))


def _states(P, f):
    """MC-limited PLM states on the face between cells f-1 and f (Sec. 2.2)."""
    q = P[:, :, 0, 0]
    Pl = np.array([q[v, f - 1] + 0.5 * orc.mc_slope(q[v, f - 2], q[v, f - 1], q[v, f]) for v in range(8)])
    Pr = np.array([q[v, f] - 0.5 * orc.mc_slope(q[v, f - 1], q[v, f], q[v, f + 1]) for v in range(8)])
    return Pl, Pr


def _phys_flux(cfg, Ps):
    return orc.point_state(cfg, 0.5, 0.5, Ps)["F"][1]


def _speeds(cfg, Ps):
    return orc.point_state(cfg, 0.5, 0.5, Ps)["speeds"][0]   # (c1, c2) along X1


def _check_one_sided(v, expect_left):
    cfg = _cfg("hll")
    P = _line(v, bx=0.05, by=0.02)
    F, _ = orc.fluxes(cfg, P, 1)
    Fllf, _ = orc.fluxes(_cfg("llf"), P, 1)
    checked = 0
    for f in range(2, N - 1):              # stencils off the periodic wrap
        Pl, Pr = _states(P, f)
        cl, cr = _speeds(cfg, Pl), _speeds(cfg, Pr)
        if expect_left:
            assert min(cl[1], cr[1]) > 0.0  # every wave moves right
        else:
            assert max(cl[0], cr[0]) < 0.0  # every wave moves left
        Fx = _phys_flux(cfg, Pl if expect_left else Pr)
        got = F[:, f, 0, 0]
        scale = np.abs(Fx).max()
        assert np.abs(got[:8] - Fx[:8]).max() <= 4e-16 * scale * 4, (f, got, Fx)
        # the limit is not the LLF flux: LLF keeps dissipation where the states differ
        if np.abs(Pl - Pr).max() > 1e-6:
            assert np.abs(Fllf[:8, f, 0, 0] - Fx[:8]).max() > 1e-8 * scale
        checked += 1
    assert checked == N - 3


def test_all_waves_right_gives_the_left_flux():
    _check_one_sided(0.9, expect_left=True)


def test_all_waves_left_gives_the_right_flux():
    _check_one_sided(-0.9, expect_left=False)


def test_equal_signal_speeds_give_the_lax_friedrichs_flux():
    # at rest with a uniform pressure the sound speed differs between the states only through
    # the density, so take a uniform density too and vary the field along X2 (transverse): then
    # c_max = c_min on every face, and HLL must reduce to LLF to round-off
    P = _line(0.0, bx=0.0, by=0.05)
    P[0] = 1.0
    P[1] = 1e-3 / (5.0 / 3.0 - 1.0)
    P[6, :, 0, 0] = 0.05 * (1.0 + 0.2 * np.sin(2 * math.pi * (np.arange(N) + 0.5) / N))
    Fh, cwh = orc.fluxes(_cfg("hll"), P, 1)
    Fl, cwl = orc.fluxes(_cfg("llf"), P, 1)
    assert cwh == cwl
    for f in range(2, N - 1):
        Pl, Pr = _states(P, f)
        cl, cr = _speeds(_cfg("hll"), Pl), _speeds(_cfg("hll"), Pr)
        assert math.isclose(max(cl[0], cr[0]), -min(cl[1], cr[1]), rel_tol=1e-15)
    scale = np.abs(Fl).max(axis=(1, 2, 3), keepdims=True)
    assert np.all(np.abs(Fh - Fl) <= 1e-15 * np.maximum(scale, 1e-300))
    # and the face states do differ, so the dissipation term is exercised
    assert np.abs(np.diff(P[6, :, 0, 0])).max() > 1e-3


def test_moving_flow_hll_differs_from_llf():
    """Away from those limits the two solvers differ (HLL is not LLF in disguise)."""
    P = _line(0.3, bx=0.05, by=0.02)
    P[1] *= 1e3          # hot: sound speed above 0.3, waves both ways
    Fh, _ = orc.fluxes(_cfg("hll"), P, 1)
    Fl, _ = orc.fluxes(_cfg("llf"), P, 1)
    assert np.abs(Fh - Fl).max() > 1e-6 * np.abs(Fl).max()


def test_planted_weight_swap_fails(tmp_path):
    swap = ("F[q] = (cmax * Fl[q] + cmin * Fr[q] - cmax * cmin * (Ur[q] - Ul[q])) / (cmax + cmin);",
            "F[q] = (cmin * Fl[q] + cmax * Fr[q] - cmax * cmin * (Ur[q] - Ul[q])) / (cmax + cmin);")
    with variant(tmp_path, "hll_swap", [swap]):
        with pytest.raises(AssertionError):
            _check_one_sided(0.9, expect_left=True)
    # the original passes again outside the variant
    _check_one_sided(0.9, expect_left=True)
