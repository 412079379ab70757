"""Pins of the oracle's primitive->4-vector map, conserved variables, fluxes, wave speeds, MC
limiter and geometric source against closed forms and identities.

Paper passages: u~ and b^mu definitions and T^{mu nu}, Sec. 2.1; PLM/MC limiter, simplified
dispersion relation and the Lax-Friedrichs flux, Sec. 2.2; centred source, Sec. 2.2.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from tests._states import random_state

RNG = np.random.default_rng(2024)
KERR = orc.make_cfg(None, n1=64, n2=64, n3=1, spin=0.9375, r_out=40.0, gam=13.0 / 9.0)
FLAT = orc.make_cfg(None, coords="cart", n1=8, n2=8, n3=8, gam=5.0 / 3.0)


def _kerr_points(n):
    for _ in range(n):
        yield RNG.uniform(math.log(1.4), math.log(500.0)), RNG.uniform(0.03, 0.97)


def _bsq_fn(cfg, X1, X2):
    def f(P):
        s = orc.point_state(cfg, X1, X2, P)
        return s["bcon"] @ s["bcov"]
    return f


def test_four_velocity_normalised_and_b_orthogonal():
    for X1, X2 in _kerr_points(40):
        gcov = orc.geom(KERR, X1, X2)[0]
        P = random_state(RNG, gcov)
        s = orc.point_state(KERR, X1, X2, P)
        assert s["ucon"] @ s["ucov"] == pytest.approx(-1.0, abs=1e-12)
        bmag = math.sqrt(abs(s["bcon"] @ s["bcov"]))
        assert abs(s["bcon"] @ s["ucov"]) < 1e-12 * max(1.0, bmag * s["ucon"][0])


def test_rest_frame_conserved_and_flux_closed_forms():
    gam = FLAT.gam
    B = np.array([0.3, -0.2, 0.5])
    rho, u = 0.7, 0.9
    P = np.array([rho, u, 0, 0, 0, *B])
    s = orc.point_state(FLAT, 0.0, 0.0, P)
    p = (gam - 1) * u
    b2 = B @ B
    U_ref = [rho, -(rho + u + 0.5 * b2), 0, 0, 0, *B, p / rho ** (gam - 1)]
    assert np.allclose(s["U"], U_ref, rtol=1e-15, atol=1e-15)
    F1_ref = [0, 0, p + 0.5 * b2 - B[0] ** 2, -B[0] * B[1], -B[0] * B[2], 0, 0, 0, 0]
    assert np.allclose(s["F"][1], F1_ref, rtol=1e-15, atol=1e-15)


def test_moving_hydro_conserved_closed_form():
    gam = FLAT.gam
    rho, u, v = 0.3, 0.2, 0.6
    lor = 1 / math.sqrt(1 - v * v)
    P = np.array([rho, u, lor * v, 0, 0, 0, 0, 0])
    s = orc.point_state(FLAT, 0.0, 0.0, P)
    p = (gam - 1) * u
    w = rho + u + p
    assert s["U"][0] == pytest.approx(rho * lor, rel=1e-14)
    assert s["U"][1] == pytest.approx(-(w * lor * lor - p), rel=1e-14)
    assert s["U"][2] == pytest.approx(w * lor * lor * v, rel=1e-14)
    assert s["F"][1][2] == pytest.approx(w * lor * lor * v * v + p, rel=1e-14)


def test_sound_speeds_add_relativistically_in_flat_space():
    gam = FLAT.gam
    for v in (-0.9, -0.3, 0.0, 0.5, 0.95):
        rho, u = 1.0, 0.4
        lor = 1 / math.sqrt(1 - v * v)
        P = np.array([rho, u, lor * v, 0, 0, 0, 0, 0])
        c1, c2 = orc.point_state(FLAT, 0.0, 0.0, P)["speeds"][0]
        p = (gam - 1) * u
        cs = math.sqrt(gam * p / (rho + u + p))
        assert c1 == pytest.approx((v + cs) / (1 + v * cs), rel=1e-13, abs=1e-15)
        assert c2 == pytest.approx((v - cs) / (1 - v * cs), rel=1e-13, abs=1e-15)


def _flux_jacobian_eigs(P, d=1, eps=1e-6):
    """Eigenvalues of dF^d/dU (mass, energy-momentum and field rows) by central differences."""
    n = 8
    dU = np.zeros((n, n))
    dF = np.zeros((n, n))
    for q in range(n):
        h = eps * max(1.0, abs(P[q]))
        Pp, Pm = P.copy(), P.copy()
        Pp[q] += h
        Pm[q] -= h
        sp = orc.point_state(FLAT, 0.0, 0.0, Pp)
        sm = orc.point_state(FLAT, 0.0, 0.0, Pm)
        dU[:, q] = (sp["U"][:8] - sm["U"][:8]) / (2 * h)
        dF[:, q] = (sp["F"][d][:8] - sm["F"][d][:8]) / (2 * h)
    return np.linalg.eigvals(dF @ np.linalg.inv(dU))


def test_flux_jacobian_perpendicular_field_gives_fast_speed():
    """k perpendicular to B: the only non-zero characteristic speeds are +-sqrt(v_a^2 + c_s^2(1 - v_a^2)),
    which is also what the simplified dispersion relation returns (exact in this geometry)."""
    gam = FLAT.gam
    rho, u, B2 = 1.0, 0.5, 0.8
    P = np.array([rho, u, 0, 0, 0, 0.0, B2, 0.0])
    ev = _flux_jacobian_eigs(P)
    assert np.abs(ev.imag).max() < 1e-6
    p = (gam - 1) * u
    w = rho + u + p
    va2 = B2 ** 2 / (B2 ** 2 + w)
    cf = math.sqrt(va2 + gam * p / w * (1 - va2))
    ev = np.sort(ev.real)
    assert ev[-1] == pytest.approx(cf, rel=1e-6)
    assert ev[0] == pytest.approx(-cf, rel=1e-6)
    assert np.abs(ev[1:-1]).max() < 1e-6
    c1, c2 = orc.point_state(FLAT, 0.0, 0.0, P)["speeds"][0]
    assert c1 == pytest.approx(cf, rel=1e-13) and c2 == pytest.approx(-cf, rel=1e-13)


def test_flux_jacobian_parallel_field_gives_sound_and_alfven_speeds():
    """k parallel to B: +-c_s once and +-v_A twice, v_A^2 = b^2/(w + b^2).  A wrong sign of the
    induction flux turns the Alfven pair imaginary, so this pins the induction flux."""
    gam = FLAT.gam
    rho, u, B1 = 1.0, 0.5, 0.8
    P = np.array([rho, u, 0, 0, 0, B1, 0.0, 0.0])
    ev = _flux_jacobian_eigs(P)
    assert np.abs(ev.imag).max() < 1e-6
    p = (gam - 1) * u
    w = rho + u + p
    cs = math.sqrt(gam * p / w)
    va = math.sqrt(B1 ** 2 / (w + B1 ** 2))
    ev = np.sort(ev.real)
    ref = np.sort([-cs, cs, -va, -va, va, va, 0.0, 0.0])
    assert np.allclose(ev, ref, atol=1e-6)


def test_mc_limiter_equals_minmod_form():
    def minmod_ref(qm, q0, qp):
        dm, dp, dc = q0 - qm, qp - q0, qp - qm
        if dm * dp <= 0:
            return 0.0
        return math.copysign(min(2 * abs(dm), 2 * abs(dp), 0.5 * abs(dc)), dc)
    for _ in range(20000):
        q = RNG.normal(size=3) * 10 ** RNG.uniform(-8, 3, size=3)
        if RNG.random() < 0.1:
            q[RNG.integers(3)] = q[1]
        assert orc.mc_slope(*q) == minmod_ref(*q)


def test_mc_limiter_linear_data_and_extrema():
    # the data a - s, a, a + s are rounded when formed: each carries up to half an ulp of |a| + |s|,
    # so the limited slope equals s within a few ulp of |a| + |s| (not of |s| alone)
    rng = np.random.default_rng(7)
    for _ in range(200):
        a, s = rng.normal(), rng.normal()
        tol = 4 * np.finfo(float).eps * (abs(a) + abs(s))
        assert abs(orc.mc_slope(a - s, a, a + s) - s) <= tol
    assert orc.mc_slope(0.0, 1.0, 0.5) == 0.0
    assert orc.mc_slope(1.0, 0.0, 0.5) == 0.0


def test_source_vanishes_for_t_and_phi_and_matches_metric_derivative_form():
    """S_nu = sqrt(-g) T^k_l Gamma^l_{nu k} = 1/2 sqrt(-g) T^{kl} d_nu g_{kl}; d_t g = d_phi g = 0."""
    for X1, X2 in _kerr_points(20):
        gcov, gcon, gdet, _ = orc.geom(KERR, X1, X2)
        P = random_state(RNG, gcov, beta=10 ** RNG.uniform(-1, 3), point_state=_bsq_fn(KERR, X1, X2))
        s = orc.point_state(KERR, X1, X2, P)
        ucon, bcon = s["ucon"], s["bcon"]
        gam = KERR.gam
        p = (gam - 1) * P[1]
        w = P[0] + P[1] + p
        b2 = bcon @ s["bcov"]
        T = (w + b2) * np.outer(ucon, ucon) + (p + b2 / 2) * gcon - np.outer(bcon, bcon)
        scale = gdet * np.abs(T).max() * np.abs(gcov).max()
        assert abs(s["src"][0]) < 1e-11 * scale and abs(s["src"][3]) < 1e-11 * scale
        for nu in (1, 2):
            e = 1e-4
            d = [e if nu == 1 else 0, e if nu == 2 else 0]
            gp = orc.geom(KERR, X1 + d[0], X2 + d[1])[0]
            gm = orc.geom(KERR, X1 - d[0], X2 - d[1])[0]
            gp2 = orc.geom(KERR, X1 + d[0] / 2, X2 + d[1] / 2)[0]
            gm2 = orc.geom(KERR, X1 - d[0] / 2, X2 - d[1] / 2)[0]
            dg = (4 * (gp2 - gm2) / e - (gp - gm) / (2 * e)) / 3
            ref = 0.5 * gdet * np.sum(T * dg)
            assert s["src"][nu] == pytest.approx(ref, rel=1e-6, abs=1e-9 * scale)
