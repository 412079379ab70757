"""Pins of the oracle's geometry (metric, inverse, sqrt(-g), connection) against facts that do
not come from the oracle's own formulas.

Paper passages: Kerr-Schild line element and MKS coordinates, Sec. 4.1; centred source term
sqrt(-g) T^k_l Gamma^l_{nu k}, Sec. 2.2.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc

RNG = np.random.default_rng(12345)


def _cfg(a, h=0.3):
    return orc.make_cfg(None, n1=64, n2=64, n3=1, spin=a, h=h, r_out=40.0)


def _points(n=25):
    for _ in range(n):
        a = RNG.uniform(-0.99, 0.99)
        X1 = RNG.uniform(math.log(1.2), math.log(900.0))
        X2 = RNG.uniform(0.02, 0.98)
        yield a, X1, X2


def _bl_metric(a, r, th):
    """Textbook Boyer-Lindquist Kerr metric (M = 1), written independently of the KS form."""
    s2 = math.sin(th) ** 2
    sig = r * r + a * a * math.cos(th) ** 2
    dlt = r * r - 2 * r + a * a
    g = np.zeros((4, 4))
    g[0, 0] = -(1 - 2 * r / sig)
    g[0, 3] = g[3, 0] = -2 * a * r * s2 / sig
    g[1, 1] = sig / dlt
    g[2, 2] = sig
    g[3, 3] = (r * r + a * a + 2 * a * a * r * s2 / sig) * s2
    return g


def _mks_jac(X1, X2, h=0.3):
    th = math.pi * X2 + 0.5 * (1 - h) * math.sin(2 * math.pi * X2)
    return math.exp(X1), th, np.diag([1.0, math.exp(X1), math.pi * (1 + (1 - h) * math.cos(2 * math.pi * X2)), 1.0])


def test_metric_times_inverse_is_identity():
    for a, X1, X2 in _points():
        gcov, gcon, gdet, _ = orc.geom(_cfg(a), X1, X2)
        assert np.allclose(gcov @ gcon, np.eye(4), rtol=0, atol=1e-13), (a, X1, X2)


def test_sqrt_minus_det_matches_numerical_determinant():
    for a, X1, X2 in _points():
        gcov, gcon, gdet, _ = orc.geom(_cfg(a), X1, X2)
        assert gdet == pytest.approx(math.sqrt(-np.linalg.det(gcov)), rel=1e-12)


def test_ks_metric_is_boyer_lindquist_transformed():
    """g_KS = L^T g_BL L with dt_BL = dt_KS - 2r/Delta dr, dphi_BL = dphi_KS - a/Delta dr."""
    for a, X1, X2 in _points():
        r, th, J = _mks_jac(X1, X2)
        gcov, _, _, _ = orc.geom(_cfg(a), X1, X2)
        ks = np.linalg.inv(J).T @ gcov @ np.linalg.inv(J)
        dlt = r * r - 2 * r + a * a
        L = np.eye(4)
        L[0, 1] = -2 * r / dlt
        L[3, 1] = -a / dlt
        bl_from_ks = L.T @ _bl_metric(a, r, th) @ L
        assert np.allclose(ks, bl_from_ks, rtol=1e-12, atol=1e-12 * np.abs(ks).max()), (a, r, th)


def test_contracted_connection_is_gradient_of_log_sqrt_g():
    """Gamma^l_{l mu} = d_mu ln sqrt(-g) (the sqrt(-g) derivative by central differences)."""
    for a, X1, X2 in _points(15):
        _, _, gdet, conn = orc.geom(_cfg(a), X1, X2)
        e = 1e-5
        for mu, (d1, d2) in ((1, (e, 0)), (2, (0, e))):
            gp = orc.geom(_cfg(a), X1 + d1, X2 + d2)[2]
            gm = orc.geom(_cfg(a), X1 - d1, X2 - d2)[2]
            fd = (math.log(gp) - math.log(gm)) / (2 * e)
            assert np.trace(conn[:, mu, :]) == pytest.approx(fd, rel=1e-7, abs=1e-9)
        assert abs(np.trace(conn[:, 0, :])) < 1e-14
        assert abs(np.trace(conn[:, 3, :])) < 1e-14


def test_connection_matches_richardson_differences_of_the_metric():
    for a, X1, X2 in _points(10):
        gcov, gcon, _, conn = orc.geom(_cfg(a), X1, X2)
        dg = np.zeros((4, 4, 4))
        for mu in (1, 2):
            def g_at(s):
                return orc.geom(_cfg(a), X1 + (s if mu == 1 else 0), X2 + (s if mu == 2 else 0))[0]
            e = 1e-3
            d1 = (g_at(e) - g_at(-e)) / (2 * e)
            d2 = (g_at(e / 2) - g_at(-e / 2)) / e
            dg[mu] = (4 * d2 - d1) / 3
        low = 0.5 * (np.einsum("msn->smn", dg) + np.einsum("nsm->smn", dg) - dg)
        ref = np.einsum("ls,smn->lmn", gcon, low)
        scale = np.abs(ref).max()
        assert np.allclose(conn, ref, rtol=0, atol=1e-8 * scale)


def test_circular_equatorial_geodesic_has_no_radial_acceleration():
    """For a prograde circular equatorial orbit (Bardeen-Press-Teukolsky E, L), the geodesic
    equation requires Gamma^r_{mu nu} u^mu u^nu = 0 and Gamma^theta_{mu nu} u^mu u^nu = 0."""
    for a in (-0.7, 0.0, 0.5, 0.9375):
        for r in (8.0, 12.0, 41.0):
            sr = math.sqrt(r)
            den = r ** 0.75 * math.sqrt(r ** 1.5 - 3 * sr + 2 * a)
            E = (r ** 1.5 - 2 * sr + a) / den
            Lz = (r * r - 2 * a * sr + a * a) / den
            sig, dlt = r * r, r * r - 2 * r + a * a
            A = (r * r + a * a) ** 2 - a * a * dlt
            ut = (A * E - 2 * a * r * Lz) / (sig * dlt)
            # BL inverse at the equator: g^{t phi} = -2ar/(Sigma Delta), g^{phi phi} = (Delta - a^2)/(Sigma Delta)
            uph = (-2 * a * r / (sig * dlt)) * (-E) + ((dlt - a * a) / (sig * dlt)) * Lz
            X1 = math.log(r)
            X2 = 0.5
            _, _, _, conn = orc.geom(_cfg(a), X1, X2)
            u = np.array([ut, 0.0, 0.0, uph])  # u^r = 0: KS and MKS share u^t, u^phi
            acc = np.einsum("lmn,m,n->l", conn, u, u)
            assert abs(acc[1]) < 1e-12 * ut * ut and abs(acc[2]) < 1e-12 * ut * ut, (a, r, acc)


def test_flat_space_geometry():
    c = orc.make_cfg(None, coords="cart", n1=8, n2=8, n3=8)
    gcov, gcon, gdet, conn = orc.geom(c, 0.3, 0.7)
    assert np.array_equal(gcov, np.diag([-1.0, 1, 1, 1]))
    assert gdet == 1.0 and not conn.any()
