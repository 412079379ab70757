"""Pins of the oracle's PPM reconstruction: Colella & Woodward (1984), the upgrade of the MC-limited
PLM that Sec. 2.2 names.  Each pin holds for the method and not for a plausible slip in it.

- Exactness: on cell averages of a cubic where no limiter acts, both face states equal the cubic's
  point value at the face (the interface value is fourth order; a dropped or mis-weighted slope
  term leaves an O(h^2) error that the test sees).
- Bounds: on random data both states lie between the two cells that share the face (the limited
  slopes keep the interface value there, and the constraints only move an edge towards the cell
  average).
- Monotone cells: with a cell's lower and upper edge values read from its two faces, the parabola
  has no extremum strictly inside the cell, and a local extremum of the data gives the flat profile.
- Order: the face-state error on cell averages of exp(x) falls as h^4 (PLM with MC: h^2).
- Wiring into the flux sweep (flat space): on data linear in the cell index both reconstructions
  are exact, so the PPM and PLM fluxes agree on faces whose stencils stay off the periodic wrap;
  mirroring random data along a direction mirrors its fluxes, which fails for an off-centre stencil
  or swapped face states; at rest the momentum flux is the mean pressure of the face states, which
  ties each face to its six cells in order.
- A grid with fewer active cells than the three ghost cells PPM needs is refused.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc


def _cubic_avgs(x0, h, n, c):
    """Exact cell averages of c0 + c1 x + c2 x^2 + c3 x^3 on cells [x0 + m h, x0 + (m+1) h]."""
    def F(x):
        return c[0] * x + c[1] * x * x / 2 + c[2] * x ** 3 / 3 + c[3] * x ** 4 / 4
    e = x0 + h * np.arange(n + 1)
    return (F(e[1:]) - F(e[:-1])) / h


def _plm_face(q6):
    dl = orc.mc_slope(q6[1], q6[2], q6[3])
    dr = orc.mc_slope(q6[2], q6[3], q6[4])
    return q6[2] + 0.5 * dl, q6[3] - 0.5 * dr


def test_cubic_data_gives_the_point_value_on_both_sides():
    c = (1.0, 0.8, 0.3, 0.1)        # increasing and convex on [0, 2]: no limiter or constraint acts
    h = 0.05
    a = _cubic_avgs(0.0, h, 40, c)
    for f in range(3, 38):          # face between cells f-1 and f
        xf = f * h
        exact = c[0] + c[1] * xf + c[2] * xf ** 2 + c[3] * xf ** 3
        ql, qr = orc.ppm_face(a[f - 3:f + 3])
        assert ql == pytest.approx(exact, rel=2e-14, abs=0)
        assert qr == pytest.approx(exact, rel=2e-14, abs=0)
        # the test discriminates: PLM misses the quadratic part of the profile
        pl, pr = _plm_face(a[f - 3:f + 3])
        assert abs(pl - exact) > 1e-6 * abs(exact) or abs(pr - exact) > 1e-6 * abs(exact)


def test_states_lie_between_the_two_cells_of_the_face():
    rng = np.random.default_rng(5)
    for trial in range(4000):
        q = rng.standard_normal(6) * rng.choice([1e-3, 1.0, 1e3])
        if trial % 3 == 0:
            q = np.sort(q)                          # monotone runs too
        ql, qr = orc.ppm_face(q)
        lo, hi = min(q[2], q[3]), max(q[2], q[3])
        assert lo <= ql <= hi and lo <= qr <= hi, q


def _edges(a):
    """Lower and upper edge values of cells 3..len(a)-4 from the states of their faces."""
    M = len(a)
    r = np.full(M, np.nan)
    l = np.full(M, np.nan)
    for f in range(3, M - 2):                       # face between cells f-1 and f
        r[f - 1], l[f] = orc.ppm_face(a[f - 3:f + 3])
    return l[3:M - 3], r[3:M - 3], a[3:M - 3], a[2:M - 4], a[4:M - 2]


@pytest.mark.parametrize("kind", ["noise", "steps", "smooth"])
def test_each_cell_parabola_is_monotone(kind):
    rng = np.random.default_rng(7)
    M = 400
    x = np.arange(M) / M
    if kind == "noise":
        a = rng.standard_normal(M)
    elif kind == "steps":
        a = np.where(x < 0.3, 1.0, 0.1) + np.where(x > 0.7, 2.0, 0.0) + 1e-3 * rng.random(M)
    else:
        a = np.sin(12 * np.pi * x) + 0.3 * np.cos(31 * np.pi * x)
    l, r, a0, am, ap = _edges(a)
    da = r - l
    a6 = 6.0 * (a0 - 0.5 * (l + r))
    scale = np.abs(a0) + np.abs(l) + np.abs(r)
    assert np.all(np.abs(a6) <= np.abs(da) + 1e-13 * scale)
    ext = (ap - a0) * (a0 - am) <= 0.0
    assert ext.sum() > 5
    assert np.all(l[ext] == a0[ext]) and np.all(r[ext] == a0[ext])
    # a cell's edges lie between its own average and its neighbours'
    assert np.all((l - a0) * (am - a0) >= 0.0) and np.all((r - a0) * (ap - a0) >= 0.0)


def _face_error(n, face):
    h = 1.0 / n
    e = h * np.arange(n + 1)
    a = (np.exp(e[1:]) - np.exp(e[:-1])) / h
    err = 0.0
    for f in range(3, n - 2):
        ql, qr = face(a[f - 3:f + 3])
        ex = math.exp(f * h)
        err = max(err, abs(ql - ex), abs(qr - ex))
    return err


def test_face_states_converge_at_fourth_order_on_smooth_monotone_data():
    e = [_face_error(n, orc.ppm_face) for n in (16, 32, 64)]
    assert e[0] / e[1] > 12.0 and e[1] / e[2] > 12.0, e
    p = [_face_error(n, _plm_face) for n in (16, 32, 64)]
    assert p[0] / p[1] < 6.0 and p[1] / p[2] < 6.0, p   # PLM: second order


def _cart(recon, n=(12, 10, 9), **kw):
    return orc.make_cfg(None, coords="cart", n1=n[0], n2=n[1], n3=n[2], gam=4.0 / 3.0, cfl=0.4,
                        recon=recon, **kw)


def test_linear_data_gives_the_plm_fluxes_away_from_the_wrap():
    n = (12, 10, 9)
    rng = np.random.default_rng(2)
    I, J, K = np.meshgrid(np.arange(n[0]), np.arange(n[1]), np.arange(n[2]), indexing="ij")
    P = np.zeros((8,) + n)
    base = np.array([1.0, 0.8, 0.1, -0.05, 0.08, 0.3, -0.2, 0.25])
    for v in range(8):
        s = 0.01 * rng.standard_normal(3) * max(abs(base[v]), 0.1)
        P[v] = base[v] + s[0] * I + s[1] * J + s[2] * K
    for d in (1, 2, 3):
        Fp, _ = orc.fluxes(_cart("ppm", n), P, d)
        Fl, _ = orc.fluxes(_cart("plm", n), P, d)
        sl = [slice(None)] * 4
        sl[d] = slice(3, n[d - 1] - 1)             # stencils of both methods inside the data
        a, b = Fp[tuple(sl)], Fl[tuple(sl)]
        scale = np.abs(Fl).max(axis=(1, 2, 3), keepdims=True)
        assert np.all(np.abs(a - b) <= 1e-13 * scale), d


def test_mirrored_data_gives_mirrored_fluxes():
    n = (11, 10, 9)
    rng = np.random.default_rng(4)
    P = np.zeros((8,) + n)
    P[0] = 0.5 + rng.random(n)
    P[1] = 0.2 + rng.random(n)
    P[2:5] = 0.4 * rng.standard_normal((3,) + n)
    P[5:8] = 0.5 * rng.standard_normal((3,) + n)
    for d in (1, 2, 3):
        for riem in ("llf", "hll"):
            cfg = _cart("ppm", n, riemann=riem)
            F, _ = orc.fluxes(cfg, P, d)
            Q = np.flip(P, axis=d).copy()
            Q[1 + d] *= -1.0                      # u~^d
            Q[4 + d] *= -1.0                      # B^d
            G, _ = orc.fluxes(cfg, Q, d)
            G = np.flip(G, axis=d)                # face f of the mirror is face n_d - f
            sign = -np.ones(9)
            sign[1 + d] = 1.0                     # T^d_d is even, every other flux odd
            scale = np.abs(F).max(axis=(1, 2, 3))
            for q in range(9):
                if q == 4 + d:
                    continue                      # normal-field flux: zero on both sides
                assert np.all(np.abs(G[q] - sign[q] * F[q]) <= 1e-13 * scale[q]), (d, riem, q)


@pytest.mark.parametrize("riem", ["llf", "hll"])
def test_momentum_flux_at_rest_is_the_mean_pressure_of_the_face_states(riem):
    """With every velocity and field zero and uniform density, the momentum of both face states is
    zero, so either Riemann flux of T^d_d is the mean of the two face pressures (gam - 1) u / 2: the
    flux sweep must hand each face the states of its six cells taken in order."""
    n = (13, 11, 10)
    gam = 4.0 / 3.0
    rng = np.random.default_rng(9)
    P = np.zeros((8,) + n)
    P[0] = 1.0
    P[1] = 0.1 + rng.random(n) ** 3            # rough, with many local extrema
    for d in (1, 2, 3):
        cfg = orc.make_cfg(None, coords="cart", n1=n[0], n2=n[1], n3=n[2], gam=gam, cfl=0.4,
                           recon="ppm", riemann=riem)
        F, _ = orc.fluxes(cfg, P, d)
        u = np.moveaxis(P[1], d - 1, 0)
        Fm = np.moveaxis(F[1 + d], d - 1, 0)
        m = n[d - 1]
        for f in range(m + 1):                   # face between cells f-1 and f, periodic
            idx = [(f + o) % m for o in range(-3, 3)]
            for a in range(u.shape[1]):
                for b in range(u.shape[2]):
                    ql, qr = orc.ppm_face(u[idx, a, b])
                    want = 0.5 * (gam - 1.0) * (ql + qr)
                    assert abs(Fm[f, a, b] - want) <= 1e-15 * want, (d, f, a, b)


def test_grids_below_three_active_cells_are_refused_for_ppm():
    P = np.zeros((8, 8, 6, 2))
    P[0] = 1.0
    P[1] = 1.0
    with pytest.raises(RuntimeError):
        orc.step(_cart("ppm", (8, 6, 2)), P, 1)
    Q, _, nf, _ = orc.step(_cart("plm", (8, 6, 2)), P, 1)
    assert nf == 0 and np.isfinite(Q).all()


def test_ppm_torus_steps_keep_the_corner_divergence():
    """On the MKS torus (three ghost layers at the poles and radial edges) PPM steps run without a
    failed inversion and flux-CT still keeps the corner divergence of sqrt(-g) B at round-off."""
    from paper_2205_02484_amd.torus_init import TorusConfig, make_torus
    from tests.test_oracle_step import _centre_gdet, corner_divb
    c = TorusConfig(n1=32, n2=24, n3=1, r_out=40.0, gam=13.0 / 9.0, delta=0.04, seed=21, cfl=0.45)
    P0 = make_torus(c)
    cfg = orc.make_cfg(c, recon="ppm")
    P, dts, nfail, _ = orc.step(cfg, P0, 5)
    assert nfail == 0 and np.isfinite(P).all()
    gd = _centre_gdet(cfg)[..., None]
    dx = [(math.log(cfg.r_out) - math.log(cfg.r_in)) / c.n1, 1.0 / c.n2]
    bscale = np.abs(P0[5:7] * gd[None]).max() / min(dx)
    assert np.abs(corner_divb(P0, gd, dx, 2)).max() < 1e-13 * bscale
    assert np.abs(corner_divb(P, gd, dx, 2)).max() < 1e-13 * bscale
    Q, _, _, _ = orc.step(orc.make_cfg(c), P0, 5)
    assert np.abs(Q - P).max() > 0.0             # the reconstruction option is live on this path
