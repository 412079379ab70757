"""Seeded synthetic inputs: Fishbone-Moncrief tori in modified Kerr-Schild coordinates.

This module builds the primitive state P = (rho, u, u~1, u~2, u~3, B1, B2, B3) that both
the HIP stepper and the CPU oracle start from.  It is an input generator only: it carries its
own metric evaluation (Boyer-Lindquist for the torus, Kerr-Schild/MKS for the velocity
transform and the field normalisation) and shares no code with either side of the hot path.

Paper passages followed (arXiv 2205.02484):
  * torus in hydrostatic equilibrium after Fishbone & Moncrief (1976), set by (r_in, r_max),
    density normalised to rho_max = 1, pressure rescaled with it   -- Sec. "Physical models"
  * seed field A_phi = max(rho/rho_max - 0.2, 0), normalised by beta_0 -- same section, Eq. for A_phi
  * random perturbation of the gas pressure (4 per cent)              -- same section
  * MKS grid r = exp(X1) (hyper-exponential beyond r_br), theta(X2) refined towards the equator
                                                                      -- Sec. "Metric, numerical grid"
  * density/energy floors                                             -- Sec. "Flooring model"

The FM torus is built from the constant angular momentum l = u^t u_phi.  With the ZAMO
decomposition u_(phi)^2 = x one has x(1+x) = l^2 Sigma^2 Delta / (A^2 sin^2 theta), and the
first integral of the relativistic Euler equation for this rotation law is
      ln h = ln u^t - x - omega l  + const,      omega = 2 a r / A,
with the constant fixed by h = 1 at (r_in, pi/2).  l is u^t u_phi of the prograde circular
equatorial geodesic at r_max (Bardeen, Press & Teukolsky 1972), which puts the pressure
maximum at r_max.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class TorusConfig:
    """One synthetic torus workload (grid + physics + generator knobs)."""
    n1: int
    n2: int
    n3: int
    spin: float = 0.9375
    h: float = 0.3                 # MKS theta refinement
    r_out: float = 40.0            # outer radial grid edge
    r_in_grid: Optional[float] = None  # inner radial grid edge; default 0.98 r_horizon
    gam: float = 4.0 / 3.0         # adiabatic index the run evolves with
    gam_init: Optional[float] = None   # adiabatic index used to build the torus (default gam)
    r_in: float = 6.0              # torus inner edge
    r_max: float = 12.0            # torus pressure maximum
    beta: float = 100.0            # field normalisation target
    beta_mode: str = "max_ratio"   # "max_ratio": p_g,max/p_B,max ; "min": min(p_g/p_B)
    delta: float = 0.04            # relative amplitude of the u perturbation
    seed: int = 1
    rho_fl_coef: float = 1e-5
    rho_fl_pow: float = -0.5
    u_fl_coef: float = 1e-5 / 3.0
    u_fl_pow: float = -2.5
    fl_abs: float = 1e-20
    cfl: float = 0.45
    kappa: float = 1e-3            # polytropic constant (cancels after normalisation)
    field: bool = True
    r_br: float = 0.0              # > 0: radius where r(X1) turns hyper-exponential
    n_x: int = 4                   # power of the hyper-exponential term
    recon: str = "plm"             # face reconstruction: "plm" (MC limiter) or "ppm"
    pole_fix: int = 0              # cells next to each pole whose u~2 is interpolated to 0 (paper: 2)
    # optional structure of a magnetised funnel (off by default; checks of the magnetisation
    # ceilings and the Lorentz cap): a vertical field of this amplitude threading the whole grid,
    # atmosphere included (A_phi = b_vert r^2 sin^2(theta) / 2, added after the loop's beta
    # normalisation), and a radial outflow of Lorentz factor jet_lorentz in the jet_cells rows next
    # to each pole beyond twice the horizon radius
    b_vert: float = 0.0
    jet_lorentz: float = 0.0
    jet_cells: int = 4

    @property
    def r_horizon(self) -> float:
        return 1.0 + math.sqrt(1.0 - self.spin * self.spin)

    @property
    def r_grid_in(self) -> float:
        return self.r_in_grid if self.r_in_grid is not None else 0.98 * self.r_horizon

    @property
    def zones(self) -> int:
        return self.n1 * self.n2 * self.n3


# ----------------------------------------------------------------------------------------------
# grid (MKS) -- the generator's own copy of the coordinate map
# ----------------------------------------------------------------------------------------------

def r_of_x1(cfg: TorusConfig, X1):
    """(r, dr/dX1): r = exp(X1) below x_b = ln r_br, exp(X1 + (X1 - x_b)^n_x) beyond."""
    X1 = np.asarray(X1, dtype=np.float64)
    if cfg.r_br <= 0.0:
        r = np.exp(X1)
        return r, r
    xb = math.log(cfg.r_br)
    u = np.maximum(X1 - xb, 0.0)
    r = np.exp(X1 + u ** cfg.n_x)
    return r, r * (1.0 + cfg.n_x * u ** (cfg.n_x - 1))


def x1_range(cfg: TorusConfig):
    """(X1 at r_grid_in, X1 at r_out); the latter by bisection when the map is hyper-exponential."""
    lo_x = math.log(cfg.r_grid_in)
    hi = math.log(cfg.r_out)
    if cfg.r_br <= 0.0 or cfg.r_out <= cfg.r_br:
        return lo_x, hi
    lo = math.log(cfg.r_br)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if float(r_of_x1(cfg, mid)[0]) < cfg.r_out:
            lo = mid
        else:
            hi = mid
    return lo_x, 0.5 * (lo + hi)


def mks_centres(cfg: TorusConfig, i: np.ndarray, j: np.ndarray):
    """(r, theta, dtheta/dX2) at possibly fractional cell indices (i, j); centre of cell 0 is 0."""
    x1lo, x1hi = x1_range(cfg)
    dx1 = (x1hi - x1lo) / cfg.n1
    dx2 = 1.0 / cfg.n2
    X1 = x1lo + (np.asarray(i, dtype=np.float64) + 0.5) * dx1
    X2 = (np.asarray(j, dtype=np.float64) + 0.5) * dx2
    r = r_of_x1(cfg, X1)[0]
    th = np.pi * X2 + 0.5 * (1.0 - cfg.h) * np.sin(2.0 * np.pi * X2)
    dth = np.pi * (1.0 + (1.0 - cfg.h) * np.cos(2.0 * np.pi * X2))
    return r, th, dth


def _bl_functions(a, r, th):
    c = np.cos(th)
    s = np.sin(th)
    sig = r * r + a * a * c * c
    dlt = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - a * a * dlt * s * s
    return sig, dlt, big_a, s


def circular_orbit_ell(a: float, r: float) -> float:
    """l = u^t u_phi of the prograde circular equatorial geodesic at BL radius r."""
    sr = math.sqrt(r)
    den = r ** 0.75 * math.sqrt(r ** 1.5 - 3.0 * sr + 2.0 * a)
    e = (r ** 1.5 - 2.0 * sr + a) / den
    ang = (r * r - 2.0 * a * sr + a * a) / den
    sig = r * r
    dlt = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - a * a * dlt
    ut = (big_a * e - 2.0 * a * r * ang) / (sig * dlt)
    return ut * ang


def _fm_pieces(a, ell, r, th):
    """ln u^t - x - omega*l, together with u^t and u^phi (BL) of the torus rotation law."""
    sig, dlt, big_a, s = _bl_functions(a, r, th)
    s2 = np.maximum(s * s, 1e-300)
    x = 0.5 * (-1.0 + np.sqrt(1.0 + 4.0 * ell * ell * sig * sig * dlt / (big_a * big_a * s2)))
    alpha = np.sqrt(sig * dlt / big_a)
    lor = np.sqrt(1.0 + x)
    omega = 2.0 * a * r / big_a
    ut = lor / alpha
    gpp = big_a * s2 / sig
    uphi = lor * omega / alpha + np.sqrt(x) / np.sqrt(gpp)
    return np.log(ut) - x - omega * ell, ut, uphi


def fm_lnh(a, ell, r_in, r, th):
    """ln h of the torus, zero at (r_in, pi/2)."""
    val, _, _ = _fm_pieces(a, ell, r, th)
    ref, _, _ = _fm_pieces(a, ell, np.float64(r_in), np.float64(np.pi / 2))
    return val - ref


def fm_torus_2d(cfg: TorusConfig, i: np.ndarray, j: np.ndarray):
    """Unnormalised torus (rho, u, u^t, u^phi BL) at cell indices (i, j); zeros outside."""
    a = cfg.spin
    gam = cfg.gam_init if cfg.gam_init is not None else cfg.gam
    ell = circular_orbit_ell(a, cfg.r_max)
    r, th, _ = mks_centres(cfg, i, j)
    with np.errstate(invalid="ignore", divide="ignore"):
        lnh = fm_lnh(a, ell, cfg.r_in, r, th)
        _, ut, uphi = _fm_pieces(a, ell, r, th)
    inside = (r >= cfg.r_in) & np.isfinite(lnh) & (lnh > 0.0)
    hh = np.where(inside, np.exp(np.where(inside, lnh, 0.0)), 1.0)
    rho = np.where(inside, ((hh - 1.0) * (gam - 1.0) / (cfg.kappa * gam)) ** (1.0 / (gam - 1.0)), 0.0)
    u = np.where(inside, cfg.kappa * rho ** gam / (gam - 1.0), 0.0)
    ut = np.where(inside, ut, 0.0)
    uphi = np.where(inside, uphi, 0.0)
    return rho, u, ut, uphi, inside


def mks_drdx(cfg: TorusConfig, i: np.ndarray):
    """dr/dX1 at (possibly fractional) radial cell indices i."""
    x1lo, x1hi = x1_range(cfg)
    return r_of_x1(cfg, x1lo + (np.asarray(i, dtype=np.float64) + 0.5) * (x1hi - x1lo) / cfg.n1)[1]


def _mks_metric_cov(cfg: TorusConfig, r, th, dth, dr=None):
    """Non-zero MKS covariant components (tt, t1, t3, 11, 13, 22, 33) and sqrt(-g); dr = dr/dX1
    (default r, the plain exponential map)."""
    a = cfg.spin
    c = np.cos(th)
    s = np.sin(th)
    s2 = s * s
    sig = r * r + a * a * c * c
    z = 2.0 * r / sig
    if dr is None:
        dr = r
    g = {
        "tt": -(1.0 - z),
        "t1": z * dr,
        "t3": -a * z * s2,
        "11": (1.0 + z) * dr * dr,
        "13": -a * (1.0 + z) * s2 * dr,
        "22": sig * dth * dth,
        "33": s2 * (sig + a * a * (1.0 + z) * s2),
    }
    gdet = sig * np.abs(s) * dr * dth
    return g, gdet, sig


def _bsq(cfg, r, th, dth, ut1, ut3, B1, B2, dr=None):
    """b^2 for u~ = (u~1, 0, u~3) and B = (B1, B2, 0) (generator-side helper)."""
    if dr is None:
        dr = r
    g, _, sig = _mks_metric_cov(cfg, r, th, dth, dr)
    # lapse and shift from the KS inverse metric carried to MKS: g^{tt}=-(1+2r/Sigma),
    # g^{t1} = (2r/Sigma)/(dr/dX1)
    gcon_tt = -(1.0 + 2.0 * r / sig)
    gcon_t1 = 2.0 / sig if cfg.r_br <= 0.0 else (2.0 * r / sig) / dr
    alpha = 1.0 / np.sqrt(-gcon_tt)
    lor = np.sqrt(1.0 + g["11"] * ut1 * ut1 + 2.0 * g["13"] * ut1 * ut3 + g["33"] * ut3 * ut3)
    ut = lor / alpha
    u1 = ut1 - lor * alpha * gcon_t1
    u3 = ut3
    u_1 = g["t1"] * ut + g["11"] * u1 + g["13"] * u3
    bt = B1 * u_1
    b1 = (B1 + bt * u1) / ut
    b2 = B2 / ut
    b3 = (bt * u3) / ut
    bsq = (g["tt"] * bt * bt + 2 * g["t1"] * bt * b1 + 2 * g["t3"] * bt * b3 + g["11"] * b1 * b1
           + 2 * g["13"] * b1 * b3 + g["22"] * b2 * b2 + g["33"] * b3 * b3)
    return bsq


def make_torus(cfg: TorusConfig) -> np.ndarray:
    """Primitive state P[8][n1][n2][n3] (float64, C order, phi fastest) for `cfg`."""
    n1, n2, n3 = cfg.n1, cfg.n2, cfg.n3
    a = cfg.spin
    ii, jj = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    rho, u, ut, uphi, inside = fm_torus_2d(cfg, ii, jj)
    if not inside.any():
        raise ValueError("torus does not intersect the grid")
    rho_max = rho.max()
    rho = rho / rho_max
    u = u / rho_max

    r, th, dth = mks_centres(cfg, ii, jj)
    dr = mks_drdx(cfg, ii)
    g, gdet, sig = _mks_metric_cov(cfg, r, th, dth, dr)
    # MKS contravariant velocity (u^r = u^theta = 0 in the torus, u^phi unchanged by BL->KS)
    u1 = np.zeros_like(ut)
    u3 = uphi
    # u~^i = u^i - u^t g^{ti}/g^{tt}; with KS g^{tt} = -(1+2r/Sigma), g^{t1}_MKS = (2r/Sigma)/r
    gcon_tt = -(1.0 + 2.0 * r / sig)
    gcon_t1 = (2.0 * r / sig) / (r if cfg.r_br <= 0.0 else dr)
    ut1 = np.where(inside, u1 - ut * gcon_t1 / gcon_tt, 0.0)
    ut3 = np.where(inside, u3, 0.0)

    B1 = np.zeros_like(rho)
    B2 = np.zeros_like(rho)
    if cfg.field:
        # A_phi at cell corners (i-1/2, j-1/2): average of the four adjacent cell densities
        ie, je = np.meshgrid(np.arange(-1, n1 + 1), np.arange(-1, n2 + 1), indexing="ij")
        rho_e = fm_torus_2d(cfg, ie, je)[0] / rho_max
        rc = 0.25 * (rho_e[:-1, :-1] + rho_e[1:, :-1] + rho_e[:-1, 1:] + rho_e[1:, 1:])
        aphi = np.maximum(rc - 0.2, 0.0)      # shape (n1+1, n2+1), corner (i,j) = lower-left of cell (i,j)
        x1lo, x1hi = x1_range(cfg)
        dx1 = (x1hi - x1lo) / n1
        dx2 = 1.0 / n2
        B1 = (aphi[:-1, 1:] + aphi[1:, 1:] - aphi[:-1, :-1] - aphi[1:, :-1]) / (2.0 * dx2 * gdet)
        B2 = -(aphi[1:, :-1] + aphi[1:, 1:] - aphi[:-1, :-1] - aphi[:-1, 1:]) / (2.0 * dx1 * gdet)

    # broadcast to 3D, then perturb u inside the torus (one uniform draw per interior cell, C order)
    shape = (n1, n2, n3)
    rng = np.random.default_rng(cfg.seed)
    xi = rng.random(shape)
    rho3 = np.broadcast_to(rho[:, :, None], shape).copy()
    u3d = np.broadcast_to(u[:, :, None], shape).copy()
    ins3 = np.broadcast_to(inside[:, :, None], shape)
    u3d = np.where(ins3, u3d * (1.0 + cfg.delta * (2.0 * xi - 1.0)), u3d)

    if cfg.field:
        gam = cfg.gam
        bsq = _bsq(cfg, r, th, dth, ut1, ut3, B1, B2, dr)
        pb = 0.5 * bsq
        pg = (gam - 1.0) * u3d
        pb3 = np.broadcast_to(pb[:, :, None], shape)
        if cfg.beta_mode == "max_ratio":
            beta_cur = pg[ins3].max() / pb.max()
        elif cfg.beta_mode == "min":
            sel = ins3 & (pb3 > 0.0)
            beta_cur = (pg[sel] / pb3[sel]).min()
        else:
            raise ValueError(f"unknown beta_mode {cfg.beta_mode}")
        scale = math.sqrt(beta_cur / cfg.beta)
        B1 = B1 * scale
        B2 = B2 * scale

    if cfg.b_vert != 0.0:
        ie, je = np.meshgrid(np.arange(n1 + 1) - 0.5, np.arange(n2 + 1) - 0.5, indexing="ij")
        rc_, thc_, _ = mks_centres(cfg, ie, je)
        av = 0.5 * cfg.b_vert * rc_ * rc_ * np.sin(thc_) ** 2
        x1lo, x1hi = x1_range(cfg)
        dx1 = (x1hi - x1lo) / n1
        dx2 = 1.0 / n2
        B1 = B1 + (av[:-1, 1:] + av[1:, 1:] - av[:-1, :-1] - av[1:, :-1]) / (2.0 * dx2 * gdet)
        B2 = B2 - (av[1:, :-1] + av[1:, 1:] - av[:-1, :-1] - av[:-1, 1:]) / (2.0 * dx1 * gdet)
    if cfg.jet_lorentz > 1.0:
        jet = (r > 2.0 * cfg.r_horizon) & ((jj < cfg.jet_cells) | (jj >= n2 - cfg.jet_cells)) & ~inside
        ut1 = np.where(jet, math.sqrt(cfg.jet_lorentz ** 2 - 1.0) / np.sqrt(g["11"]), ut1)

    # floors (the atmosphere starts at the floor values with u~ = 0 outside a jet)
    r3 = np.broadcast_to(r[:, :, None], shape)
    rho_fl = np.maximum(cfg.fl_abs, cfg.rho_fl_coef * r3 ** cfg.rho_fl_pow)
    u_fl = np.maximum(cfg.fl_abs, cfg.u_fl_coef * r3 ** cfg.u_fl_pow)
    rho3 = np.maximum(rho3, rho_fl)
    u3d = np.maximum(u3d, u_fl)

    P = np.empty((8,) + shape, dtype=np.float64)
    P[0] = rho3
    P[1] = u3d
    P[2] = np.broadcast_to(ut1[:, :, None], shape)
    P[3] = 0.0
    P[4] = np.broadcast_to(ut3[:, :, None], shape)
    P[5] = np.broadcast_to(B1[:, :, None], shape)
    P[6] = np.broadcast_to(B2[:, :, None], shape)
    P[7] = 0.0
    return np.ascontiguousarray(P)
