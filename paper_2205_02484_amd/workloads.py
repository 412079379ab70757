"""The synthetic torus workloads the stepper is measured and checked on.

Each entry names a grid and the physics of one Fishbone-Moncrief torus run.  The sizes follow
the resolutions the paper evolves (256^3-class 3D grids, Sec. "Physical models", Table 1) plus a
small 2D case that the CPU oracle finishes in seconds.
"""
from __future__ import annotations

from .torus_init import TorusConfig


def torus_2d_64() -> TorusConfig:
    """2D 64x64 torus, a=0.9375, gamma=4/3, r in [0.98 r_h, 40], min-beta 100, CFL 0.8."""
    return TorusConfig(n1=64, n2=64, n3=1, spin=0.9375, h=0.3, r_out=40.0, gam=4.0 / 3.0,
                       r_in=6.0, r_max=12.0, beta=100.0, beta_mode="min", delta=0.02, seed=1,
                       rho_fl_coef=1e-4, rho_fl_pow=-1.5, u_fl_coef=1e-6, u_fl_pow=-2.5,
                       cfl=0.8)


def torus_128x64x64() -> TorusConfig:
    """3D 128x64x64 torus to r_out=200, gamma=13/9, beta_0=100, 4 per cent perturbation."""
    return TorusConfig(n1=128, n2=64, n3=64, spin=0.9375, h=0.3, r_out=200.0, gam=13.0 / 9.0,
                       r_in=6.0, r_max=12.0, beta=100.0, beta_mode="max_ratio", delta=0.04,
                       seed=2, cfl=0.45)


def torus_256cubed() -> TorusConfig:
    """3D 256^3 torus to r_out=1000, gamma=5/3, r_in=20, r_max=41, beta_0=100."""
    return TorusConfig(n1=256, n2=256, n3=256, spin=0.9375, h=0.3, r_out=1000.0, gam=5.0 / 3.0,
                       r_in=20.0, r_max=41.0, beta=100.0, beta_mode="max_ratio", delta=0.04,
                       seed=3, cfl=0.45)


WORKLOADS = {
    "torus2d_64x64": torus_2d_64,
    "torus3d_128x64x64": torus_128x64x64,
    "torus3d_256x256x256": torus_256cubed,
}
