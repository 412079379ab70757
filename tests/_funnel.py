"""Workloads on which the magnetisation ceilings and the Lorentz cap of Sec. 2.4 act: the seeded
torus plus a vertical field threading the low-density atmosphere (b^2/rho above 50 and b^2/u above
2500 there) and, in the second kind, a radial polar outflow faster than a lowered Lorentz cap.

  "ceil"  paper thresholds (b^2/rho < 50, b^2/u < 2500, Gamma <= 50), b_vert = 0.02: both
          ceilings act in most atmosphere cells
  "cap"   b_vert = 0.005, polar outflow at Gamma = 6 with the cap lowered to 5: the energy
          ceiling and the cap act (and, in 2D, the density ceiling)

Each on the 2D 64^2 torus and on 3D tori of both metric paths (n3 = 16: per-lane metric;
n3 = 64: a wave's cells share (r, theta)).  A Lorentz factor near the paper's cap of 50 makes the
energy equation so ill-conditioned (~Gamma^2 (rho + b^2)/p) that the oracle's own one-step result
moves by ~1e-9 under 1e-15 input noise, so the cap's branch is exercised at a lowered threshold.
"""
import dataclasses

from paper_2205_02484_amd.torus_init import TorusConfig
from paper_2205_02484_amd.workloads import torus_2d_64

KINDS = {"ceil": dict(b_vert=0.02), "cap": dict(b_vert=0.005, jet_lorentz=6.0)}
OVER = {"ceil": {}, "cap": dict(gamma_max=5.0)}
# limiters each (grid, kind) must show acting on the oracle after one step
ACTS = {
    ("2d", "ceil"): ("bsq_rho_max", "bsq_u_max"), ("2d", "cap"): ("bsq_rho_max", "bsq_u_max", "gamma_max"),
    ("gen", "ceil"): ("bsq_rho_max", "bsq_u_max"), ("gen", "cap"): ("bsq_u_max", "gamma_max"),
    ("uni", "ceil"): ("bsq_rho_max", "bsq_u_max"), ("uni", "cap"): ("bsq_u_max", "gamma_max"),
}


def funnel(grid, kind):
    if grid == "2d":
        base = torus_2d_64()
        jc = 4
    elif grid == "gen":
        base = TorusConfig(n1=40, n2=24, n3=16, r_out=60.0, gam=13.0 / 9.0, delta=0.04, seed=5, cfl=0.45)
        jc = 3
    else:
        base = TorusConfig(n1=24, n2=16, n3=64, r_out=60.0, gam=5.0 / 3.0, delta=0.04, seed=6, cfl=0.45)
        jc = 2
    return dataclasses.replace(base, jet_cells=jc, **KINDS[kind]), OVER[kind]
