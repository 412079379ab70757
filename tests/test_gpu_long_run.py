"""The 128x64x64 torus (r_out = 200, gamma = 13/9, beta_0 = 100, 4 per cent perturbation) advanced
1000 RK2 steps at CFL 0.45 on the GPU, in the graph-replayed launch chain, with PLM and with PPM
plus the polar u~2 interpolation: the state stays finite with no cell left unfixed, the corner
divergence of sqrt(-g) B that flux-CT preserves (Sec. 2.2) stays at round-off, and the torus is
still in place.  There is no oracle run at this length (the
CPU would need minutes); the properties checked hold for any correct step.
"""
import math
import time

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import make_torus
from paper_2205_02484_amd.workloads import torus_128x64x64
from tests.test_oracle_step import _centre_gdet, corner_divb

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02484_amd import grmhd
    grmhd.load()
    return grmhd


@pytest.mark.parametrize("variant", ["plm", "ppm_polefix"])
def test_thousand_steps_128x64x64_stable_and_divergence_free(G, variant):
    c = torus_128x64x64()
    if variant == "ppm_polefix":
        c.recon, c.pole_fix = "ppm", 2
    P0 = make_torus(c)
    cfg = orc.make_cfg(c)
    gd = _centre_gdet(cfg)[..., None]
    dx = [(math.log(cfg.r_out) - math.log(cfg.r_in)) / c.n1, 1.0 / c.n2, 2.0 * math.pi / c.n3]
    d0 = corner_divb(P0, gd, dx, 3)
    bscale = np.abs(P0[5:8] * gd[None]).max() / min(dx)
    assert np.abs(d0).max() < 1e-13 * bscale

    ctx = G.Context(c, P0)
    ctx.steps(1)
    ctx.get_time()
    t0 = time.perf_counter()
    ctx.steps(999)
    t, nstep, nfail = ctx.get_time()
    el = time.perf_counter() - t0
    P1 = ctx.get_prims()
    mdot, phib = ctx.diag()
    ctx.close()
    print(f"1000 steps of 128x64x64 ({variant}): t = {t:.3f} M, {999 * c.n1 * c.n2 * c.n3 / el:.3e} zone-updates/s")

    assert nstep == 1000 and t > 0.0
    assert np.isfinite(P1).all()
    assert nfail == 0
    assert (P1[0] > 0.0).all() and (P1[1] > 0.0).all()
    d1 = corner_divb(P1, gd, dx, 3)
    assert np.abs(d1).max() < 1e-11 * bscale
    # the torus is still there: its density maximum moved little over a small fraction of an orbit
    assert 0.5 < P1[0].max() / P0[0].max() < 1.5
    assert math.isfinite(mdot) and math.isfinite(phib)


def test_thousand_steps_2d_64_torus_keeps_corner_divergence(G):
    """The 64^2 torus at CFL 0.8 for 1000 steps: corner div of sqrt(-g) B stays at round-off."""
    from paper_2205_02484_amd.workloads import torus_2d_64
    c = torus_2d_64()
    P0 = make_torus(c)
    cfg = orc.make_cfg(c)
    gd = _centre_gdet(cfg)[..., None]
    dx = [(math.log(cfg.r_out) - math.log(cfg.r_in)) / c.n1, 1.0 / c.n2]
    bscale = np.abs(P0[5:7] * gd[None]).max() / min(dx)
    ctx = G.Context(c, P0)
    ctx.steps(1000)
    t, nstep, nfail = ctx.get_time()
    P1 = ctx.get_prims()
    ctx.close()
    d1 = corner_divb(P1, gd, dx, 2)
    print(f"64^2 torus, 1000 steps to t = {t:.2f} M: max corner div / scale = {np.abs(d1).max() / bscale:.2e}")
    assert nstep == 1000 and np.isfinite(P1).all()
    assert np.abs(d1).max() < 1e-13 * bscale
