"""Seeded sweep of run configurations through the HIP path against the oracle, one RK2 step each
with equal method-code maps: grid sizes drawn ragged (2D and 3D, phi counts on both metric paths),
spin, adiabatic index, Riemann solver, reconstruction, the polar u~2 interpolation and the
hyper-exponential radial map, with the seeded torus generator.

The bar of each draw comes from the conditioning of its own state, measured on the oracle alone:
rho, the largest change of the oracle's one-step result when its input is perturbed by 1e-15
relative noise (two trials), and sigma, its change when the inversion tolerance goes from 1e-10
to 1e-14.  Two correct codes that round differently differ by a few times rho, and by up to sigma
where the Newton-Raphson stopping rule decides.  Generic random tori give rho from ~1e-13 to a few
1e-12 (cells in low-density polar regions), so the bar is max(1e-12, 5 rho, 2 sigma); a draw whose
bar would exceed 1e-10 is skipped, and most draws must run.  An indexing or formula error moves
results by far more than that.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import TorusConfig, make_torus
from tests._parity import assert_parity, max_rel_err

pytestmark = pytest.mark.gpu

NDRAW = 24


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02484_amd import grmhd
    grmhd.load()
    return grmhd


def _draw(seed):
    rng = np.random.default_rng(1000 + seed)
    recon = str(rng.choice(["plm", "ppm"]))
    n1 = int(rng.integers(12, 49))
    n2 = int(rng.integers(8, 33))
    n3 = int(rng.choice([1, 3, 5, 8, 13, 20, 64]))
    hyper = bool(rng.random() < 0.3)
    r_out = float(rng.uniform(30.0, 80.0)) if not hyper else 2000.0
    cfg = TorusConfig(n1=n1, n2=n2, n3=n3, spin=float(rng.uniform(0.0, 0.98)),
                      gam=float(rng.choice([4.0 / 3.0, 13.0 / 9.0, 5.0 / 3.0])), r_out=r_out,
                      r_br=200.0 if hyper else 0.0, n_x=4, delta=0.04, seed=int(rng.integers(1, 1000)),
                      cfl=float(rng.uniform(0.3, 0.8)), recon=recon,
                      pole_fix=int(rng.choice([0, 2])) if n2 >= 5 else 0)
    riemann = str(rng.choice(["llf", "hll"]))
    return cfg, riemann


def _bar(cfg, P, riemann, seed):
    ocfg = orc.make_cfg(cfg, riemann=riemann)
    a, *_ = orc.step(ocfg, P, 1)
    rng = np.random.default_rng(seed)
    rho = max(max_rel_err(orc.step(ocfg, P * (1.0 + 1e-15 * rng.standard_normal(P.shape)), 1)[0], a)
              for _ in range(2))
    b, *_ = orc.step(orc.make_cfg(cfg, riemann=riemann, c2p_tol=1e-14), P, 1)
    sigma = max_rel_err(b, a)
    return max(1e-12, 5.0 * rho, 2.0 * sigma)


def test_random_configurations_match_the_oracle(G):
    ran = 0
    for seed in range(NDRAW):
        cfg, riemann = _draw(seed)
        P = make_torus(cfg)
        bar = _bar(cfg, P, riemann, seed)
        if bar > 1e-10:
            continue
        tag = (seed, cfg.n1, cfg.n2, cfg.n3, cfg.recon, riemann, cfg.pole_fix, cfg.r_br, bar)
        print("draw", tag, flush=True)
        ocfg = orc.make_cfg(cfg, riemann=riemann)
        Po, dto, nfo, co = orc.step(ocfg, P, 1)
        ctx = G.Context(cfg, P, riemann=riemann)
        dtg = ctx.step()
        Pg = ctx.get_prims()
        cg = ctx.get_codes()
        ctx.close()
        assert dtg == pytest.approx(dto[0], rel=1e-13), tag
        assert np.array_equal(cg, co), tag
        assert_parity(Pg, Po, bar)
        ran += 1
    assert ran >= NDRAW * 3 // 4, ran
