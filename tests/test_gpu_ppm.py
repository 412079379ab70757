"""Parity of the PPM reconstruction (Colella & Woodward 1984, the upgrade of PLM that Sec. 2.2
names) on the HIP path with the oracle's, through the C ABI, to the same bars as PLM: face fluxes to
1e-12 of each component's largest value, 1e-12 after one RK2 step and 1e-8 after ten (the device
divides the slope difference by 6 as a multiply by 1/3 of the half slopes, a last-bit difference;
the CW84 limiter is continuous, so such differences stay at round-off).  Cases: the 2D and 3D torus
on both metric paths (n3 % 64 == 0 and not), ragged sizes, both Riemann solvers, the slow path (the
entropy inversion everywhere), a flat periodic box and line, the hyper-exponential grid, a batch
mixing PLM and PPM runs, and the size checks.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import TorusConfig, make_torus
from paper_2205_02484_amd.workloads import torus_2d_64, torus_128x64x64
from tests._parity import assert_parity, scaled_abs_err
from tests.test_gpu_parity import _flat_box, _run_both, _small3d

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02484_amd import grmhd
    grmhd.load()
    return grmhd


def _ppm(c):
    c.recon = "ppm"
    return c


@pytest.mark.parametrize("which", ["2d", "3d", "3d_uniform"])
def test_ppm_face_fluxes_match_oracle(G, which):
    if which == "2d":
        c = _ppm(torus_2d_64())
    elif which == "3d":
        c = _ppm(_small3d())
    else:
        c = _ppm(_small3d(n1=24, n2=16, n3=64))
    P = make_torus(c)
    if c.n3 > 1:
        P[7] = 0.3 * P[5] - 0.1 * P[6]           # a toroidal share, so X3 states are not trivial
        P[4] *= 1.0 + 0.05 * np.sin(np.arange(c.n3) * 2 * np.pi / c.n3 * 3)[None, None, :]
    ctx = G.Context(c, P)
    cfg = orc.make_cfg(c)
    assert cfg.recon == 1
    for d in (1, 2, 3) if c.n3 > 1 else (1, 2):
        Fg, cg = ctx.debug_fluxes(d)
        Fo, co = orc.fluxes(cfg, P, d)
        assert scaled_abs_err(Fg, Fo) < 1e-12, d
        assert cg == pytest.approx(co, rel=1e-13)
        # the reconstruction is live: PLM fluxes differ
        Fl, _ = orc.fluxes(orc.make_cfg(c, recon="plm"), P, d)
        assert scaled_abs_err(Fl, Fo) > 1e-8, d
    ctx.close()


def test_ppm_one_and_ten_steps_2d_torus(G):
    c = _ppm(torus_2d_64())
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, (t, ns, nf, nfo) = _run_both(G, c, P, 1)
    assert dtg[0] == pytest.approx(dto[0], rel=1e-13)
    assert np.array_equal(cg, co)
    assert nf == nfo == 0
    assert_parity(Pg, Po, 1e-12)
    Pg, Po, dtg, dto, cg, co, (t, ns, nf, nfo) = _run_both(G, c, P, 10)
    assert np.allclose(dtg, dto, rtol=1e-10)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-8)


@pytest.mark.parametrize("riemann", ["llf", "hll"])
def test_ppm_small_3d_torus_steps(G, riemann):
    c = _ppm(_small3d())
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1, riemann=riemann)
    assert_parity(Pg, Po, 1e-12)
    assert np.array_equal(cg, co)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 10, riemann=riemann)
    assert_parity(Pg, Po, 1e-8)
    assert np.allclose(dtg, dto, rtol=1e-10)


def test_ppm_ragged_3d_torus(G):
    """Odd sizes that fill no tile evenly; n3 = 3 is the fewest PPM allows along phi."""
    for n in ((37, 19, 13), (21, 11, 3)):
        c = _ppm(_small3d(n1=n[0], n2=n[1], n3=n[2], seed=23))
        P = make_torus(c)
        Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
        assert_parity(Pg, Po, 1e-12)
        Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 10)
        assert_parity(Pg, Po, 1e-8)


def test_ppm_uniform_metric_path_128x64x64(G):
    """n3 % 64 == 0: the flux kernels take the wave-uniform metric path."""
    c = _ppm(torus_128x64x64())
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
    assert dtg[0] == pytest.approx(dto[0], rel=1e-13)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)


@pytest.mark.parametrize("recon", ["plm", "ppm"])
def test_slow_path_entropy_fluxes_follow_the_reconstruction(G, recon):
    """With the entropy inversion taken by every magnetised cell, the slow path recomputes the
    entropy fluxes of its faces; they must use the run's reconstruction."""
    c = _small3d(n1=24, n2=16, n3=8, recon=recon)
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 2, beta_entropy=1e12)
    assert (co == 2).sum() > 100
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)


def test_ppm_flat_periodic_box_and_line(G):
    c, P = _flat_box()
    c.recon = "ppm"
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 3)
    assert_parity(Pg, Po, 1e-12)
    assert np.allclose(dtg, dto, rtol=1e-13)
    c, P = _flat_box((64, 1, 1))
    c.recon = "ppm"
    Pg, Po, *_ = _run_both(G, c, P, 5)
    assert_parity(Pg, Po, 1e-12)


def test_ppm_on_the_hyperexponential_grid(G):
    c = TorusConfig(n1=48, n2=24, n3=16, r_out=5000.0, r_br=400.0, n_x=4, gam=13.0 / 9.0, delta=0.04,
                    seed=17, cfl=0.45, recon="ppm")
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
    assert_parity(Pg, Po, 1e-12)
    assert np.array_equal(cg, co)


def test_batch_mixing_plm_and_ppm_runs_matches_solo_runs(G):
    cfgs = [_small3d(n1=24, n2=16, n3=8, seed=3),
            _small3d(n1=24, n2=16, n3=8, seed=3, recon="ppm"),
            _small3d(n1=20, n2=12, n3=64, seed=4, recon="ppm"),
            _small3d(n1=20, n2=12, n3=64, seed=5)]
    steps = [4, 4, 3, 5]
    solo = []
    for c, n in zip(cfgs, steps):
        ctx = G.Context(c, make_torus(c))
        ctx.steps(n)
        solo.append((ctx.get_prims(), ctx.get_time()))
        ctx.close()
    b = G.Batch()
    ids = [b.admit(c, make_torus(c), n) for c, n in zip(cfgs, steps)]
    done = set()
    for _ in range(10):
        b.advance(1)
        done |= set(b.poll())
    assert done == set(ids)
    for jid, (Ps, (ts, ns, _)) in zip(ids, solo):
        Pb, tb, nb = b.fetch(jid)
        assert nb == ns and tb == ts
        assert np.array_equal(Pb, Ps)
    b.close()
    assert not np.array_equal(solo[0][0], solo[1][0])   # same torus, the two methods differ


def test_ppm_size_checks(G):
    c = _small3d(n1=24, n2=16, n3=2, recon="ppm")
    with pytest.raises(G.GrmhdError) as ei:
        G.Context(c, make_torus(c))
    assert ei.value.code == G.EINVAL
    ctx = G.Context(_small3d(n1=24, n2=16, n3=2), make_torus(_small3d(n1=24, n2=16, n3=2)))
    ctx.close()
    c = _small3d(n1=24, n2=16, n3=4)
    P = make_torus(c)
    p = G.make_params(c)
    p.recon = 7
    import ctypes
    out = ctypes.c_void_p()
    rc = G.load().grmhd_init(ctypes.byref(out), ctypes.byref(G.make_grid(c)), ctypes.byref(p),
                             np.ascontiguousarray(P).ctypes.data, 0, None)
    assert rc == G.EINVAL and not out.value
