"""Parity of the HIP path (through the C ABI) with the FP64 oracle on the same seeded inputs.

Tolerances: the per-cell metric of tests/_parity.py must stay below 1e-12 after one RK2 step and
below 1e-8 after ten.  Face fluxes agree to 1e-12 of each component's largest value: in the torus
the Lax-Friedrichs flux is a small difference of terms (sqrt(-g) rho u^t ~ 3e3 times a wave
speed ~ 5e-3) that can be ~40 times larger than the flux itself, so a per-face relative bound would
measure that cancellation, not the code.  Method-code maps must be equal (no cell of these
workloads sits on a beta-switch or floor threshold).
"""
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import TorusConfig, make_torus
from paper_2205_02484_amd.workloads import torus_2d_64, torus_128x64x64, torus_256cubed
from tests._parity import assert_parity, max_rel_err, rel_err, scaled_abs_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02484_amd import grmhd
    grmhd.load()
    return grmhd


def _small3d(**kw):
    base = dict(n1=40, n2=24, n3=16, r_out=60.0, gam=13.0 / 9.0, delta=0.04, seed=11, cfl=0.45)
    base.update(kw)
    return TorusConfig(**base)


def _flat_box(n=(12, 10, 8)):
    class C:
        pass
    c = C()
    c.coords = "cart"
    c.n1, c.n2, c.n3 = n
    c.gam = 4.0 / 3.0
    c.cfl = 0.4
    c.xmin, c.xmax = (0.0, 0.0, 0.0), (1.0, 1.0, 1.0)
    x = [(np.arange(m) + 0.5) / m for m in n]
    X, Y, Z = np.meshgrid(*x, indexing="ij")
    s = lambda kx, ky, kz, ph: np.sin(2 * np.pi * (kx * X + ky * Y + kz * Z) + ph)
    P = np.empty((8,) + tuple(n))
    P[0] = 1.0 + 0.3 * s(1, 1, 0, 0.1)
    P[1] = 0.5 + 0.2 * s(0, 1, 1, 0.7)
    P[2] = 0.3 * s(1, 0, 1, 0.2)
    P[3] = 0.2 * s(0, 1, 1, 1.1)
    P[4] = 0.25 * s(1, 1, 1, 2.0)
    P[5] = 0.4 + 0.2 * s(0, 1, 1, 0.3)
    P[6] = 0.1 + 0.2 * s(1, 0, 1, 0.9)
    P[7] = -0.2 + 0.1 * s(1, 1, 0, 1.4)
    return c, P


@pytest.mark.parametrize("which", ["2d", "3d"])
def test_face_fluxes_match_oracle(G, which):
    c = torus_2d_64() if which == "2d" else _small3d()
    P = make_torus(c)
    ctx = G.Context(c, P)
    cfg = orc.make_cfg(c)
    for d in (1, 2, 3) if c.n3 > 1 else (1, 2):
        Fg, cg = ctx.debug_fluxes(d)
        Fo, co = orc.fluxes(cfg, P, d)
        assert scaled_abs_err(Fg, Fo) < 1e-12, d
        assert cg == pytest.approx(co, rel=1e-13)
    ctx.close()


def test_prim2cons_and_inversion_match_oracle(G):
    c = _small3d()
    P = make_torus(c)
    cfg = orc.make_cfg(c)
    ctx = G.Context(c, P)
    Ug = ctx.prim2cons(P)
    Uo = orc.prim2cons(cfg, P)
    assert scaled_abs_err(Ug, Uo) < 1e-14
    rng = np.random.default_rng(5)
    guess = P * (1 + 0.01 * rng.uniform(-1, 1, size=P.shape))
    Pg, cg = ctx.cons2prim(Uo, guess)
    Po, co = orc.cons2prim(cfg, Uo, guess)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)
    ctx.close()


@pytest.mark.parametrize("mode", ["brent", "entropy"])
def test_fallback_inversions_match_oracle(G, mode):
    over = {"c2p_maxit": 0} if mode == "brent" else {"beta_entropy": 1e12}
    c = _small3d()
    P = make_torus(c)
    cfg = orc.make_cfg(c, **over)
    ctx = G.Context(c, P, **over)
    Uo = orc.prim2cons(cfg, P)
    Pg, cg = ctx.cons2prim(Uo, P)
    Po, co = orc.cons2prim(cfg, Uo, P)
    assert np.array_equal(cg, co)
    # cells without field keep beta = infinity and stay on the energy equation
    assert (1 if mode == "brent" else 2) in set(np.unique(co))
    assert_parity(Pg, Po, 1e-12)
    ctx.close()


@pytest.mark.parametrize("over,code", [({}, 0), ({"c2p_maxit": 0}, 1), ({"beta_entropy": 1e12}, 2)])
def test_device_inversion_recovers_the_state_it_was_built_from(G, over, code):
    """prim -> cons -> prim on the device alone, through the Newton-Raphson, the Brent-only and the
    entropy inversion: each returns the state that the device's own forward map started from, to
    round-off amplified by the conditioning (bar 1e-11 on the parity metric; the oracle reaches
    6e-13 on the same states).  This checks each root finder against what its root must be, not
    against the oracle's rendering of the same method."""
    c = _small3d()
    P = make_torus(c)
    ctx = G.Context(c, P, **over)
    U = ctx.prim2cons(P)
    rng = np.random.default_rng(5)
    guess = P * (1 + 0.01 * rng.uniform(-1, 1, size=P.shape))
    Pg, cg = ctx.cons2prim(U, guess)
    ctx.close()
    assert code in set(np.unique(cg)) and (cg >= 0).all()
    assert max_rel_err(Pg, P) < 1e-11


def _run_both(G, c, P, nsteps, dt=-1.0, **over):
    cfg = orc.make_cfg(c, **over)
    Po, dto, nfo, codeo = orc.step(cfg, P, nsteps, dt)
    ctx = G.Context(c, P, **over)
    dtg = [ctx.step(dt) for _ in range(nsteps)]
    Pg = ctx.get_prims()
    codeg = ctx.get_codes()
    t, ns, nf = ctx.get_time()
    ctx.close()
    return Pg, Po, np.array(dtg), dto, codeg, codeo, (t, ns, nf, nfo)


def test_one_step_2d_torus(G):
    c = torus_2d_64()
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, (t, ns, nf, nfo) = _run_both(G, c, P, 1)
    assert dtg[0] == pytest.approx(dto[0], rel=1e-13)
    assert np.array_equal(cg, co)
    assert nf == nfo == 0 and ns == 1
    assert_parity(Pg, Po, 1e-12)


def test_ten_steps_2d_torus(G):
    c = torus_2d_64()
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, (t, ns, nf, nfo) = _run_both(G, c, P, 10)
    assert np.allclose(dtg, dto, rtol=1e-10)
    assert t == pytest.approx(dto.sum(), rel=1e-10)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-8)


@pytest.mark.parametrize("riemann", ["llf", "hll"])
def test_small_3d_torus_steps(G, riemann):
    c = _small3d()
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1, riemann=riemann)
    assert_parity(Pg, Po, 1e-12)
    assert np.array_equal(cg, co)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 10, riemann=riemann)
    assert_parity(Pg, Po, 1e-8)
    assert np.allclose(dtg, dto, rtol=1e-10)


def test_ragged_3d_torus(G):
    """Odd sizes that fill no tile evenly (block of 256 threads, 64-lane waves)."""
    c = _small3d(n1=37, n2=19, n3=13, seed=23)
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
    assert_parity(Pg, Po, 1e-12)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 10)
    assert_parity(Pg, Po, 1e-8)


def test_flat_periodic_box_steps(G):
    c, P = _flat_box()
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 3)
    assert_parity(Pg, Po, 1e-12)
    assert np.allclose(dtg, dto, rtol=1e-13)


def test_flat_1d_line(G):
    c, P = _flat_box((64, 1, 1))
    Pg, Po, *_ = _run_both(G, c, P, 5)
    assert_parity(Pg, Po, 1e-12)


def test_fixed_dt_and_diagnostics(G):
    c = torus_2d_64()
    P = make_torus(c)
    Pg, Po, dtg, *_ = _run_both(G, c, P, 2, dt=0.01)
    assert np.all(dtg == 0.01)
    assert_parity(Pg, Po, 1e-12)
    cfg = orc.make_cfg(c)
    ctx = G.Context(c, P)
    mg, fg = ctx.diag()
    mo, fo, ih = orc.diag(cfg, P)
    assert mg == pytest.approx(mo, rel=1e-12)
    assert fg == pytest.approx(fo, rel=1e-12)
    ctx.close()


def test_one_step_128x64x64_torus(G):
    c = torus_128x64x64()
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
    assert dtg[0] == pytest.approx(dto[0], rel=1e-13)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)


def test_one_step_256cubed_torus_in_bench_configuration(G):
    """Full-size parity: the same 256^3 torus, graph-replayed launch chain and CFL step that the
    benchmark times, one step against the oracle on every cell."""
    c = torus_256cubed()
    P = make_torus(c)
    cfg = orc.make_cfg(c)
    ctx = G.Context(c, P)
    ctx.steps(1)
    Pg = ctx.get_prims()
    t, ns, nf = ctx.get_time()
    ctx.close()
    Po, dto, nfo, _ = orc.step(cfg, P, 1)
    assert t == pytest.approx(dto[0], rel=1e-13)
    assert_parity(Pg, Po, 1e-12)


def _run_graph(G, c, P, nsteps, **over):
    """The benchmark's path: CFL steps enqueued as graph replays (grmhd_steps)."""
    cfg = orc.make_cfg(c, **over)
    Po, dto, nfo, codeo = orc.step(cfg, P, nsteps)
    ctx = G.Context(c, P, **over)
    ctx.steps(nsteps)
    Pg, codeg = ctx.get_prims(), ctx.get_codes()
    t, ns, nf = ctx.get_time()
    ctx.close()
    assert ns == nsteps and nf == nfo
    assert t == pytest.approx(dto.sum(), rel=1e-10)
    return Pg, Po, codeg, codeo


@pytest.mark.parametrize("recon", ["plm", "ppm"])
@pytest.mark.parametrize("shape", [(24, 16, 64), (20, 12, 128), (20, 12, 48), (16, 10, 100)])
def test_ten_steps_on_the_uniform_metric_path(G, recon, shape):
    """Ten graph-replayed CFL steps.  n3 = 64 and 128 run on the row path, which the 256^3 benchmark
    runs (a wave is one phi row: scalar metric loads, marching and lane-shift face kernels, update
    workgroups on consecutive j).  A run with n3 = 48 or 100 takes the row path only in a batch of
    >= 2^20 cells (then the lanes of a row's last chunk wrap past its end); alone, as here, it takes
    the one-face kernels, and test_batched_ragged_runs_equal_their_solo_runs shows the batched
    row-path result equal to the solo one bit for bit, so this bar covers both."""
    c = _small3d(n1=shape[0], n2=shape[1], n3=shape[2], seed=31, recon=recon)
    P = make_torus(c)
    print("case", recon, shape, flush=True)
    Pg, Po, cg, co = _run_graph(G, c, P, 1)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)
    Pg, Po, cg, co = _run_graph(G, c, P, 10)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-8)


def test_ten_steps_128x64x64_torus_graph_path(G):
    c = torus_128x64x64()
    P = make_torus(c)
    Pg, Po, cg, co = _run_graph(G, c, P, 10)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-8)


def _hyperexp(n=(96, 64, 1), **kw):
    """The paper's production radial grid (Sec. 4.1): hyper-exponential beyond r = 400, n_X = 4,
    outer edge 5000 M."""
    base = dict(n1=n[0], n2=n[1], n3=n[2], r_out=5000.0, r_br=400.0, n_x=4, gam=13.0 / 9.0, delta=0.04,
                seed=17, cfl=0.45)
    base.update(kw)
    return TorusConfig(**base)


def test_hyperexponential_grid_fluxes_and_steps(G):
    c = _hyperexp()
    P = make_torus(c)
    ctx = G.Context(c, P)
    cfg = orc.make_cfg(c)
    for d in (1, 2):
        Fg, cg = ctx.debug_fluxes(d)
        Fo, co = orc.fluxes(cfg, P, d)
        assert scaled_abs_err(Fg, Fo) < 1e-12, d
        assert cg == pytest.approx(co, rel=1e-13)
    ctx.close()
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
    assert dtg[0] == pytest.approx(dto[0], rel=1e-13)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 10)
    assert_parity(Pg, Po, 1e-8)


def test_hyperexponential_grid_3d_step(G):
    c = _hyperexp((48, 24, 16))
    P = make_torus(c)
    Pg, Po, dtg, dto, cg, co, _ = _run_both(G, c, P, 1)
    assert np.array_equal(cg, co)
    assert_parity(Pg, Po, 1e-12)


def test_unphysical_conserved_states_fail_like_the_oracle(G):
    """Fault injection through grmhd_cons2prim: negative D, zero D, negative entropy in a low-beta
    cell (entropy method only), and momentum far above what the energy allows (the energy methods
    fail, the entropy method takes over); the codes and every inverted cell agree with the oracle."""
    c = _small3d()
    P = make_torus(c)
    cfg = orc.make_cfg(c)
    U = orc.prim2cons(cfg, P)
    ctx = G.Context(c, P)
    bad = [(5, 5, 3), (20, 12, 7), (30, 18, 1), (12, 3, 9)]
    U[0][bad[0]] = -abs(U[0][bad[0]])                 # D < 0
    guess = P.copy()
    guess[5:8][(slice(None),) + bad[1]] *= 1e3        # beta of the guess << 1e-2: entropy only
    U[8][bad[1]] = -abs(U[8][bad[1]])                 # S < 0
    U[2][bad[2]] *= 1e6                               # |Q| far above the energy: no v^2 < 1
    U[0][bad[3]] = 0.0                                # D = 0
    Pg, cg = ctx.cons2prim(U, guess)
    Po, co = orc.cons2prim(cfg, U, guess)
    ctx.close()
    assert np.array_equal(cg, co)
    for b in (bad[0], bad[1], bad[3]):
        assert co[b] == -1, b
    assert co[bad[2]] == 2          # the energy methods fail; the entropy method still inverts it
    ok = co >= 0
    assert_parity(np.where(ok[None], Pg, 0.0), np.where(ok[None], Po, 0.0), 1e-12)
