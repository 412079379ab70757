"""Pins of the oracle's conserved-to-primitive inversion (Sec. 2.3), floors, ceilings and the
Lorentz cap (Sec. 2.4): exact round trips through the independent prim->cons map, closed-form
floor/ceiling bookkeeping, and the neighbour-average fixups.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from tests._states import random_state

RNG = np.random.default_rng(99)


def _kerr(**kw):
    base = dict(n1=64, n2=64, n3=1, spin=0.9375, r_out=40.0, gam=4.0 / 3.0)
    base.update(kw)
    return orc.make_cfg(None, **base)


def _bsq_fn(cfg, X1, X2):
    def f(P):
        s = orc.point_state(cfg, X1, X2, P)
        return s["bcon"] @ s["bcov"]
    return f


def _roundtrip_errors(cfg, P, X1, X2, mode, guess_jitter=0.01):
    U = orc.point_state(cfg, X1, X2, P)["U"]
    Pg = P * (1 + guess_jitter * RNG.uniform(-1, 1, size=8))
    Pr, code = orc.point_c2p(cfg, X1, X2, U, Pg, mode)
    lor = math.sqrt(1 + (P[2:5] @ orc.geom(cfg, X1, X2)[0][1:, 1:] @ P[2:5]))
    err = np.zeros(8)
    err[0] = abs(Pr[0] - P[0]) / P[0]
    err[1] = abs(Pr[1] - P[1]) / P[1]
    err[2:5] = np.abs(Pr[2:5] - P[2:5]) / lor
    bmag = np.abs(P[5:]).max()
    err[5:] = np.abs(Pr[5:] - P[5:]) / max(bmag, 1e-300)
    return err, code, lor


@pytest.mark.parametrize("gam", [4.0 / 3.0, 13.0 / 9.0, 5.0 / 3.0])
def test_roundtrip_energy_methods_moderate_states(gam):
    """Well-conditioned states (Gamma <= 3, u/rho >= 0.1, beta >= 1) come back to 1e-12; the
    wider set (Gamma <= 5, u/rho >= 1e-2, beta >= 0.3) within 1e-14 of the condition number
    kappa = Gamma^2 (rho + u + b^2) / p of the energy equation."""
    cfg = _kerr(gam=gam)
    worst = 0.0
    for _ in range(300):
        X1, X2 = RNG.uniform(math.log(1.4), math.log(300)), RNG.uniform(0.03, 0.97)
        gcov = orc.geom(cfg, X1, X2)[0]
        wide = RNG.random() < 0.5
        P = random_state(RNG, gcov, gam=gam, lor_max=5.0 if wide else 3.0,
                         beta=10 ** RNG.uniform(-0.5 if wide else 0.0, 4),
                         point_state=_bsq_fn(cfg, X1, X2))
        P[1] = max(P[1], (1e-2 if wide else 1e-1) * P[0])
        err, code, lor = _roundtrip_errors(cfg, P, X1, X2, mode=0)
        assert code == 0
        if wide:
            s = orc.point_state(cfg, X1, X2, P)
            kappa = lor * lor * (P[0] + P[1] + s["bcon"] @ s["bcov"]) / ((gam - 1) * P[1])
            assert err.max() < 1e-14 * kappa, (err, kappa)
        else:
            worst = max(worst, err.max())
    assert worst < 1e-12, worst


def test_roundtrip_energy_methods_extreme_states_within_conditioning():
    """Gamma up to 50, u/rho down to 1e-4: the energy equation fixes p only to
    ~eps * Gamma^2 (rho + b^2)/p, so the bound scales with that condition number."""
    cfg = _kerr()
    for _ in range(300):
        X1, X2 = RNG.uniform(math.log(1.4), math.log(300)), RNG.uniform(0.03, 0.97)
        gcov = orc.geom(cfg, X1, X2)[0]
        P = random_state(RNG, gcov, lor_max=50.0, beta=10 ** RNG.uniform(-1.5, 4),
                         point_state=_bsq_fn(cfg, X1, X2))
        s = orc.point_state(cfg, X1, X2, P)
        bsq = s["bcon"] @ s["bcov"]
        pg = (cfg.gam - 1) * P[1]
        if pg < 1.5e-2 * 0.5 * bsq:
            continue
        err, code, lor = _roundtrip_errors(cfg, P, X1, X2, mode=1, guess_jitter=0.0)
        assert code in (0, 1)
        kappa = lor * lor * (P[0] + bsq + P[1]) / pg
        assert err.max() < 1e-13 * max(kappa, 10.0), (err, kappa)


def test_roundtrip_entropy_method():
    cfg = _kerr(gam=5.0 / 3.0)
    worst = 0.0
    for _ in range(300):
        X1, X2 = RNG.uniform(math.log(1.4), math.log(300)), RNG.uniform(0.03, 0.97)
        gcov = orc.geom(cfg, X1, X2)[0]
        P = random_state(RNG, gcov, gam=cfg.gam, lor_max=10.0, beta=10 ** RNG.uniform(-3, 2),
                         point_state=_bsq_fn(cfg, X1, X2))
        err, code, lor = _roundtrip_errors(cfg, P, X1, X2, mode=2)
        assert code == 2
        worst = max(worst, err.max() / lor)
    assert worst < 1e-12, worst


def test_low_beta_cells_use_the_entropy_method_only():
    cfg = _kerr()
    X1, X2 = math.log(6.0), 0.3
    gcov = orc.geom(cfg, X1, X2)[0]
    P = random_state(RNG, gcov, lor_max=3.0, beta=1e-3, point_state=_bsq_fn(cfg, X1, X2), sigma_max=1e9)
    U = orc.point_state(cfg, X1, X2, P)["U"]
    Pr, code = orc.point_c2p(cfg, X1, X2, U, P, 0)
    assert code == 2
    assert np.allclose(Pr[:5], P[:5], rtol=1e-10)


def test_brent_on_w_when_newton_is_not_allowed_to_iterate():
    cfg = _kerr(c2p_maxit=0)
    for _ in range(50):
        X1, X2 = RNG.uniform(math.log(1.4), math.log(300)), RNG.uniform(0.03, 0.97)
        gcov = orc.geom(cfg, X1, X2)[0]
        P = random_state(RNG, gcov, lor_max=5.0, beta=10 ** RNG.uniform(0, 3), point_state=_bsq_fn(cfg, X1, X2))
        P[1] = max(P[1], 1e-2 * P[0])
        err, code, _ = _roundtrip_errors(cfg, P, X1, X2, mode=0)
        assert code == 1
        assert err.max() < 1e-11


def test_unphysical_conserved_states_fail():
    cfg = _kerr()
    X1, X2 = math.log(6.0), 0.45
    gcov = orc.geom(cfg, X1, X2)[0]
    P = random_state(RNG, gcov, lor_max=2.0, beta=10.0, point_state=_bsq_fn(cfg, X1, X2))
    U = orc.point_state(cfg, X1, X2, P)["U"]
    Ubad = U.copy()
    Ubad[0] = -abs(U[0])
    assert orc.point_c2p(cfg, X1, X2, Ubad, P, 0)[1] == -1
    Ubad = U.copy()
    Ubad[8] = -abs(U[8])
    Plow = P.copy()
    Plow[5:] *= 100.0  # guess with beta << 1e-2 -> entropy only, which needs S > 0
    assert orc.point_c2p(cfg, X1, X2, Ubad, Plow, 0)[1] == -1


# ---------------------------------------------------------------------------------------------
# floors / ceilings / cap
# ---------------------------------------------------------------------------------------------

def test_density_and_energy_floors():
    cfg = _kerr(rho_fl_coef=1e-4, rho_fl_pow=-1.5, u_fl_coef=1e-6, u_fl_pow=-2.5)
    r = 9.0
    P = np.array([1e-12, 1e-14, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    Pf = orc.point_floors(cfg, math.log(r), 0.5, P)
    assert Pf[0] == pytest.approx(1e-4 * r ** -1.5, rel=1e-14)
    assert Pf[1] == pytest.approx(1e-6 * r ** -2.5, rel=1e-14)


def test_ceiling_adds_mass_and_energy_at_rest_in_the_normal_frame():
    cfg = _kerr()
    X1, X2 = math.log(5.0), 0.2
    gcov, gcon, gdet, _ = orc.geom(cfg, X1, X2)
    alpha = 1 / math.sqrt(-gcon[0, 0])
    P = np.array([1e-4, 1e-5, 0.1, 0.02, 0.3, 0.05, 0.01, 0.0])
    s = orc.point_state(cfg, X1, X2, P)
    bsq = s["bcon"] @ s["bcov"]
    drho = bsq / 50 - P[0]
    du = bsq / 2500 - P[1]
    assert drho > 0 and du > 0
    Pf = orc.point_floors(cfg, X1, X2, P)
    Uf = orc.point_state(cfg, X1, X2, Pf)["U"]
    U0 = s["U"]
    added = np.array([gdet * drho / alpha, -gdet * (drho + du), 0.0, 0.0, 0.0])
    assert np.allclose(Uf[:5], U0[:5] + added, rtol=1e-11, atol=1e-13 * np.abs(U0[:5]).max())
    assert np.array_equal(Pf[5:], P[5:])


def test_lorentz_factor_cap():
    cfg = _kerr()
    X1, X2 = math.log(20.0), 0.5
    gcov = orc.geom(cfg, X1, X2)[0]
    x = np.array([0.3, 0.1, 0.2])
    x /= math.sqrt(x @ gcov[1:, 1:] @ x)
    P = np.array([1.0, 1.0, *(math.sqrt(80 ** 2 - 1) * x), 0.0, 0.0, 0.0])
    Pf = orc.point_floors(cfg, X1, X2, P)
    lor = math.sqrt(1 + Pf[2:5] @ gcov[1:, 1:] @ Pf[2:5])
    assert lor == pytest.approx(50.0, rel=1e-13)
    assert np.allclose(Pf[2:5] / np.linalg.norm(Pf[2:5]), x / np.linalg.norm(x), rtol=1e-14)


# ---------------------------------------------------------------------------------------------
# fixups
# ---------------------------------------------------------------------------------------------

def _fixup_case(bad):
    cfg = orc.make_cfg(None, coords="cart", n1=12, n2=12, n3=1, gam=4 / 3)
    Pout = np.empty((8, 12, 12, 1))
    Pout[0] = 1.0 + RNG.random((12, 12, 1))
    Pout[1] = 1.0 + RNG.random((12, 12, 1))
    Pout[2:5] = 0.1 * RNG.normal(size=(3, 12, 12, 1))
    Pout[5:] = RNG.normal(size=(3, 12, 12, 1))
    Pin = Pout + 0.5
    code = np.zeros((12, 12, 1), dtype=np.int8)
    for (i, j) in bad:
        code[i, j, 0] = -1
    return cfg, Pout, Pin, code


def test_isolated_failure_takes_the_cross_average():
    cfg, Pout, Pin, code = _fixup_case([(5, 5)])
    P, code2, left = orc.fixups(cfg, Pout, Pin, code)
    ref = 0.25 * (Pout[:5, 4, 5, 0] + Pout[:5, 6, 5, 0] + Pout[:5, 5, 4, 0] + Pout[:5, 5, 6, 0])
    assert left == 0 and code2[5, 5, 0] == 3
    assert np.allclose(P[:5, 5, 5, 0], ref, rtol=1e-15)
    assert np.array_equal(P[5:], Pout[5:])


def test_adjacent_failures_take_the_diagonal_average():
    cfg, Pout, Pin, code = _fixup_case([(5, 5), (5, 6)])
    P, _, left = orc.fixups(cfg, Pout, Pin, code)
    ref = 0.25 * (Pout[:5, 4, 4, 0] + Pout[:5, 4, 6, 0] + Pout[:5, 6, 4, 0] + Pout[:5, 6, 6, 0])
    assert left == 0 and np.allclose(P[:5, 5, 5, 0], ref, rtol=1e-15)


def test_block_of_failures_is_filled_by_jacobi_rounds():
    bad = [(i, j) for i in range(4, 7) for j in range(4, 7)]
    cfg, Pout, Pin, code = _fixup_case(bad)
    P, code2, left = orc.fixups(cfg, Pout, Pin, code)
    assert left == 0
    # the centre has no valid neighbour in round 1; in round 2 its cross neighbours are valid
    ref = 0.25 * (P[:5, 4, 5, 0] + P[:5, 6, 5, 0] + P[:5, 5, 4, 0] + P[:5, 5, 6, 0])
    assert np.allclose(P[:5, 5, 5, 0], ref, rtol=1e-15)


def test_unfixable_cells_keep_the_stage_input_fluid_and_their_field():
    bad = [(i, j) for i in range(12) for j in range(12)]
    cfg, Pout, Pin, code = _fixup_case(bad)
    P, _, left = orc.fixups(cfg, Pout, Pin, code)
    assert left == 144 and np.array_equal(P[:5], Pin[:5]) and np.array_equal(P[5:], Pout[5:])
