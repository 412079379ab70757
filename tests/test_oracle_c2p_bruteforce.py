"""Brute-force inversion on tiny grids (Sec. 2.3 pin).  In flat space every cell shares one metric, so a
grid of N cells evaluates N candidate primitive states in one call of the oracle's forward map
(prim2cons, U = sqrt(-g)(rho u^t, T^t_nu, B^i)).  An exhaustive scan of a coarse lattice over
(ln rho, ln u, u~1, u~2, u~3) (8^5 states spanning the whole range the targets are drawn from)
orders the lattice points by mismatch; a compass search from each in turn -- all 3^5 neighbours of
the current point, the step halved when none is better -- drives the sum of squared relative
mismatches of the five fluid components of U down until one reaches round-off (the mismatch also
has a nonzero local minimum on the u -> 0 edge, which a start there slides into), using nothing of
the inversion's equations or iterations (the field needs no search: with sqrt(-g) = 1 it is U's
field components).  The oracle's cons2prim, started from an unrelated
guess, must return the same states for every cell of a tiny grid.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc

GAM = 13.0 / 9.0


def _cfg(n1, n2=1):
    return orc.make_cfg(None, coords="cart", n1=n1, n2=n2, n3=1, gam=GAM)


def _forward(C):
    """Conserved vectors of the candidate states C[8][N] (flat metric)."""
    N = C.shape[1]
    return orc.prim2cons(_cfg(N), C.reshape(8, N, 1, 1)).reshape(9, N)


def _brute_force(Ut, iters=3000):
    """Primitive state whose conserved vector matches Ut[9] (one cell), by compass search."""
    B = Ut[5:8]
    scale = abs(Ut[0]) + abs(Ut[1])

    def mismatch(X):
        C = np.empty((8, X.shape[1]))
        C[0], C[1] = np.exp(X[0]), np.exp(X[1])
        C[2:5] = X[2:5]
        C[5:8] = B[:, None]
        return (((_forward(C)[:5] - Ut[:5, None]) / scale) ** 2).sum(axis=0)   # smooth, zero only at the root

    # coarse lattice: rho in [1e-3, 3], u in [1e-4, 30], each u~ component in [-2, 2]
    axes = [np.linspace(math.log(1e-3), math.log(3.0), 8), np.linspace(math.log(1e-4), math.log(30.0), 8)]
    axes += [np.linspace(-2.0, 2.0, 8)] * 3
    lat = np.array(np.meshgrid(*axes, indexing="ij")).reshape(5, -1)
    order = np.argsort(mismatch(lat))
    dirs = np.array(np.meshgrid(*[[-1.0, 0.0, 1.0]] * 5, indexing="ij")).reshape(5, -1)
    centre = int(np.where(np.all(dirs == 0.0, axis=0))[0][0])
    for start in order[:64]:
        x = lat[:, start].copy()
        step = 0.25 * np.array([(a[1] - a[0]) for a in axes])
        for _ in range(iters):
            r = mismatch(x[:, None] + step[:, None] * dirs)
            best = int(np.argmin(r))
            if best == centre or r[best] >= r[centre]:
                step *= 0.5
                if step.max() < 1e-16:
                    break
            else:
                x = x + step * dirs[:, best]
        if r[centre] < 1e-26:
            break
    C = np.empty(8)
    C[0], C[1] = math.exp(x[0]), math.exp(x[1])
    C[2:5] = x[2:5]
    C[5:8] = B
    return C, float(np.abs(_forward(C[:, None])[:5, 0] - Ut[:5]).max() / scale)


def _targets(seed, n):
    rng = np.random.default_rng(seed)
    P = np.zeros((8, n))
    P[0] = 10 ** rng.uniform(-2, 0, n)
    P[1] = P[0] * 10 ** rng.uniform(-1, 0.7, n)
    lor = 1.0 + rng.uniform(0.0, 1.0, n)                     # Lorentz factor up to 2
    d = rng.normal(size=(3, n))
    d /= np.linalg.norm(d, axis=0)
    P[2:5] = np.sqrt(lor * lor - 1.0) * d
    P[5:8] = rng.normal(size=(3, n)) * np.sqrt(P[1])[None, :]  # plasma beta of order 1-10
    return P


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5, 6])
def test_inversion_matches_brute_force_on_a_tiny_grid(seed):
    n1, n2 = 2, 2
    P = _targets(seed, n1 * n2)
    cfg = _cfg(n1, n2)
    U = orc.prim2cons(cfg, P.reshape(8, n1, n2, 1))
    guess = np.zeros_like(P)
    guess[0], guess[1] = 1.0, 1.0
    guess[5:8] = P[5:8]
    Pi, code = orc.cons2prim(cfg, U, guess.reshape(8, n1, n2, 1))
    Pi = Pi.reshape(8, -1)
    assert np.all(code == 0)
    Uf = U.reshape(9, -1)
    for c in range(n1 * n2):
        Pb, res = _brute_force(Uf[:, c])
        assert res < 1e-13, res      # the forward map's own rounding
        # the searched state and the inversion agree (and both equal the state U was made from)
        for q in range(5):
            ref = max(abs(P[q, c]), 1.0 if q >= 2 else 0.0)
            assert abs(Pi[q, c] - Pb[q]) <= 1e-10 * ref, (c, q, Pi[q, c], Pb[q])
            assert abs(Pb[q] - P[q, c]) <= 1e-10 * ref, (c, q, Pb[q], P[q, c])
        assert np.array_equal(Pi[5:8, c], Pb[5:8])
