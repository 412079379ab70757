"""Pin of what a cell left unfixed keeps (Sec. 2.3, averaging procedure; Sec. 2.2, flux-CT).

The fixups average only the fluid variables; the field of every cell, failed or not, comes from
the flux-CT update, which keeps the corner divergence of sqrt(-g) B at round-off.  A cell that no
round can fix falls back to the stage input for rho, u and u~, and must keep the updated field:
taking the input's field there would put the previous field next to updated neighbours and break
the corner divergence around it.  The pin runs the fixups with no rounds allowed (every failed
cell stays unfixed) and with rounds that leave the centre of a large block unfixed, on a
divergence-free stage output, and checks the divergence; the planted mistake (the input's field
restored too) fails it.
"""
import math

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.workloads import torus_2d_64
from paper_2205_02484_amd.torus_init import make_torus
from tests._planted import variant
from tests.test_oracle_step import _centre_gdet, corner_divb


def _case(rounds):
    c = torus_2d_64()
    cfg = orc.make_cfg(c, fixup_max_rounds=rounds)
    P0 = make_torus(c)
    P1, _, nfail, _ = orc.step(orc.make_cfg(c), P0, 3)      # a divergence-free stage output
    assert nfail == 0
    code = np.zeros((c.n1, c.n2, 1), dtype=np.int8)
    code[36, 33, 0] = -1                                     # inside the magnetised torus
    code[46:49, 30:33, 0] = -1
    code[38:45, 28:35, 0] = -1                               # 7 x 7: its centre needs 4 rounds
    Pout = P1.copy()
    Pout[0:5, code == -1] = np.nan
    Po, co, left = orc.fixups(cfg, Pout, P0, code.copy())
    return cfg, P0, P1, Po, co, left


def _check(rounds):
    cfg, P0, P1, Po, co, left = _case(rounds)
    assert left > 0
    assert np.isfinite(Po).all()
    stuck = co == -1
    assert np.array_equal(Po[0:5, stuck], P0[0:5, stuck])
    gd = _centre_gdet(cfg)
    dx = [(math.log(cfg.r_out) - math.log(cfg.r_in)) / cfg.n1, 1 / cfg.n2]
    div = corner_divb(Po, gd[..., None], dx, 2)
    bscale = np.abs(P1[5:7] * gd[None, ..., None]).max() / min(dx)
    assert np.abs(div).max() < 1e-13 * bscale
    # the test discriminates: the field did change over the steps around the failed cells
    assert np.abs(P1[5:7, stuck] - P0[5:7, stuck]).max() > 1e-6 * np.abs(P1[5:7]).max()


@pytest.mark.parametrize("rounds", [0, 2])
def test_unfixed_cells_keep_the_updated_field(rounds):
    _check(rounds)


def test_planted_field_restore_fails(tmp_path):
    rep = ("memcpy(&Pout[cidx(g, i, j, k) * NPR], &Pin[cidx(g, i, j, k) * NPR], 5 * sizeof(double));",
           "memcpy(&Pout[cidx(g, i, j, k) * NPR], &Pin[cidx(g, i, j, k) * NPR], NPR * sizeof(double));")
    with variant(tmp_path, "restore_field", [rep]):
        with pytest.raises(AssertionError):
            _check(0)
