"""The funnel workloads really exercise Sec. 2.4's limiters: on the oracle, switching each limiter
off (its threshold at 1e300) changes the one-step result of many cells by more than 1e-8, so GPU
parity on these workloads covers the ceilings' re-inversion and the Lorentz cap."""
import numpy as np
import pytest

from oracle import oracle as orc
from paper_2205_02484_amd.torus_init import make_torus
from tests._funnel import ACTS, funnel


@pytest.mark.parametrize("grid,kind", sorted(ACTS))
def test_each_limiter_acts(grid, kind):
    c, over = funnel(grid, kind)
    P = make_torus(c)
    a, _, nfail, codes = orc.step(orc.make_cfg(c, **over), P, 1)
    assert nfail == 0
    assert (codes == 2).sum() > 0            # the magnetised atmosphere takes the entropy inversion
    for name in ACTS[(grid, kind)]:
        o, *_ = orc.step(orc.make_cfg(c, **{**over, name: 1e300}), P, 1)
        changed = ((np.abs(o - a) / np.maximum(np.abs(a), 1e-300)).max(axis=0) > 1e-8).sum()
        assert changed > 50, (name, changed)
