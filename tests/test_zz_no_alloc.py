"""grmhd_diag_full_noalloc (the diagnostics entry point that allocates nothing) against
grmhd_diag_full through the C ABI: the same kernel writes the same shell sums, so horizon values and
radial profiles agree bit for bit.  Two calls in a row share the GPU's fixed array, the second on a
smaller run, and a run with n1 beyond the stated limit is refused with EINVAL."""
import ctypes

import numpy as np
import pytest

from paper_2205_02484_amd.torus_init import make_torus
from paper_2205_02484_amd.workloads import torus_2d_64, torus_128x64x64

pytestmark = pytest.mark.gpu

FIELDS = ("mdot", "phi_b", "ldot", "edot", "phi_b_norm", "i_h")


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02484_amd import grmhd
    grmhd.load()
    return grmhd


def _noalloc(G, ctx, with_radial=True):
    hz = G.Horizon()
    rad = np.full((6, ctx.grid.n1), -7.0) if with_radial else None
    rc = G.load().grmhd_diag_full_noalloc(ctx._h, ctypes.byref(hz), rad.ctypes.data if with_radial else None)
    assert rc == G.OK, G.load().grmhd_last_error()
    return {k: getattr(hz, k) for k in FIELDS}, rad


def _same(a, b):
    return np.array_equal(a, b, equal_nan=True)


def test_noalloc_diagnostics_equal_the_allocating_call_twice_the_second_smaller(G):
    big = torus_128x64x64()
    small = torus_2d_64()
    for cfg, nsteps in ((big, 4), (small, 6)):
        ctx = G.Context(cfg, make_torus(cfg))
        ctx.steps(nsteps)
        hz_ref, rad_ref = ctx.diag_full()
        hz, rad = _noalloc(G, ctx)
        assert hz == hz_ref
        assert _same(rad, rad_ref)
        hz2, _ = _noalloc(G, ctx, with_radial=False)
        assert hz2 == hz_ref
        ctx.close()


def test_noalloc_diagnostics_refuse_a_run_beyond_the_limit(G):
    cfg = torus_2d_64()
    n1 = 16385
    P = np.empty((8, n1, 8, 1))
    P[0], P[1], P[2:] = 1.0, 1.0, 0.0
    ctx = G.Context(cfg, P, n1=n1, n2=8)
    hz = G.Horizon()
    rc = G.load().grmhd_diag_full_noalloc(ctx._h, ctypes.byref(hz), None)
    assert rc == G.EINVAL
    assert b"GRMHD_NOALLOC_MAX_N1" in G.load().grmhd_last_error()
    ctx.close()
