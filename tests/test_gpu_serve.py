"""GPU test of the served request loop: jobs arriving while others run are admitted, all finish,
and each served result and its horizon diagnostics equal those of the same job run alone (bit for
bit: the batched kernels do the same arithmetic per run)."""
import numpy as np
import pytest

from paper_2205_02484_amd.torus_init import TorusConfig, make_torus

pytestmark = pytest.mark.gpu


def test_served_stream_results_equal_solo_runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_02484_amd import grmhd, serve
    cfgs = [TorusConfig(n1=40 + 4 * x, n2=32, n3=1 if x % 2 else 8, spin=0.3 + 0.1 * x, r_in=6.0, r_max=12.0,
                        r_out=60.0, seed=100 + x) for x in range(6)]
    jobs = [serve.Job(jid=x, cfg=c, nsteps=20 + 7 * x, arrival=0.02 * x) for x, c in enumerate(cfgs)]
    kept = {}

    def make_input(c):
        return make_torus(c)
    b = grmhd.Batch()
    orig_fetch = b.fetch

    def fetch(h):
        out = orig_fetch(h)
        kept[h] = out
        return out
    b.fetch = fetch
    res = serve.serve(jobs, steps_per_launch=5, batch=b, make_input=make_input, diagnose=True)
    assert res["jobs"] == 6
    for j in jobs:
        ctx = grmhd.Context(j.cfg, make_torus(j.cfg))
        ctx.steps(j.nsteps)
        P = ctx.get_prims()
        t, n, nfail = ctx.get_time()
        hz = ctx.diag_full()[0]
        ctx.close()
        Pb, tb, nb = kept[j.handle]
        assert nb == n == j.nsteps
        assert tb == t
        assert np.array_equal(Pb, P)
        assert j.horizon == hz
        assert j.unfixed == nfail
    b.close()
