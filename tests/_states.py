"""Random physical primitive states for the pin tests (test helper; no method arithmetic beyond
normalising a random direction with the metric the caller passes in)."""
import math

import numpy as np


def random_state(rng, gcov, *, gam=4.0 / 3.0, lor_max=50.0, beta=None, sigma_max=100.0,
                 point_state=None):
    """Primitive P with Lorentz factor in [1, lor_max], u/rho in [1e-4, 10] and, when beta is
    given, field scaled so that p_g / (b^2/2) = beta (b^2 via `point_state(P)` -> bsq)."""
    rho = 10 ** rng.uniform(-6, 0)
    u = rho * 10 ** rng.uniform(-4, 1)
    lor = 10 ** rng.uniform(0, math.log10(lor_max))
    x = rng.normal(size=3)
    gij = gcov[1:, 1:]
    x /= math.sqrt(x @ gij @ x)
    ut = math.sqrt(lor * lor - 1.0) * x
    B = rng.normal(size=3)
    P = np.array([rho, u, ut[0], ut[1], ut[2], B[0], B[1], B[2]])
    if beta is not None and point_state is not None:
        bsq = point_state(P)
        pg = (gam - 1.0) * u
        P[5:] *= math.sqrt(2.0 * pg / beta / bsq)
        # keep sigma = b^2/rho bounded
        bsq = point_state(P)
        if bsq / rho > sigma_max:
            P[0] = bsq / sigma_max
    return P
