"""Pin of the oracle's reference gradients: autograd through the oracle run
against central finite differences of the same run (float64)."""
import math

import numpy as np
import torch

import lbm_inputs
from oracle import adjoint


def _case():
    rv, rl = lbm_inputs.coexistence(-5.0)
    rho0 = torch.from_numpy(lbm_inputs.ligament_density(12, 12, 24, 3.5, 0.1, 1, rv, rl))
    return rho0, rv, rl


def test_autograd_matches_finite_differences():
    rho0, rv, rl = _case()
    steps = 30
    for coll in ("bgk", "mrt"):
        loss, g_rho, g_G, g_tau = adjoint.rmin_gradients(rho0, -5.0, 0.9, steps, rv, rl,
                                                         collision=coll, segment=10)
        h = 1e-5

        def L(G=-5.0, tau=0.9, rho=rho0):
            with torch.no_grad():
                return float(adjoint.rmin_after(rho, G, tau, steps, rv, rl, collision=coll))

        fd_G = (L(G=-5.0 + h) - L(G=-5.0 - h)) / (2 * h)
        fd_tau = (L(tau=0.9 + h) - L(tau=0.9 - h)) / (2 * h)
        assert abs(g_G - fd_G) <= 1e-5 * abs(fd_G) + 1e-9, (coll, g_G, fd_G)
        assert abs(g_tau - fd_tau) <= 1e-5 * abs(fd_tau) + 1e-9, (coll, g_tau, fd_tau)
        # A smooth direction in rho0: the axial cosine mode of the radius.
        z = torch.arange(rho0.shape[0], dtype=torch.float64)
        d = (torch.cos(2 * math.pi * z / rho0.shape[0])[:, None, None]
             * torch.ones_like(rho0) * 1e-3)
        fd_d = (L(rho=rho0 + h * d) - L(rho=rho0 - h * d)) / (2 * h)
        ad_d = float((g_rho * d).sum())
        assert abs(ad_d - fd_d) <= 1e-5 * abs(fd_d) + 1e-9, (coll, ad_d, fd_d)
        assert np.isfinite(loss)


def test_rate_gradients_match_finite_differences():
    rho0, rv, rl = _case()
    steps = 30
    loss, g_b, g_g = adjoint.rmin_rate_gradients(rho0, -5.0, 0.9, steps, rv, rl, 1.1, 1.2,
                                                 segment=10)
    h = 1e-5

    def L(sb=1.1, sg=1.2):
        with torch.no_grad():
            return float(adjoint.rmin_after(rho0, -5.0, 0.9, steps, rv, rl, collision="mrt",
                                            s_bulk=sb, s_ghost=sg))

    fd_b = (L(sb=1.1 + h) - L(sb=1.1 - h)) / (2 * h)
    fd_g = (L(sg=1.2 + h) - L(sg=1.2 - h)) / (2 * h)
    assert abs(g_b - fd_b) <= 1e-5 * abs(fd_b) + 1e-9, (g_b, fd_b)
    assert abs(g_g - fd_g) <= 1e-5 * abs(fd_g) + 1e-9, (g_g, fd_g)
    # both rates matter to this loss
    assert abs(fd_b) > 1e-6 and abs(fd_g) > 1e-6
