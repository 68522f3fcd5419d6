"""Liquid and vapour coexistence densities (test infrastructure only).

The paper obtains rho_l and rho_v from flat-interface simulations (Sec. 3, the
set-up paragraph before Tables 1-2) and lists them for G_0 = -5.3 in Tables 1
(SRT, velocity shift) and 2 (MRT, Guo-like forcing).

Two independent routes are given here:

* ``equal_area_rule``: the mechanical-stability condition of the Shan-Chen
  model.  For psi-based forces with a second-order forcing scheme the
  coexisting densities satisfy P(rho_v) = P(rho_l) = P0 with P of Eq. EOS_SC
  and  int_{rho_v}^{rho_l} (P0 - P(rho)) psi'(rho) / psi(rho)^(1+eps) drho = 0,
  eps = 0 (Shan and Chen 1994; Shan 2008; Li, Luo and Li 2012).  Solved with
  scipy quadrature and a root finder: a closed mathematical statement
  independent of the lattice code.
* ``flat_interface``: the paper's own route, a planar liquid slab in a
  periodic box run with the oracle step until stationary; rho_l is read at the
  slab centre, rho_v at the farthest vapour node.

Pins: the flat-interface run at G = -5.3 with MRT Guo forcing reproduces Table
2 (rho_l = 2.1086, rho_v = 0.0778) and agrees with the equal-area rule; the
BGK Guo run is independent of tau; the rule at G = -5.3 itself reproduces
Table 2.
"""
import math

import numpy as np
import torch

from . import lbm

CS2 = 1.0 / 3.0


def _psi(r, rho0):
    return rho0 * (1.0 - math.exp(-r / rho0))


def _dpsi(r, rho0):
    return math.exp(-r / rho0)


def _pressure(r, G, rho0):
    p = _psi(r, rho0)
    return r * CS2 + 0.5 * CS2 * G * p * p


def equal_area_rule(G, psi_rho0=1.0, eps=0.0, guess=(0.1, 2.0)):
    """Coexisting (rho_v, rho_l, P0) from the psi-specific equal-area rule."""
    from scipy import integrate, optimize

    def residual(v):
        rv, rl = v
        p0 = _pressure(rl, G, psi_rho0)
        area, _ = integrate.quad(
            lambda r: (p0 - _pressure(r, G, psi_rho0)) * _dpsi(r, psi_rho0)
            / _psi(r, psi_rho0) ** (1.0 + eps),
            rv, rl, epsabs=1e-14, epsrel=1e-13, limit=200)
        return [_pressure(rv, G, psi_rho0) - p0, area]

    sol = optimize.fsolve(residual, guess, xtol=1e-14, full_output=True)
    rv, rl = (float(x) for x in sol[0])
    return rv, rl, _pressure(rl, G, psi_rho0)


def slab_density(nz, rho_l, rho_v, half_width, width=2.0):
    """Planar liquid slab centred at nz/2 with tanh walls, shape [nz, 1, 1]."""
    z = torch.arange(nz, dtype=torch.float64)
    d = (z - nz / 2.0).abs() - half_width
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * torch.tanh(2.0 * d / width)
    return rho.view(nz, 1, 1)


def flat_interface(p, nz=64, half_width=16, rho_guess=(0.1, 2.0), tol=1e-13,
                   check_every=100, max_steps=200000):
    """Run a flat slab to its stationary state.

    Returns (rho_v, rho_l, steps, rho_profile).  The box is 1 x 1 x nz,
    periodic: the 3D D3Q19 stencil on a field uniform in x and y.
    Stationarity: max |rho(t) - rho(t - check_every)| < tol.
    """
    rho0 = slab_density(nz, rho_guess[1], rho_guess[0], half_width)
    f = lbm.init_rest(rho0)
    prev = lbm.density(f).clone()
    steps = 0
    while steps < max_steps:
        f = lbm.run(f, p, check_every)
        steps += check_every
        rho = lbm.density(f)
        if float((rho - prev).abs().max()) < tol:
            break
        prev = rho.clone()
    rho = lbm.density(f)[:, 0, 0]
    return float(rho[0]), float(rho[nz // 2]), steps, rho


def flat_interface_np(*args, **kw):
    """As ``flat_interface`` but returns numpy profile (convenience for scripts)."""
    rv, rl, steps, rho = flat_interface(*args, **kw)
    return rv, rl, steps, np.asarray(rho)
