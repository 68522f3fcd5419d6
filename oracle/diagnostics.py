"""Diagnostics of a state, float64 (test infrastructure only).

* pressure       P = rho c_s^2 + c_s^2 G psi^2 / 2               (Eq. EOS_SC)
* mass           sum_x rho
* momentum       sum_x (j + F/2) = sum_x rho u^b                 (Eq. barycentric)
* radius profile the paper measures the "minimum ligament radius", the
                 smallest radial coordinate of the interface, with the
                 interface at mid-thickness (Sec. 4, Fig. 5 discussion).
                 Reading taken here: liquid area of each z-slice
                 A(z) = sum_{x,y} clamp((rho - rho_v)/(rho_l - rho_v), 0, 1),
                 equivalent radius r(z) = sqrt(A(z)/pi), r_min = min_z r(z),
                 ties broken towards the smallest z.  It needs no axis
                 position and is piecewise differentiable.
* velocity magnitude v* = |u^b| / (R0 / t_cap)                    (Sec. 4, Fig. 6)
* break-up         the paper compares ligaments up to the pinch-off but
                   states no criterion for it (Sec. 4, Fig. 2b).  Reading
                   taken here: the column is cut once some z-slice holds no
                   node denser than the mid density (rho_l + rho_v) / 2.

Pins (tests/test_oracle_diagnostics.py): the liquid area of a sharp disc
slice is its lattice-node count and its equivalent radius is the disc radius
to O(1/R) (Gauss circle count); a tanh wall of width W adds pi^3 W^2 / 48 to
the area (closed form); densities above rho_l count 1, below rho_v 0, the mid
density 1/2; equal minima go to the smallest z; a state at rest has zero
momentum; v* of a uniform flow is |u| t_cap / R0; the neck is cut when one
slice lies wholly at or below the mid density and not while a single node of
every slice is above it.  The pressure is not pinned
by restating Eq. EOS_SC: the EoS is pinned through the flat-interface
coexistence densities and the Laplace law (tests/test_oracle_physics.py).
"""
import math

import torch

from . import lbm

CS2 = 1.0 / 3.0


def pressure(rho, G, psi_rho0=1.0):
    """Eq. EOS_SC: P = rho c_s^2 + c_s^2 G psi^2 / 2."""
    psi = lbm.pseudo_potential(rho, psi_rho0)
    return rho * CS2 + 0.5 * CS2 * G * psi * psi


def mass(f):
    return float(lbm.density(f).sum())


def total_momentum(f, p):
    """sum_x (j + F/2), the momentum carried by the barycentric velocity."""
    F = lbm.force_of_state(f, p)
    return (lbm.momentum(f) + 0.5 * F).sum(dim=(1, 2, 3))


def liquid_area(rho, rho_v, rho_l):
    """A(z) = sum_{x,y} clamp((rho - rho_v)/(rho_l - rho_v), 0, 1); rho is [nz, ny, nx]."""
    frac = ((rho - rho_v) / (rho_l - rho_v)).clamp(0.0, 1.0)
    return frac.sum(dim=(-2, -1))


def radius_profile(rho, rho_v, rho_l):
    """r(z) = sqrt(A(z)/pi)."""
    return torch.sqrt(liquid_area(rho, rho_v, rho_l) / math.pi)


def minimum_radius(rho, rho_v, rho_l):
    """(r_min, z_argmin) with the smallest z among ties."""
    r = radius_profile(rho, rho_v, rho_l)
    rmin = float(r.min())
    z = int(torch.nonzero(r == r.min())[0, 0])
    return rmin, z


def neck_is_cut(rho, rho_v, rho_l):
    """True once some z-slice of rho [nz, ny, nx] has no node above (rho_l + rho_v)/2."""
    slice_max = rho.amax(dim=(-2, -1))
    return bool((slice_max <= 0.5 * (rho_l + rho_v)).any())


def interface_diagnostics(f, p, rho_v, rho_l):
    """Everything the GPU library reports for a state, as a dict of floats."""
    rho = lbm.density(f)
    r = radius_profile(rho, rho_v, rho_l)
    rmin, z = minimum_radius(rho, rho_v, rho_l)
    mom = total_momentum(f, p)
    return {
        "mass": float(rho.sum()),
        "mom": [float(m) for m in mom],
        "r_of_z": r,
        "r_min": rmin,
        "z_argmin": z,
    }


def velocity_magnitude_star(f, p, R0, t_cap):
    """v* = |u^b| / (R0 / t_cap) (Sec. 4, Fig. 6)."""
    ub = lbm.barycentric_velocity(f, p)
    return torch.sqrt((ub * ub).sum(dim=0)) / (R0 / t_cap)
