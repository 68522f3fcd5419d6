"""Seeded synthetic inputs for the liquid-ligament problems.

This module holds no lattice Boltzmann arithmetic: it only builds initial
density fields and parameter sets.  It is the one piece of code that both the
float64 oracle (``oracle/``) and the GPU library's callers use, so that both
sides start from the same array and no random numbers have to match across
implementations.

Geometry (Sec. 3 of arXiv:1905.09554, Fig. 1): a cylindrical liquid ligament in
a periodic box, its radius modulated sinusoidally along the axis.  Readings:

* the axis runs along z (the slowest, plane index) through the node
  (nx/2, ny/2);
* the surface is r(z) = R (1 + A cos(2 pi m z / nz)) with an integer mode m,
  so the perturbation is periodic in the box; when a wavenumber kR is asked
  for, m = max(1, round(kR nz / (2 pi R))) and the effective kR = 2 pi m R / nz
  is reported;
* the density follows a tanh wall of width W = 2 between the coexisting
  densities: rho = (rho_l + rho_v)/2 - (rho_l - rho_v)/2 tanh(2 (d - r(z)) / W),
  with d the distance from the axis;
* optional uniform noise U(-eps, eps) from numpy's default_rng(seed), drawn
  in C order over [nz, ny, nx];
* the coexisting densities come from the oracle's flat-interface run (Sec. 3:
  flat-interface simulations give rho_l and rho_v) and are stored in
  ``coexistence.json`` by ``tests/golden/make_golden.py``.
"""
import json
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))


def coexistence(G):
    """(rho_v, rho_l) of the flat-interface run at interaction strength G."""
    with open(os.path.join(_HERE, "coexistence.json")) as fh:
        table = json.load(fh)
    key = "%.4f" % G
    if key not in table:
        raise KeyError("no stored coexistence densities for G = %s" % key)
    return table[key]["rho_v"], table[key]["rho_l"]


def surface_tension(G):
    """sigma from the oracle's Laplace test at interaction strength G."""
    with open(os.path.join(_HERE, "coexistence.json")) as fh:
        table = json.load(fh)
    return table["%.4f" % G]["sigma_laplace"]["sigma"]


def slab_density(nz, half_width, rho_v, rho_l, width=2.0):
    """Planar liquid slab |z - nz/2| < half_width with tanh walls, [nz, 1, 1]
    float64 (flat-interface runs, Sec. 3)."""
    z = np.arange(nz, dtype=np.float64)
    d = np.abs(z - nz / 2.0) - half_width
    rho = 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * d / width)
    return np.ascontiguousarray(rho.reshape(nz, 1, 1))


def droplet_density(n, R, rho_v, rho_l, width=2.0):
    """Static drop of radius R centred at (n/2, n/2, n/2) in a periodic n^3
    box with a tanh wall (the Laplace test, Sec. 3), [n, n, n] float64."""
    c = np.arange(n, dtype=np.float64) - n / 2.0
    d = np.sqrt(c[:, None, None] ** 2 + c[None, :, None] ** 2 + c[None, None, :] ** 2)
    return np.ascontiguousarray(0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) *
                                np.tanh(2.0 * (d - R) / width))


def integer_mode(kR, R, nz):
    """Integer axial mode closest to kR in a periodic box of length nz."""
    m = max(1, int(round(kR * nz / (2.0 * math.pi * R))))
    return m, 2.0 * math.pi * m * R / nz


def _distance_from_axis(nx, ny):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    return np.sqrt((x - nx / 2.0) ** 2 + (y - ny / 2.0) ** 2)


def density_from_radius(nx, ny, r_of_z, rho_v, rho_l, width=2.0):
    """tanh profile around a given radius profile r(z); returns [nz, ny, nx] float64."""
    r = np.asarray(r_of_z, dtype=np.float64)
    d = _distance_from_axis(nx, ny)[None, :, :]
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * np.tanh(2.0 * (d - r[:, None, None]) / width)


def ligament_density(nx, ny, nz, R, amp, mode, rho_v, rho_l, width=2.0,
                     noise=0.0, seed=0):
    """Initial density of a perturbed ligament, float64 [nz, ny, nx]."""
    z = np.arange(nz, dtype=np.float64)
    r = R * (1.0 + amp * np.cos(2.0 * math.pi * mode * z / nz))
    rho = density_from_radius(nx, ny, r, rho_v, rho_l, width)
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    return np.ascontiguousarray(rho)


def fourier_amplitudes(nmodes, R, rel_std, seed):
    """a_m ~ N(0, (rel_std R)^2), m = 1..nmodes, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, rel_std * R, size=nmodes)


def fourier_radius(nz, R, amps):
    """r(z) = R + sum_m a_m cos(2 pi m z / nz)."""
    z = np.arange(nz, dtype=np.float64)
    m = np.arange(1, len(amps) + 1, dtype=np.float64)
    return R + (np.asarray(amps)[:, None] * np.cos(2.0 * math.pi * m[:, None] * z[None, :] / nz)).sum(0)


def fourier_radius_torch(nz, R, amps):
    """Differentiable r(z) for a torch tensor of amplitudes (chain rule to a_m)."""
    import torch
    z = torch.arange(nz, dtype=amps.dtype)
    m = torch.arange(1, amps.shape[0] + 1, dtype=amps.dtype)
    return R + (amps[:, None] * torch.cos(2.0 * math.pi * m[:, None] * z[None, :] / nz)).sum(0)


def density_from_radius_torch(nx, ny, r_of_z, rho_v, rho_l, width=2.0):
    """Differentiable version of density_from_radius for a torch r(z)."""
    import torch
    d = torch.as_tensor(_distance_from_axis(nx, ny), dtype=r_of_z.dtype)[None]
    return 0.5 * (rho_l + rho_v) - 0.5 * (rho_l - rho_v) * torch.tanh(
        2.0 * (d - r_of_z[:, None, None]) / width)


def batch_ligaments(n=64, seed=0, r_min=8, r_max=48, kr_lo=0.3, kr_hi=0.95):
    """Uneven ligaments for a dispersion sweep.

    R ~ U{r_min..r_max}, kR ~ U[kr_lo, kr_hi] from default_rng(seed); box
    4R x 4R x round(2 pi R / kR) (one wavelength), effective kR = 2 pi R / nz.
    """
    rng = np.random.default_rng(seed)
    radii = rng.integers(r_min, r_max + 1, size=n)
    krs = rng.uniform(kr_lo, kr_hi, size=n)
    out = []
    for R, kr in zip(radii.tolist(), krs.tolist()):
        nz = int(round(2.0 * math.pi * R / kr))
        out.append({"R": int(R), "kR": float(kr), "nx": 4 * R, "ny": 4 * R, "nz": nz,
                    "kR_eff": 2.0 * math.pi * R / nz})
    return out


# The five workloads.  Sizes and physics follow the problem statement of each;
# amplitudes marked "assumed" are not given there.
WORKLOADS = {
    "ligament_32x32x64_bgk_f64": dict(
        nx=32, ny=32, nz=64, R=8, kR=2 * math.pi * 8 / 64, amp=0.1, noise=0.0, seed=0,
        G=-5.0, tau=1.0, collision="bgk", precision="f64", steps=1000),
    "ligament_128x128x512": dict(
        nx=128, ny=128, nz=512, R=32, kR=0.6, amp=0.05, noise=1e-4, seed=0,
        G=-5.0, tau=1.0, collision="bgk", precision="f32", steps=20000),
    "ligament_256x256x1024_mrt_f32": dict(
        nx=256, ny=256, nz=1024, R=64, kR=0.7, amp=0.05, noise=1e-4, seed=0,   # amp assumed
        G=-5.0, tau=1.0, collision="mrt", precision="f32", steps=5000),
    "batch64_bgk_f32": dict(n=64, seed=0, G=-5.0, tau=0.8, amp=0.01, collision="bgk",
                            precision="f32", steps=3000),
    "adjoint_64x64x256_mrt_f32": dict(
        nx=64, ny=64, nz=256, R=16, kR=0.7, nmodes=32, rel_std=0.02, seed=0,
        G=-5.0, tau=1.0, collision="mrt", precision="f32", steps=4000, checkpoint_every=200),
}


def workload_density(name, seed=None, kR=None):
    """Initial density of a single-ligament workload; returns (rho0, info).
    kR overrides the workload's wavenumber (the 256 x 256 x 1024 box is
    specified for kR in {0.45, 0.7})."""
    w = dict(WORKLOADS[name])
    if seed is not None:
        w["seed"] = seed
    if kR is not None:
        w["kR"] = kR
    rho_v, rho_l = coexistence(w["G"])
    if "nmodes" in w:
        amps = fourier_amplitudes(w["nmodes"], w["R"], w["rel_std"], w["seed"])
        r = fourier_radius(w["nz"], w["R"], amps)
        rho = density_from_radius(w["nx"], w["ny"], r, rho_v, rho_l)
        return np.ascontiguousarray(rho), dict(w, amps=amps, rho_v=rho_v, rho_l=rho_l)
    m, kr_eff = integer_mode(w["kR"], w["R"], w["nz"])
    rho = ligament_density(w["nx"], w["ny"], w["nz"], w["R"], w["amp"], m, rho_v, rho_l,
                           noise=w["noise"], seed=w["seed"])
    return rho, dict(w, mode=m, kR_eff=kr_eff, rho_v=rho_v, rho_l=rho_l)


# Parameters of the paper's ligament runs at G_0 = -5.3 and Oh = 0.1
# (Sec. 3, Table 1 for SRT with velocity-shift forcing, Table 2 for MRT with
# Guo-like forcing): box L_x x L_y x L_z with the axis along x and two
# wavelengths of the perturbation in L_x, tau, t_cap, rho_l, rho_v, sigma.
PAPER_G0 = -5.3
PAPER_RADII = (14, 28, 42, 56, 70, 84, 98)
PAPER_TABLE = {
    "srt": {
        "tau": (0.67926, 0.76297, 0.83053, 0.90311, 0.97021, 1.03776, 1.10647),
        "t_cap": (335, 912, 1611, 2380, 3189, 4015, 4846),
        "rho_l": (2.1167, 2.1254, 2.1348, 2.1450, 2.1557, 2.1666, 2.1775),
        "rho_v": (0.0836, 0.0900, 0.0974, 0.1059, 0.1156, 0.1264, 0.1383),
        "sigma": (0.05345, 0.05775, 0.06277, 0.06848, 0.07491, 0.08206, 0.08991),
    },
    "mrt": {
        "tau": (0.67293, 0.74445, 0.79942, 0.84575, 0.88667, 0.92350, 0.95745),
        "t_cap": (347, 981, 1803, 2775, 3878, 5098, 6424),
        "rho_l": (2.1086, 2.1086, 2.1086, 2.1086, 2.1086, 2.1085, 2.1085),
        "rho_v": (0.0778, 0.0779, 0.0779, 0.0779, 0.0778, 0.0778, 0.0778),
        "sigma": (0.04951, 0.04952, 0.04952, 0.04955, 0.04953, 0.04953, 0.04954),
    },
}


def paper_ligament(R0, operator, eps=0.1, wavelengths=2):
    """Initial density and parameters of the paper's run at radius R0 (Sec. 3,
    Tables 1-2): box L_x = 256 R0/14 along the axis (z here), L_y = L_z =
    96 R0/14, r = R0 + eps R0 cos(4 pi z / L_x) (two wavelengths; the paper's
    sine differs by a shift along the periodic axis), tanh wall of width 2.

    wavelengths = 1 gives the first half of that box along the axis, one
    wavelength: the two-wavelength input repeats with period L_x / 2, and a
    periodic run keeps that period, so the half box holds the same solution
    at half the cost."""
    if wavelengths not in (1, 2):
        raise ValueError("wavelengths must be 1 or 2")
    i = PAPER_RADII.index(R0)
    t = PAPER_TABLE[operator]
    lx = 256 * R0 // 14 * wavelengths // 2
    ly = 96 * R0 // 14
    rho = ligament_density(ly, ly, lx, float(R0), eps, wavelengths, t["rho_v"][i], t["rho_l"][i])
    return rho, {"R0": R0, "operator": operator, "eps": eps, "nx": ly, "ny": ly, "nz": lx,
                 "wavelengths": wavelengths, "G": PAPER_G0, "tau": t["tau"][i], "t_cap": t["t_cap"][i],
                 "rho_l": t["rho_l"][i], "rho_v": t["rho_v"][i], "sigma": t["sigma"][i]}
