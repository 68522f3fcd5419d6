"""Pins of the oracle's diagnostics and of its macroscopic helpers against what
geometry, the paper's tables and closed forms fix.

* Radius profile (Sec. 4, the minimum ligament radius with the interface at
  mid-thickness): on a slice that is a sharp liquid disc of radius R, the
  liquid area is the number of lattice nodes inside the disc, which the Gauss
  circle count puts within a few R of pi R^2, so the equivalent radius is R
  to O(1/R).  A slice all above rho_l counts every node once (clamp at 1), a
  slice all below rho_v counts none (clamp at 0), a slice at the mid density
  counts half of every node.  Equal minima resolve to the smallest z.
* Capillary time (Eq. Oh_Tcap): Tables 1 and 2 print t_cap for seven radii
  each; recomputed from the same columns' rho_l, sigma and R0, every printed
  value sits 1.46-1.62 % above the formula (a uniform offset of the tables,
  not an R0 dependence, so the exponents are fixed).
* Laplace fit (Sec. 3, Laplace test): the oracle's own laplace_sigma on static
  cylinders at G0 = -5.3 gives the surface tension of Table 2 within 5 %, with
  Delta P linear in 1/R.
* v* (Sec. 4, Fig. 6): a uniform state at equilibrium with velocity u has
  no force, so u^b = u and v* = |u| t_cap / R0.
"""
import math

import numpy as np
import pytest
import torch

import lbm_inputs
from oracle import coexistence, diagnostics, lbm, physics

RV, RL = 0.12, 1.9


def _disc_slices(n, radii):
    """[len(radii), n, n] with rho_l strictly inside each disc (centre on the
    node (n/2, n/2)) and rho_v outside; also the node count of each disc."""
    yy, xx = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    d2 = xx * xx + yy * yy
    rho = np.full((len(radii), n, n), RV)
    counts = []
    for k, R in enumerate(radii):
        inside = d2 < R * R
        rho[k][inside] = RL
        counts.append(int(inside.sum()))
    return torch.from_numpy(rho), counts


def test_liquid_area_of_a_sharp_disc_is_its_node_count():
    rho, counts = _disc_slices(256, [10, 37, 90])
    A = diagnostics.liquid_area(rho, RV, RL)
    assert A.tolist() == [float(c) for c in counts]


@pytest.mark.parametrize("R", [20.0, 50.5, 100.0, 200.0])
def test_radius_of_a_sharp_cylinder_is_its_radius(R):
    # Gauss circle count: |N(R) - pi R^2| is far below the perimeter 2 pi R,
    # so the equivalent radius is R within 1/(2R) relative.
    rho, _ = _disc_slices(448, [R])
    r = float(diagnostics.radius_profile(rho, RV, RL)[0])
    assert abs(r / R - 1) < 0.5 / R, (r, R)


def test_radius_of_a_diffuse_cylinder():
    # tanh wall of width W about r = R: the liquid fraction is
    # (1 - tanh(2 s / W)) / 2 at distance s past the wall, whose area is
    # pi R^2 + 2 pi int s [frac - step] ds = pi R^2 + pi^3 W^2 / 48
    # (int_0^inf t (1 - tanh t) dt = pi^2 / 24).
    R, W = 40.0, 2.0
    rho = torch.from_numpy(lbm_inputs.density_from_radius(160, 160, [R], RV, RL, width=W))
    A = float(diagnostics.liquid_area(rho, RV, RL)[0])
    assert abs(A - (math.pi * R * R + math.pi ** 3 * W * W / 48)) < 0.5
    r = float(diagnostics.radius_profile(rho, RV, RL)[0])
    assert abs(r - math.sqrt(R * R + math.pi ** 2 * W * W / 48)) < 2e-3


def test_liquid_fraction_is_clamped_and_linear():
    # Densities with exact binary fractions, so every fraction is exact.
    n, rv, rl = 8, 0.125, 1.875
    vals = [rl * 1.5,     # above rho_l: 1 per node
            rv * 0.5,     # below rho_v: 0
            1.0,          # the mid density (rho_l + rho_v)/2: 1/2
            0.5625]       # a quarter of the way from rho_v to rho_l: 1/4
    rho = torch.stack([torch.full((n, n), v, dtype=torch.float64) for v in vals])
    A = diagnostics.liquid_area(rho, rv, rl).tolist()
    assert A == [64.0, 0.0, 32.0, 16.0]


def test_minimum_radius_ties_go_to_the_smallest_z():
    nz, n = 12, 32
    r_of_z = [9.0] * nz
    r_of_z[3] = r_of_z[8] = 5.0  # two equal necks
    rho = torch.from_numpy(lbm_inputs.density_from_radius(n, n, r_of_z, RV, RL))
    r = diagnostics.radius_profile(rho, RV, RL)
    assert float(r[3]) == float(r[8])
    rmin, z = diagnostics.minimum_radius(rho, RV, RL)
    assert z == 3 and rmin == float(r[3])
    assert rmin < float(r[0])


def test_interface_diagnostics_of_a_state_at_rest():
    # f = w rho: mass is the density sum; the pair-antisymmetric Shan-Chen
    # force sums to zero over the periodic box, so the momentum vanishes.
    rho0 = torch.from_numpy(lbm_inputs.ligament_density(16, 16, 20, 4.0, 0.1, 1, RV, RL))
    f = lbm.init_rest(rho0)
    d = diagnostics.interface_diagnostics(f, lbm.Params(G=-5.0, tau=1.0), RV, RL)
    assert abs(d["mass"] - float(rho0.sum())) < 1e-12 * d["mass"]
    assert max(abs(m) for m in d["mom"]) < 1e-13
    assert d["r_min"] == float(d["r_of_z"].min())


@pytest.mark.parametrize("op", ["srt", "mrt"])
def test_capillary_time_against_tables_1_and_2(op):
    t = lbm_inputs.PAPER_TABLE[op]
    ratios = []
    for i, R0 in enumerate(lbm_inputs.PAPER_RADII):
        ratios.append(t["t_cap"][i] / physics.capillary_time(t["rho_l"][i], t["sigma"][i], R0))
    assert min(ratios) > 1.0140 and max(ratios) < 1.0165, ratios
    assert max(ratios) - min(ratios) < 0.002


def test_ohnesorge_and_capillary_time_closed_forms():
    # mu = rho_l nu with nu = (tau - 1/2)/3; Oh t_cap = mu R0 / sigma.
    rho_l, sigma, R0, tau = 2.0, 0.05, 20.0, 0.8
    oh = physics.ohnesorge(tau, rho_l, sigma, R0)
    tc = physics.capillary_time(rho_l, sigma, R0)
    assert abs(oh * tc - rho_l * 0.1 * R0 / sigma) < 1e-12
    assert abs(tc * tc * sigma / (rho_l * R0 ** 3) - 1) < 1e-15


@pytest.mark.slow
def test_laplace_sigma_reproduces_table2():
    rv, rl, _ = coexistence.equal_area_rule(-5.3)
    radii = (8, 12, 16)
    # Jumps converged to 1e-6 (1.6e-4 of the smallest jump) keep this pin to
    # half a minute; the stored sigma of the workloads uses 1e-9.
    sigma, icpt, dps = physics.laplace_sigma(-5.3, rv, rl, radii=radii, tol=1e-6)
    # Linear in 1/R, slope sigma (cylinders: Delta P = sigma / R).
    inv = np.array([1.0 / R for R in radii])
    pred = sigma * inv + icpt
    ss_res = float(((np.array(dps) - pred) ** 2).sum())
    ss_tot = float(((np.array(dps) - np.mean(dps)) ** 2).sum())
    assert 1 - ss_res / ss_tot > 0.999
    assert abs(icpt) < 0.05 * sigma / radii[-1]
    assert abs(sigma / 0.0495 - 1) < 0.05
    # The jumps themselves: sigma / R within the fit's scatter.
    for R, dp in zip(radii, dps):
        assert abs(dp * R / 0.0495 - 1) < 0.08


def test_velocity_magnitude_star_of_a_uniform_flow():
    n = 6
    rho = torch.full((n, n, n), 1.3, dtype=torch.float64)
    u = torch.tensor([0.03, -0.04, 0.0], dtype=torch.float64).view(3, 1, 1, 1).expand(3, n, n, n)
    f = lbm.equilibrium(rho, u)
    R0, t_cap = 14.0, 347.0
    v = diagnostics.velocity_magnitude_star(f, lbm.Params(G=-5.3, tau=0.7), R0, t_cap)
    assert float((v - 0.05 * t_cap / R0).abs().max()) < 1e-13


def test_neck_is_cut_once_one_slice_is_wholly_vapour():
    nz, n = 10, 16
    rv, rl = 0.125, 1.875
    mid = 0.5 * (rv + rl)
    rho = torch.from_numpy(lbm_inputs.density_from_radius(n, n, [5.0] * nz, rv, rl))
    assert not diagnostics.neck_is_cut(rho, rv, rl)
    cut = rho.clone()
    cut[7] = rv                      # slice 7 all vapour
    assert diagnostics.neck_is_cut(cut, rv, rl)
    cut[7, 3, 4] = mid + 1e-9        # one node above the mid density keeps it whole
    assert not diagnostics.neck_is_cut(cut, rv, rl)
    cut[7, 3, 4] = mid               # at the mid density it is cut
    assert diagnostics.neck_is_cut(cut, rv, rl)
