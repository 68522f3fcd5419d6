"""Physics pins of the oracle: numbers the paper prints and laws the method obeys.

* Table 2 (MRT, Guo-like forcing, G_0 = -5.3): rho_l = 2.1086, rho_v = 0.0778,
  sigma = 0.0495 (Sec. 3, Table 2).
* Table 1 (SRT, velocity shift, G_0 = -5.3): tau-dependent rho_l and rho_v
  (Sec. 3, Table 1).  Reproducing it needs the velocity-shift forcing of
  Eq. vel_shift exactly as written.
* The psi-specific equal-area rule for the coexisting densities.
* The Laplace law (Sec. 3, the Laplace test used to measure sigma) is pinned
  through the oracle's own laplace_sigma in tests/test_oracle_diagnostics.py.
* Plateau-Rayleigh: perturbations grow only for kR < 1 (Sec. 1 and Sec. 4).

Tolerances: the flat-interface densities of a diffuse, four-node interface
differ from the continuum rule by up to 0.5 % in rho_v (a discretisation effect
that also depends on where the slab sits relative to the nodes); the tables
print four significant digits.
"""
import math

import pytest
import torch

import lbm_inputs
from oracle import coexistence, diagnostics, lbm

TABLE2 = {"rho_l": 2.1086, "rho_v": 0.0778, "sigma": 0.0495}
# Table 1 columns: tau -> (rho_l, rho_v)
TABLE1 = {0.83053: (2.1348, 0.0974), 1.10647: (2.1775, 0.1383)}


def test_equal_area_rule_reproduces_table2():
    rv, rl, _ = coexistence.equal_area_rule(-5.3)
    assert abs(rl - TABLE2["rho_l"]) < 2e-4
    assert abs(rv - TABLE2["rho_v"]) < 1e-4


def test_flat_interface_mrt_reproduces_table2():
    p = lbm.Params(G=-5.3, tau=1.0, collision="mrt", s_bulk=1.0, s_ghost=1.2)
    rv, rl, steps, _ = coexistence.flat_interface(p, nz=32, half_width=8,
                                                  rho_guess=(0.08, 2.1), tol=1e-10)
    assert abs(rl / TABLE2["rho_l"] - 1) < 5e-4
    assert abs(rv / TABLE2["rho_v"] - 1) < 6e-3
    rv0, rl0, _ = coexistence.equal_area_rule(-5.3)
    assert abs(rl / rl0 - 1) < 5e-4 and abs(rv / rv0 - 1) < 6e-3


def test_flat_interface_guo_is_tau_independent():
    out = []
    for tau, coll in ((0.8, "bgk"), (1.0, "bgk"), (0.95745, "mrt")):
        p = lbm.Params(G=-5.3, tau=tau, collision=coll, s_bulk=1.0 / tau, s_ghost=1.0)
        rv, rl, _, _ = coexistence.flat_interface(p, nz=32, half_width=8,
                                                  rho_guess=(0.08, 2.1), tol=1e-10)
        out.append((rv, rl))
    for rv, rl in out[1:]:
        assert abs(rv - out[0][0]) < 1e-8 and abs(rl - out[0][1]) < 1e-8


@pytest.mark.parametrize("tau", sorted(TABLE1))
def test_flat_interface_velocity_shift_reproduces_table1(tau):
    p = lbm.Params(G=-5.3, tau=tau, collision="bgk", forcing="shift")
    rv, rl, _, _ = coexistence.flat_interface(p, nz=32, half_width=8,
                                              rho_guess=(0.08, 2.1), tol=1e-10)
    rl_t, rv_t = TABLE1[tau]
    assert abs(rl / rl_t - 1) < 1e-3
    assert abs(rv / rv_t - 1) < 1.5e-2


def test_stored_coexistence_matches_oracle():
    # The stored G = -5 densities that feed the ligament inputs come from this
    # very run; recompute and compare.
    rv_s, rl_s = lbm_inputs.coexistence(-5.0)
    rv0, rl0, _ = coexistence.equal_area_rule(-5.0)
    p = lbm.Params(G=-5.0, tau=1.0)
    rv, rl, _, _ = coexistence.flat_interface(p, nz=32, half_width=8, rho_guess=(rv0, rl0),
                                              tol=1e-10)
    assert abs(rv - rv_s) < 1e-12 and abs(rl - rl_s) < 1e-12
    assert abs(rl / rl0 - 1) < 5e-4 and abs(rv / rv0 - 1) < 6e-3


def _mode_amplitude(f, nz, rv, rl):
    z = torch.arange(nz, dtype=torch.float64)
    r = diagnostics.radius_profile(lbm.density(f), rv, rl)
    return float((r * torch.cos(2 * math.pi * z / nz)).sum() * 2 / nz)


@pytest.mark.parametrize("nz,grows", [(48, True), (30, False)])
def test_plateau_rayleigh_growth_only_below_kR_one(nz, grows):
    R, n = 6, 24
    rv, rl = lbm_inputs.coexistence(-5.0)
    rho = torch.from_numpy(lbm_inputs.ligament_density(n, n, nz, R, 0.05, 1, rv, rl))
    p = lbm.Params(G=-5.0, tau=1.0)
    f = lbm.run(lbm.init_rest(rho), p, 200)
    a0 = _mode_amplitude(f, nz, rv, rl)
    f = lbm.run(f, p, 400)
    a1 = _mode_amplitude(f, nz, rv, rl)
    kR = 2 * math.pi * R / nz
    assert (kR < 1) == grows
    if grows:
        assert a1 > 1.5 * a0
    else:
        assert a1 < 0.5 * a0


def test_weber_growth_rate_limits_and_paper_value():
    from oracle import physics
    # Inviscid limit: (omega t_cap)^2 = x^2 (1 - x^2) / 2, maximum at x^2 = 1/2.
    for x in (0.3, 0.5, 1 / math.sqrt(2), 0.9):
        assert abs(physics.growth_rate_weber(x, 0.0) - math.sqrt(0.5 * x * x * (1 - x * x))) < 1e-15
    assert physics.growth_rate_weber(1.0, 0.1) == 0.0
    assert physics.growth_rate_weber(1.2, 0.1) == 0.0
    # Viscosity lowers the rate.
    assert physics.growth_rate_weber(0.7, 0.3) < physics.growth_rate_weber(0.7, 0.1)
    # The paper's linear-stability curve (Fig. 3) uses omega t_cap = 0.2800 at
    # kR0 ~ 0.687, Oh = 0.1 (T_break = -ln(eps) / 0.28 for all its points).
    assert abs(physics.growth_rate_weber(0.687, 0.1) / 0.2800 - 1) < 0.04


def test_ohnesorge_of_the_tables():
    # Eq. Oh_Tcap with nu = (tau - 1/2)/3 gives Oh = 0.1 for Table 2's columns.
    from oracle import physics
    t = lbm_inputs.PAPER_TABLE["mrt"]
    for i, R0 in enumerate(lbm_inputs.PAPER_RADII):
        oh = physics.ohnesorge(t["tau"][i], t["rho_l"][i], t["sigma"][i], R0)
        assert abs(oh - 0.1) < 0.002, (R0, oh)
