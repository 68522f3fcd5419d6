"""Pins of the oracle's single step against closed forms and invariants.

Each check is chosen so that a plausible mistake in the oracle (a dropped
term, a wrong sign, a wrong index or streaming direction, a transposed
operand) fails at least one of them.
"""
import math

import mpmath as mp
import pytest
import torch

from oracle import diagnostics, lattice, lbm

mp.mp.dps = 30
DT = torch.float64


def _rand_state(shape=(4, 5, 6), seed=0, amp=0.05):
    g = torch.Generator().manual_seed(seed)
    rho = 1.0 + 0.3 * torch.rand(shape, generator=g, dtype=DT)
    f = lbm.init_rest(rho)
    f = f * (1.0 + amp * (torch.rand(f.shape, generator=g, dtype=DT) - 0.5))
    return f


# ---------------------------------------------------------------- equilibrium
def test_equilibrium_moments():
    g = torch.Generator().manual_seed(1)
    rho = 0.5 + torch.rand((3, 4, 5), generator=g, dtype=DT)
    u = 0.1 * (torch.rand((3, 3, 4, 5), generator=g, dtype=DT) - 0.5)
    feq = lbm.equilibrium(rho, u)
    c = lattice.velocities()
    assert torch.allclose(feq.sum(0), rho, rtol=0, atol=1e-15)
    j = torch.einsum("ad,a...->d...", c, feq)
    assert torch.allclose(j, rho * u, rtol=0, atol=1e-15)
    pi = torch.einsum("ad,ae,a...->de...", c, c, feq)
    for d in range(3):
        for e in range(3):
            expect = rho * u[d] * u[e] + (rho / 3.0 if d == e else 0.0)
            assert torch.allclose(pi[d, e], expect, rtol=0, atol=1e-15)


def test_guo_source_moments():
    g = torch.Generator().manual_seed(2)
    u = 0.1 * (torch.rand((3, 3, 4, 5), generator=g, dtype=DT) - 0.5)
    F = 0.01 * (torch.rand((3, 3, 4, 5), generator=g, dtype=DT) - 0.5)
    S = lbm.guo_source(u, F)
    c = lattice.velocities()
    assert float(S.sum(0).abs().max()) < 1e-17
    assert torch.allclose(torch.einsum("ad,a...->d...", c, S), F, rtol=0, atol=1e-17)
    pi = torch.einsum("ad,ae,a...->de...", c, c, S)
    for d in range(3):
        for e in range(3):
            assert torch.allclose(pi[d, e], u[d] * F[e] + F[d] * u[e], rtol=0, atol=1e-17)


# ---------------------------------------------------------------------- force
def _psi_mp(r):
    return 1 - mp.exp(-mp.mpf(r))


def _bump(n=4, p=(1, 1, 1), rho_b=1.5):
    rho = torch.ones((n, n, n), dtype=DT)
    rho[p[2], p[1], p[0]] = rho_b
    return rho


def test_uniform_psi_has_no_force():
    psi = torch.full((3, 4, 5), 0.7, dtype=DT)
    F = lbm.shan_chen_force(psi, -5.0)
    assert float(F.abs().max()) < 1e-16


def test_single_bump_force_closed_form():
    G = -5.0
    rho = _bump()
    F = lbm.shan_chen_force(lbm.pseudo_potential(rho), G)
    # At p + e_x the only neighbour with a different psi is p, reached along
    # -e_x with weight 1/18:  F = -G psi(1) (1/18) (psi(1.5) - psi(1)) (-e_x).
    fx = G * _psi_mp(1) * (_psi_mp(1.5) - _psi_mp(1)) / 18
    assert abs(float(fx) - (-2.541638789174962e-2)) < 1e-16
    assert abs(float(F[0, 1, 1, 2]) - float(fx)) < 1e-17
    assert abs(float(F[1, 1, 1, 2])) < 1e-17 and abs(float(F[2, 1, 1, 2])) < 1e-17
    # At p + e_x + e_y the link to p is the diagonal (-1,-1,0), weight 1/36.
    fd = G * _psi_mp(1) * (_psi_mp(1.5) - _psi_mp(1)) / 36
    assert abs(float(F[0, 1, 2, 2]) - float(fd)) < 1e-17
    assert abs(float(F[1, 1, 2, 2]) - float(fd)) < 1e-17
    # No force on the bump itself, and the pair forces cancel in total.
    assert float(F[:, 1, 1, 1].abs().max()) < 1e-17
    assert float(F.sum(dim=(1, 2, 3)).abs().max()) < 1e-15
    # Nodes that are not neighbours of p feel nothing.
    assert float(F[:, 3, 3, 3].abs().max()) == 0.0


# ---------------------------------------------------- hand-derived single step
def _hand_value_at_bump(a, tau, G=-5.0, rho_b=1.5):
    """f_a at the bump node p after one step, derived by hand.

    Before the step f = w rho, j = 0.  After streaming, f_a(p) comes from the
    node q = p - c_a.  For a = 0 that is p itself, where F = 0, so the
    collision leaves w_0 rho_b.  For a != 0, q has rho = 1, j = 0 and sees p
    along +c_a, hence F(q) = phi c_a with phi = -G psi(1) w_a (psi(rho_b) -
    psi(1)); then u = F / 2, c.u = phi |c|^2 / 2, u.u = phi^2 |c|^2 / 4,
    c.F = phi |c|^2, u.F = phi^2 |c|^2 / 2, and the collision is
    f* = w + (f^eq - w)/tau + (1 - 1/(2 tau)) S.
    """
    c = lattice.C_INT[a]
    w = lattice.W_FRAC[a]
    wm = mp.mpf(w.numerator) / w.denominator
    if a == 0:
        return wm * rho_b
    c2 = sum(k * k for k in c)
    phi = -G * _psi_mp(1) * wm * (_psi_mp(rho_b) - _psi_mp(1))
    cu = phi * c2 / 2
    uu = phi * phi * c2 / 4
    cF = phi * c2
    uF = phi * phi * c2 / 2
    feq = wm * (1 + 3 * cu + mp.mpf(9) / 2 * cu * cu - mp.mpf(3) / 2 * uu)
    S = wm * (3 * (cF - uF) + 9 * cu * cF)
    tau = mp.mpf(tau)
    return wm + (feq - wm) / tau + (1 - 1 / (2 * tau)) * S


@pytest.mark.parametrize("tau", [1.0, 0.8])
def test_hand_checked_step_on_4cubed(tau):
    rho = _bump()
    p = lbm.Params(G=-5.0, tau=tau, collision="bgk", forcing="guo")
    f1 = lbm.step(lbm.init_rest(rho), p)
    for a in range(19):
        expect = float(_hand_value_at_bump(a, tau))
        assert abs(float(f1[a, 1, 1, 1]) - expect) < 1e-15, (a, float(f1[a, 1, 1, 1]), expect)


def test_hand_checked_step_far_node_is_rest():
    # A node whose whole neighbourhood (distance 2) is uniform stays at w rho.
    rho = torch.ones((6, 6, 6), dtype=DT)
    rho[1, 1, 1] = 1.5
    f1 = lbm.step(lbm.init_rest(rho), lbm.Params(G=-5.0, tau=0.9))
    w = lattice.weights()
    assert torch.allclose(f1[:, 4, 4, 4], w, rtol=0, atol=1e-16)


# ------------------------------------------------------------------ collision
def test_mrt_with_equal_rates_is_bgk():
    f = _rand_state()
    tau = 0.77
    pb = lbm.Params(G=-5.0, tau=tau, collision="bgk")
    pm = lbm.Params(G=-5.0, tau=tau, collision="mrt", s_bulk=1 / tau, s_ghost=1 / tau,
                    s_conserved=1 / tau)
    assert torch.allclose(lbm.step(f, pb), lbm.step(f, pm), rtol=0, atol=2e-15)


def test_conserved_rates_have_no_effect():
    f = _rand_state(seed=3)
    pa = lbm.Params(G=-5.0, tau=0.9, collision="mrt", s_conserved=0.3)
    pb = lbm.Params(G=-5.0, tau=0.9, collision="mrt", s_conserved=1.7)
    assert torch.allclose(lbm.step(f, pa), lbm.step(f, pb), rtol=0, atol=2e-15)


@pytest.mark.parametrize("coll", ["bgk", "mrt"])
def test_post_collision_momentum_is_j_plus_F(coll):
    f = _rand_state(seed=4)
    p = lbm.Params(G=-5.0, tau=0.7, collision=coll)
    fs = lbm.collide(f, p)
    F = lbm.force_of_state(f, p)
    assert torch.allclose(lbm.density(fs), lbm.density(f), rtol=0, atol=1e-14)
    assert torch.allclose(lbm.momentum(fs), lbm.momentum(f) + F, rtol=0, atol=1e-14)


@pytest.mark.parametrize("coll,forcing", [("bgk", "guo"), ("mrt", "guo"), ("bgk", "shift")])
def test_uniform_rest_state_is_fixed_point(coll, forcing):
    f = lbm.init_rest(torch.full((3, 4, 5), 0.9, dtype=DT))
    p = lbm.Params(G=-5.0, tau=0.8, collision=coll, forcing=forcing)
    assert torch.allclose(lbm.step(f, p), f, rtol=0, atol=1e-16)


def test_tau_one_gives_equilibrium_plus_half_source():
    f = _rand_state(seed=5)
    p = lbm.Params(G=-4.0, tau=1.0)
    rho, j = lbm.density(f), lbm.momentum(f)
    F = lbm.force_of_state(f, p)
    ub = (j + 0.5 * F) / rho
    expect = lbm.equilibrium(rho, ub) + 0.5 * lbm.guo_source(ub, F)
    assert torch.allclose(lbm.collide(f, p), expect, rtol=0, atol=1e-16)


# ----------------------------------------------------------- whole-run checks
def _ligament(nx=16, ny=16, nz=32, R=5.0, amp=0.1):
    z = torch.arange(nz, dtype=DT)
    y, x = torch.meshgrid(torch.arange(ny, dtype=DT), torch.arange(nx, dtype=DT), indexing="ij")
    d = torch.sqrt((x - nx / 2) ** 2 + (y - ny / 2) ** 2)
    r = R * (1 + amp * torch.cos(2 * math.pi * z / nz))
    return 1.0 - 0.88 * torch.tanh(d[None] - r[:, None, None])


@pytest.mark.parametrize("coll", ["bgk", "mrt"])
def test_mass_and_momentum_conserved(coll):
    rho0 = _ligament()
    p = lbm.Params(G=-5.0, tau=0.8, collision=coll)
    f0 = lbm.init_rest(rho0)
    f = lbm.run(f0, p, 200)
    m0, m1 = float(lbm.density(f0).sum()), float(lbm.density(f).sum())
    assert abs(m1 - m0) / m0 < 1e-13
    mom = diagnostics.total_momentum(f, p)
    assert float(mom.abs().max()) < 1e-12 * m0


def test_translation_equivariance_bitwise():
    rho0 = _ligament(nx=12, ny=10, nz=16, R=3.0)
    p = lbm.Params(G=-5.0, tau=0.8, collision="mrt")
    f = lbm.run(lbm.init_rest(rho0), p, 5)
    shift = (3, -2, 5)
    fs = lbm.run(lbm.init_rest(torch.roll(rho0, shift, dims=(0, 1, 2))), p, 5)
    assert torch.equal(torch.roll(f, shift, dims=(1, 2, 3)), fs)


def test_mirror_symmetry():
    # A profile symmetric under x -> nx - x about the axis node stays so;
    # populations map a -> a' with cx -> -cx.
    nx = 16
    rho0 = _ligament(nx=nx, ny=16, nz=16, R=4.0)
    p = lbm.Params(G=-5.0, tau=0.8, collision="mrt")
    f = lbm.run(lbm.init_rest(rho0), p, 30)
    idx = {c: a for a, c in enumerate(lattice.C_INT)}
    perm = [idx[(-c[0], c[1], c[2])] for c in lattice.C_INT]
    xi = [(nx - x) % nx for x in range(nx)]
    fm = f[perm][..., xi]
    assert float((fm - f).abs().max()) < 1e-13


def _wave_amplitude(field, k_idx, dim):
    n = field.shape[dim]
    pos = torch.arange(n, dtype=DT)
    shape = [1] * field.dim()
    shape[dim] = n
    return float((field * torch.sin(2 * math.pi * k_idx * pos / n).view(shape)).mean() * 2)


@pytest.mark.parametrize("coll,tau", [("bgk", 0.8), ("mrt", 0.8), ("mrt", 1.3)])
def test_shear_wave_decays_at_shear_viscosity(coll, tau):
    # u_x(z) = U sin(k z) decays as exp(-nu k^2 t), nu = c_s^2 (tau - 1/2):
    # pins the relaxation of the shear rows (G = 0, no interaction).
    nz = 64
    k = 2 * math.pi / nz
    z = torch.arange(nz, dtype=DT)
    u = torch.zeros((3, nz, 1, 1), dtype=DT)
    u[0] = (1e-4 * torch.sin(k * z)).view(nz, 1, 1)
    rho = torch.ones((nz, 1, 1), dtype=DT)
    f = lbm.equilibrium(rho, u)
    p = lbm.Params(G=0.0, tau=tau, collision=coll, s_bulk=1.0, s_ghost=1.2)
    a0 = _wave_amplitude(lbm.momentum(f)[0], 1, 0)
    t = 400
    f = lbm.run(f, p, t)
    a1 = _wave_amplitude(lbm.momentum(f)[0], 1, 0)
    nu = (tau - 0.5) / 3
    # The lattice adds an O(k^2) relative correction (about 1e-3 here).
    assert abs(-math.log(a1 / a0) / (nu * k * k * t) - 1) < 3e-3


def test_sound_wave_damping_sets_bulk_row():
    # Longitudinal wave: amplitude damping Gamma = (4 nu / 3 + xi) k^2 / 2 with
    # shear nu = (1/s_shear - 1/2)/3 and bulk xi = (2/9)(1/s_bulk - 1/2) for
    # the D3Q19 d'Humieres basis.  Two bulk rates, same shear rate: the damping
    # must change as predicted, which pins the energy row's rate.
    nz = 64
    k = 2 * math.pi / nz
    z = torch.arange(nz, dtype=DT)
    rho = (1.0 + 1e-5 * torch.cos(k * z)).view(nz, 1, 1)
    f0 = lbm.init_rest(rho)
    rates = []
    for s_bulk in (1.0, 1.6):
        p = lbm.Params(G=0.0, tau=0.6, collision="mrt", s_bulk=s_bulk, s_ghost=1.2)
        f = f0
        period = 2 * math.pi / (k / math.sqrt(3.0))
        nper = 4
        t = int(round(nper * period))
        energies = []
        for step in range(t + 1):
            if step in (0, t):
                dr = lbm.density(f)[:, 0, 0] - 1.0
                jz = lbm.momentum(f)[2, :, 0, 0]
                energies.append(float((dr * dr / 3.0 + jz * jz).sum()))
            if step < t:
                f = lbm.step(f, p)
        rates.append(-math.log(energies[1] / energies[0]) / (2 * t))
        nu = (0.6 - 0.5) / 3
        xi = (2.0 / 9.0) * (1.0 / s_bulk - 0.5)
        gamma = 0.5 * (4 * nu / 3 + xi) * k * k
        assert abs(rates[-1] / gamma - 1) < 0.03, (s_bulk, rates[-1], gamma)
    assert rates[0] > rates[1]
