"""One time step of the D3Q19 pseudo-potential lattice Boltzmann method, float64.

Test infrastructure only (see the package docstring).  Follows Sec. 2 of
arXiv:1905.09554 in the paper's notation; every step is written on whole
arrays, in the order the method applies it, with no fusion:

 1. moments            rho = sum_a f_a,  rho u = sum_a c_a f_a     (Eq. momentum)
 2. pseudo-potential   psi = rho0 (1 - exp(-rho / rho0))            (Sec. 2, after Eq. SC_force)
 3. Shan-Chen force    F(x) = -G psi(x) sum_a w_a psi(x + c_a) c_a  (Eq. SC_force)
 4. forcing            Guo-like: u^b = u + F / (2 rho) in f^eq plus
                       the Guo (2002) source term                   (Eq. barycentric)
                       or velocity shift u' = u + tau F / rho       (Eq. vel_shift)
 5. equilibrium        f^eq = w rho [1 + c.u/c_s^2 + (c.u)^2/(2c_s^4)
                                     - u.u/(2c_s^2)]                (Eq. local_eq)
 6. collision          SRT (BGK) or MRT, Omega = M^-1 Lambda M      (Eq. LBE and the
                                                                    collision-operator cases)
 7. streaming          f_a(x + c_a, t + 1) = f*_a(x, t)             (Eq. LBE)

Readings of the text (each listed in the design notes of the repository):

* Eq. local_eq as printed lacks the leading "1 +" inside the bracket; it is
  restored, which is what makes sum_a f^eq_a = rho hold.
* The Shan-Chen sum uses the lattice weights w_a themselves; only this choice
  gives the equation of state of Eq. EOS_SC, P = rho c_s^2 + c_s^2 G psi^2 / 2.
* Guo forcing source (Guo, Zheng and Shi 2002, cited for the MRT forcing):
  S_a = w_a [ (c_a - u^b).F / c_s^2 + (c_a.u^b)(c_a.F) / c_s^4 ], added as
  (1 - 1/(2 tau)) S in SRT and as M^-1 (I - Lambda/2) M S in MRT.
* MRT equilibrium moments are taken as M f^eq(rho, u^b), so MRT with every rate
  equal to 1/tau is exactly the SRT operator.
* Fully periodic boundaries.

State convention: ``f`` is the post-streaming population field at time n,
shape [19, nz, ny, nx].

Pins (tests/test_oracle_*.py): equilibrium moments, Guo-source moments, the
closed-form single-bump force, a hand-derived single step on a 4^3 lattice,
MRT == SRT when all rates are 1/tau, conserved-row rates without effect,
mass/momentum conservation, translation and mirror symmetry, the flat-interface
coexistence densities of Table 2 and the psi equal-area rule, the Laplace law,
growth only for kR < 1.
"""
import torch

from . import lattice

_C = lattice.C_INT


def density(f):
    """rho = sum_a f_a (Eq. momentum)."""
    return f.sum(dim=0)


def momentum(f):
    """rho u = sum_a c_a f_a (Eq. momentum); returns [3, nz, ny, nx]."""
    c = lattice.velocities().to(f.dtype)
    return torch.einsum("ad,a...->d...", c, f)


def pseudo_potential(rho, psi_rho0=1.0):
    """psi = rho0 [1 - exp(-rho / rho0)] (Sec. 2, after Eq. SC_force)."""
    return psi_rho0 * (1.0 - torch.exp(-rho / psi_rho0))


def neighbour(field, c):
    """field(x + c) on the periodic lattice; field is [nz, ny, nx]."""
    cx, cy, cz = c
    return torch.roll(field, shifts=(-cz, -cy, -cx), dims=(-3, -2, -1))


def shan_chen_force(psi, G):
    """F(x) = -G psi(x) sum_a w_a psi(x + c_a) c_a (Eq. SC_force); [3, nz, ny, nx].

    The a = 0 term has c_0 = 0 and drops out.
    """
    w = lattice.weights()
    acc = torch.zeros((3,) + tuple(psi.shape), dtype=psi.dtype)
    for a in range(1, lattice.Q):
        pn = neighbour(psi, _C[a])
        for d in range(3):
            if _C[a][d] != 0:
                acc[d] = acc[d] + w[a] * _C[a][d] * pn
    return -G * psi.unsqueeze(0) * acc


def equilibrium(rho, u):
    """f^eq_a = w_a rho [1 + 3 c.u + 4.5 (c.u)^2 - 1.5 u.u] (Eq. local_eq, c_s^2 = 1/3)."""
    c = lattice.velocities().to(rho.dtype)
    w = lattice.weights().to(rho.dtype)
    cu = torch.einsum("ad,d...->a...", c, u)
    uu = (u * u).sum(dim=0)
    shape = (lattice.Q,) + (1,) * rho.dim()
    return w.view(shape) * rho.unsqueeze(0) * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu.unsqueeze(0))


def guo_source(u, F):
    """S_a = w_a [3 (c_a - u).F + 9 (c_a.u)(c_a.F)] (Guo et al. 2002 forcing term)."""
    c = lattice.velocities().to(u.dtype)
    w = lattice.weights().to(u.dtype)
    cu = torch.einsum("ad,d...->a...", c, u)
    cF = torch.einsum("ad,d...->a...", c, F)
    uF = (u * F).sum(dim=0)
    shape = (lattice.Q,) + (1,) * (u.dim() - 1)
    return w.view(shape) * (3.0 * (cF - uF.unsqueeze(0)) + 9.0 * cu * cF)


def collide_bgk_guo(f, feq, S, tau):
    """SRT with Guo source: f* = f - (f - f^eq)/tau + (1 - 1/(2 tau)) S."""
    return f - (f - feq) / tau + (1.0 - 0.5 / tau) * S


def collide_mrt_guo(f, feq, S, lam):
    """MRT with Guo source: f* = f - M^-1 Lambda M (f - f^eq) + M^-1 (I - Lambda/2) M S.

    M is the d'Humieres matrix, Lambda = diag(lam); M^-1 is obtained by a
    library inverse, not from the orthogonality of the rows.
    """
    M = lattice.mrt_matrix().to(f.dtype)
    Minv = torch.linalg.inv(M)
    lam = lam.to(f.dtype)
    m_neq = torch.einsum("ab,b...->a...", M, f - feq)
    m_src = torch.einsum("ab,b...->a...", M, S)
    shape = (lattice.Q,) + (1,) * (f.dim() - 1)
    lam_v = lam.view(shape)
    dm = -lam_v * m_neq + (1.0 - 0.5 * lam_v) * m_src
    return f + torch.einsum("ab,b...->a...", Minv, dm)


def stream(fstar):
    """f_a(x + c_a) = f*_a(x) on the periodic lattice (Eq. LBE)."""
    out = []
    for a in range(lattice.Q):
        cx, cy, cz = _C[a]
        out.append(torch.roll(fstar[a], shifts=(cz, cy, cx), dims=(-3, -2, -1)))
    return torch.stack(out, dim=0)


class Params:
    """Physical and numerical parameters of one run.

    collision: "bgk" or "mrt"; forcing: "guo" or "shift" (velocity shift, SRT
    only, Eq. vel_shift).  G is the paper's G_0; psi_rho0 its rho_0 (fixed to
    1.0 in the paper).  s_bulk, s_ghost are the MRT rates of the bulk and
    ghost rows; the shear rows relax at 1/tau.
    """

    def __init__(self, G=-5.0, tau=1.0, collision="bgk", forcing="guo",
                 psi_rho0=1.0, s_bulk=1.0, s_ghost=1.2, s_conserved=1.0):
        self.G = G
        self.tau = tau
        self.collision = collision
        self.forcing = forcing
        self.psi_rho0 = psi_rho0
        self.s_bulk = s_bulk
        self.s_ghost = s_ghost
        self.s_conserved = s_conserved

    def rates(self):
        return lattice.mrt_rates(self.tau, self.s_bulk, self.s_ghost, self.s_conserved)


def force_of_state(f, p):
    """Shan-Chen force of the state f (Eq. SC_force with psi of Sec. 2)."""
    psi = pseudo_potential(density(f), p.psi_rho0)
    return shan_chen_force(psi, p.G)


def barycentric_velocity(f, p, F=None):
    """u^b = u + F/(2 rho) = (j + F/2)/rho (Eq. barycentric)."""
    rho = density(f)
    j = momentum(f)
    if F is None:
        F = force_of_state(f, p)
    return (j + 0.5 * F) / rho.unsqueeze(0)


def collide(f, p):
    """Post-collision populations f* at every node (no streaming)."""
    rho = density(f)
    j = momentum(f)
    F = force_of_state(f, p)
    if p.forcing == "guo":
        ub = (j + 0.5 * F) / rho.unsqueeze(0)
        feq = equilibrium(rho, ub)
        S = guo_source(ub, F)
        if p.collision == "bgk":
            return collide_bgk_guo(f, feq, S, p.tau)
        if p.collision == "mrt":
            return collide_mrt_guo(f, feq, S, p.rates())
        raise ValueError(p.collision)
    if p.forcing == "shift":
        if p.collision != "bgk":
            raise ValueError("velocity-shift forcing is the SRT scheme")
        ushift = (j + p.tau * F) / rho.unsqueeze(0)
        feq = equilibrium(rho, ushift)
        return f - (f - feq) / p.tau
    raise ValueError(p.forcing)


def step(f, p):
    """One full time step: collide at x, stream to x + c_a (Eq. LBE)."""
    return stream(collide(f, p))


def run(f, p, nsteps):
    for _ in range(nsteps):
        f = step(f, p)
    return f


def init_rest(rho0):
    """Initial state at zero momentum: f_a = w_a rho0(x)."""
    w = lattice.weights().to(rho0.dtype)
    return w.view((lattice.Q,) + (1,) * rho0.dim()) * rho0.unsqueeze(0)
