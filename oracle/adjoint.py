"""Reference gradients by automatic differentiation of the oracle (float64).

Test infrastructure only.  The loss is the minimum ligament radius after a
number of steps (Sec. 4, Fig. 5: the smallest radial coordinate of the
interface, here r(z) = sqrt(A(z)/pi) as in ``diagnostics``).  torch autograd
through the whole oracle run gives dL/drho0, dL/dG and dL/dtau, and for MRT
dL/ds_bulk and dL/ds_ghost (the bulk and ghost relaxation rates); segments are
wrapped in ``torch.utils.checkpoint`` so memory stays bounded, which does not
change the arithmetic.

Pin: the same gradients by central finite differences of the oracle itself
(tests/test_oracle_adjoint.py).
"""
import torch
from torch.utils.checkpoint import checkpoint

from . import diagnostics, lbm


def rmin_after(rho0, G, tau, steps, rho_v, rho_l, collision="bgk", s_bulk=1.0, s_ghost=1.2,
               segment=25):
    """Minimum radius after `steps` steps from f = w rho0 (differentiable)."""
    p = lbm.Params(G=G, tau=tau, collision=collision, s_bulk=s_bulk, s_ghost=s_ghost)
    f = lbm.init_rest(rho0)

    def run(fin, k):
        for _ in range(k):
            fin = lbm.step(fin, p)
        return fin

    done = 0
    while done < steps:
        k = min(segment, steps - done)
        if f.requires_grad:
            f = checkpoint(run, f, k, use_reentrant=False)
        else:
            f = run(f, k)
        done += k
    r = diagnostics.radius_profile(lbm.density(f), rho_v, rho_l)
    return r.min()


def rmin_gradients(rho0, G, tau, steps, rho_v, rho_l, **kw):
    """(r_min, dL/drho0 [nz,ny,nx], dL/dG, dL/dtau) by autograd."""
    rho0 = torch.as_tensor(rho0, dtype=torch.float64).clone().requires_grad_(True)
    Gt = torch.tensor(float(G), dtype=torch.float64, requires_grad=True)
    taut = torch.tensor(float(tau), dtype=torch.float64, requires_grad=True)
    loss = rmin_after(rho0, Gt, taut, steps, rho_v, rho_l, **kw)
    loss.backward()
    return float(loss.detach()), rho0.grad.detach(), float(Gt.grad), float(taut.grad)


def rmin_rate_gradients(rho0, G, tau, steps, rho_v, rho_l, s_bulk, s_ghost, segment=25):
    """(r_min, dL/ds_bulk, dL/ds_ghost) of the MRT run by autograd."""
    sb = torch.tensor(float(s_bulk), dtype=torch.float64, requires_grad=True)
    sg = torch.tensor(float(s_ghost), dtype=torch.float64, requires_grad=True)
    rho0 = torch.as_tensor(rho0, dtype=torch.float64).clone().requires_grad_(True)
    loss = rmin_after(rho0, G, tau, steps, rho_v, rho_l, collision="mrt", s_bulk=sb, s_ghost=sg,
                      segment=segment)
    loss.backward()
    return float(loss.detach()), float(sb.grad), float(sg.grad)
