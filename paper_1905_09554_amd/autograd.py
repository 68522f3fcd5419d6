"""torch.autograd bridge for the hand-written adjoint.

``ligament_rmin(rho0, G, tau, config)`` returns the minimum ligament radius
after ``config['steps']`` steps (Sec. 4, Fig. 5 of the paper) as a torch
scalar that supports ``backward()``: the forward pass runs the HIP step with
checkpoints every ``config['segment']`` steps, the backward pass the HIP
adjoint (recomputing one segment at a time).  Gradients flow to rho0 (and
through torch to whatever built it, e.g. Fourier amplitudes of the initial
perturbation), to G and to tau.
"""
import torch

from . import lbsc


class LigamentRmin(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, G, tau, config):
        nz, ny, nx = rho0.shape
        params = lbsc.make_params(nx, ny, nz, collision=config["collision"],
                                  precision=config["precision"], G=float(G), tau=float(tau),
                                  s_bulk=config.get("s_bulk", 1.0),
                                  s_ghost=config.get("s_ghost", 1.2),
                                  rho_ref=config.get("rho_ref", 1.0))
        sim = lbsc.Simulation(rho0.detach().to("cpu", torch.float64).numpy(), params,
                              device=config.get("device", "cuda:0"))
        sim.adjoint_forward(config["steps"], config["segment"])
        rhobar, rmin = sim.rmin_gradient(config["rho_v"], config["rho_l"])
        ctx.sim = sim
        ctx.rhobar = rhobar
        ctx.rho0_device = rho0.device
        return torch.tensor(rmin, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        rho0bar, dG, dtau = ctx.sim.adjoint_backward(ctx.rhobar)
        ctx.sim.close()
        g = float(grad_out)
        return (rho0bar.to(ctx.rho0_device) * g, torch.tensor(dG * g, dtype=torch.float64),
                torch.tensor(dtau * g, dtype=torch.float64), None)


def ligament_rmin(rho0, G, tau, config):
    G = G if torch.is_tensor(G) else torch.tensor(float(G), dtype=torch.float64)
    tau = tau if torch.is_tensor(tau) else torch.tensor(float(tau), dtype=torch.float64)
    return LigamentRmin.apply(rho0, G, tau, config)
