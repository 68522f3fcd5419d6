"""torch.autograd bridge for the hand-written adjoint.

``ligament_rmin(rho0, G, tau, config)`` returns the minimum ligament radius
after ``config['steps']`` steps (Sec. 4, Fig. 5 of the paper) as a torch
scalar that supports ``backward()``: the forward pass runs the HIP step with
checkpoints every ``config['segment']`` steps, the backward pass the HIP
adjoint (recomputing one segment at a time).  Gradients flow to rho0 (and
through torch to whatever built it, e.g. Fourier amplitudes of the initial
perturbation), to G and to tau, and for MRT to the bulk and ghost relaxation
rates when they are passed as tensors.
"""
import torch

from . import lbsc


class LigamentRmin(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rho0, G, tau, s_bulk, s_ghost, config):
        nz, ny, nx = rho0.shape
        params = lbsc.make_params(nx, ny, nz, collision=config["collision"],
                                  precision=config["precision"], G=float(G), tau=float(tau),
                                  s_bulk=float(s_bulk), s_ghost=float(s_ghost),
                                  rho_ref=config.get("rho_ref", 1.0))
        sim = lbsc.Simulation(rho0.detach().to("cpu", torch.float64).numpy(), params,
                              device=config.get("device", "cuda:0"))
        sim.adjoint_forward(config["steps"], config["segment"])
        rhobar, rmin = sim.rmin_gradient(config["rho_v"], config["rho_l"])
        ctx.sim = sim
        ctx.rhobar = rhobar
        ctx.rho0_device = rho0.device
        # device and shape of each scalar input, for its gradient
        ctx.scalars = [(v.device, v.shape) for v in (G, tau, s_bulk, s_ghost)]
        return torch.tensor(rmin, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        rho0bar, dG, dtau = ctx.sim.adjoint_backward(ctx.rhobar)
        dsb, dsg = ctx.sim.rate_gradients()
        ctx.sim.close()
        g = float(grad_out)
        grads = [torch.full(shape, v * g, dtype=torch.float64, device=dev)
                 for v, (dev, shape) in zip((dG, dtau, dsb, dsg), ctx.scalars)]
        return (rho0bar.to(ctx.rho0_device) * g, *grads, None)


def ligament_rmin(rho0, G, tau, config, s_bulk=None, s_ghost=None):
    """r_min after config["steps"] steps; s_bulk and s_ghost default to
    config["s_bulk"] (1.0) and config["s_ghost"] (1.2) and take gradients when
    given as tensors that require them."""
    def as_t(v):
        return v if torch.is_tensor(v) else torch.tensor(float(v), dtype=torch.float64)

    s_bulk = config.get("s_bulk", 1.0) if s_bulk is None else s_bulk
    s_ghost = config.get("s_ghost", 1.2) if s_ghost is None else s_ghost
    return LigamentRmin.apply(rho0, as_t(G), as_t(tau), as_t(s_bulk), as_t(s_ghost), config)
