"""The hand-written adjoint (through the C ABI) against the oracle's autograd
gradient and against central finite differences of the GPU forward run.

Loss: minimum ligament radius after the run (Sec. 4, Fig. 5).  Gradients with
respect to G, tau, the MRT bulk and ghost rates, the initial density, and
through torch to the Fourier amplitudes of the initial radius.
"""
import math

import numpy as np
import pytest
import torch

import lbm_inputs
from oracle import adjoint as oadj
from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu


def _gpu_grads(rho0, G, tau, steps, segment, coll, prec, rv, rl, rates=False):
    from paper_1905_09554_amd import lbsc
    nz, ny, nx = rho0.shape
    prm = lbsc.make_params(nx, ny, nz, collision=coll, precision=prec, G=G, tau=tau)
    sim = lbsc.Simulation(rho0, prm)
    sim.adjoint_forward(steps, segment)
    rhobar, rmin = sim.rmin_gradient(rv, rl)
    g_rho, g_G, g_tau = sim.adjoint_backward(rhobar)
    out = (rmin, g_rho.cpu().numpy(), g_G, g_tau)
    if rates:
        out = out + sim.rate_gradients()
    sim.close()
    return out


def _rmin(rho0, G, tau, steps, coll, prec, rv, rl, s_bulk=1.0, s_ghost=1.2):
    from paper_1905_09554_amd import lbsc
    nz, ny, nx = rho0.shape
    prm = lbsc.make_params(nx, ny, nz, collision=coll, precision=prec, G=G, tau=tau,
                           s_bulk=s_bulk, s_ghost=s_ghost)
    sim = lbsc.Simulation(rho0, prm)
    sim.step(steps)
    r = sim.diagnostics(rv, rl)["r_min"]
    sim.close()
    return r


@pytest.mark.parametrize("coll", ["bgk", "mrt"])
def test_adjoint_matches_oracle_autograd(coll):
    rv, rl = lbm_inputs.coexistence(-5.0)
    rho0 = lbm_inputs.ligament_density(16, 16, 40, 4.5, 0.1, 1, rv, rl, noise=1e-3, seed=3)
    steps, seg = 60, 16
    rmin, g_rho, g_G, g_tau = _gpu_grads(rho0, -5.0, 0.9, steps, seg, coll, "f64", rv, rl)
    o_rmin, o_rho, o_G, o_tau = oadj.rmin_gradients(torch.from_numpy(rho0), -5.0, 0.9, steps,
                                                    rv, rl, collision=coll, segment=20)
    print("%s: r_min %.6f  dG %.6e (oracle %.6e)  dtau %.6e (oracle %.6e)"
          % (coll, rmin, g_G, o_G, g_tau, o_tau), flush=True)
    assert abs(rmin - o_rmin) < 1e-12
    assert abs(g_G - o_G) <= 1e-9 * abs(o_G)
    assert abs(g_tau - o_tau) <= 1e-9 * abs(o_tau)
    o_rho = o_rho.numpy()
    assert float(np.abs(g_rho - o_rho).max()) <= 1e-9 * float(np.abs(o_rho).max())


def test_mrt_rate_gradients_match_oracle_autograd():
    """dL/ds_bulk and dL/ds_ghost of the MRT adjoint against the oracle's
    autograd (itself pinned to finite differences); BGK reports zeros."""
    rv, rl = lbm_inputs.coexistence(-5.0)
    rho0 = lbm_inputs.ligament_density(16, 16, 40, 4.5, 0.1, 1, rv, rl, noise=1e-3, seed=3)
    steps, seg = 60, 16
    out = _gpu_grads(rho0, -5.0, 0.9, steps, seg, "mrt", "f64", rv, rl, rates=True)
    g_b, g_g = out[4], out[5]
    o_rmin, o_b, o_g = oadj.rmin_rate_gradients(torch.from_numpy(rho0), -5.0, 0.9, steps, rv,
                                                rl, 1.0, 1.2, segment=20)
    print("ds_bulk %.8e (oracle %.8e)  ds_ghost %.8e (oracle %.8e)" % (g_b, o_b, g_g, o_g),
          flush=True)
    assert abs(out[0] - o_rmin) < 1e-12
    assert abs(g_b - o_b) <= 1e-9 * abs(o_b) and abs(g_g - o_g) <= 1e-9 * abs(o_g)
    bgk = _gpu_grads(rho0, -5.0, 0.9, steps, seg, "bgk", "f64", rv, rl, rates=True)
    assert bgk[4] == 0.0 and bgk[5] == 0.0


def _fourier_case(nx, ny, nz, R, nmodes, seed):
    rv, rl = lbm_inputs.coexistence(-5.0)
    amps = lbm_inputs.fourier_amplitudes(nmodes, R, 0.02, seed)
    return amps, rv, rl


def _rho_from_amps(amps, nx, ny, nz, R, rv, rl):
    r = lbm_inputs.fourier_radius(nz, R, amps)
    return lbm_inputs.density_from_radius(nx, ny, r, rv, rl)


@pytest.mark.parametrize("prec,tol", [("f64", 1e-6), ("f32", 1e-4)])
def test_adjoint_matches_central_differences(prec, tol):
    from paper_1905_09554_amd import autograd as lag
    nx = ny = 24
    nz, R, steps, seg = 64, 6.0, 300, 64
    amps, rv, rl = _fourier_case(nx, ny, nz, R, 8, seed=1)
    cfg = dict(collision="mrt", precision=prec, steps=steps, segment=seg, rho_v=rv, rho_l=rl)
    a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
    G = torch.tensor(-5.0, dtype=torch.float64, requires_grad=True)
    tau = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    sb = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    sg = torch.tensor(1.2, dtype=torch.float64, requires_grad=True)
    r = lbm_inputs.fourier_radius_torch(nz, R, a)
    rho0 = lbm_inputs.density_from_radius_torch(nx, ny, r, rv, rl)
    loss = lag.ligament_rmin(rho0, G, tau, cfg, s_bulk=sb, s_ghost=sg)
    loss.backward()
    h = 1e-4

    def L(am=amps, Gv=-5.0, tv=1.0, bv=1.0, gv=1.2):
        # Finite differences in float64 whatever the adjoint's precision.
        return _rmin(_rho_from_amps(am, nx, ny, nz, R, rv, rl), Gv, tv, steps, "mrt", "f64",
                     rv, rl, s_bulk=bv, s_ghost=gv)

    fd = {"G": (L(Gv=-5.0 + h) - L(Gv=-5.0 - h)) / (2 * h),
          "tau": (L(tv=1.0 + h) - L(tv=1.0 - h)) / (2 * h),
          "s_bulk": (L(bv=1.0 + h) - L(bv=1.0 - h)) / (2 * h),
          "s_ghost": (L(gv=1.2 + h) - L(gv=1.2 - h)) / (2 * h)}
    ad = {"G": float(G.grad), "tau": float(tau.grad), "s_bulk": float(sb.grad),
          "s_ghost": float(sg.grad)}
    for m in (0, 1, 5):
        e = np.zeros_like(amps)
        e[m] = h
        fd["a%d" % (m + 1)] = (L(am=amps + e) - L(am=amps - e)) / (2 * h)
        ad["a%d" % (m + 1)] = float(a.grad[m])
    for k in fd:
        print("%s %s: adjoint %.8e  fd %.8e  rel err %.2e"
              % (prec, k, ad[k], fd[k], abs(ad[k] - fd[k]) / abs(fd[k])), flush=True)
    # Each component within tol of itself, except a component below 1e-3 of
    # the largest: dL/ds_ghost here is 7e-7 against 0.85 for dL/da1.  Central
    # differences of the float64 loss resolve it only to about 1e-11, and the
    # float32 run's own rounding moves it by about 2e-8 (3 % of itself, 3e-8 of
    # the gradient's scale), so such a component is held to tol times 1e-3 of
    # the largest component instead.
    scale = max(abs(v) for v in fd.values())
    for k in fd:
        bound = tol * abs(fd[k]) if abs(fd[k]) >= 1e-3 * scale else tol * 1e-3 * scale
        assert abs(ad[k] - fd[k]) <= bound, k


def test_config5_full_size_adjoint_against_fd():
    """64 x 64 x 256, R = 16, 32 Fourier modes (std 0.02 R), MRT, loss r_min
    at step 4000, checkpoints every 200 steps.  The float32 adjoint and the
    float64 adjoint against float64 central differences (h = 1e-4)."""
    from paper_1905_09554_amd import autograd as lag
    w = lbm_inputs.WORKLOADS["adjoint_64x64x256_mrt_f32"]
    nx, ny, nz, R = w["nx"], w["ny"], w["nz"], w["R"]
    amps, rv, rl = _fourier_case(nx, ny, nz, R, w["nmodes"], w["seed"])
    steps, seg = w["steps"], w["checkpoint_every"]
    res = {}
    for prec in ("f32", "f64"):
        cfg = dict(collision="mrt", precision=prec, steps=steps, segment=seg, rho_v=rv, rho_l=rl)
        a = torch.tensor(amps, dtype=torch.float64, requires_grad=True)
        G = torch.tensor(w["G"], dtype=torch.float64, requires_grad=True)
        tau = torch.tensor(w["tau"], dtype=torch.float64, requires_grad=True)
        rho0 = lbm_inputs.density_from_radius_torch(nx, ny, lbm_inputs.fourier_radius_torch(nz, R, a),
                                                    rv, rl)
        loss = lag.ligament_rmin(rho0, G, tau, cfg)
        loss.backward()
        res[prec] = {"r_min": float(loss.detach()), "G": float(G.grad), "tau": float(tau.grad),
                     "a1": float(a.grad[0]), "a2": float(a.grad[1]), "a9": float(a.grad[8])}
        print(prec, res[prec], flush=True)
    h = 1e-4

    def L(am=amps, Gv=w["G"], tv=w["tau"]):
        return _rmin(_rho_from_amps(am, nx, ny, nz, R, rv, rl), Gv, tv, steps, "mrt", "f64", rv, rl)

    fd = {"G": (L(Gv=w["G"] + h) - L(Gv=w["G"] - h)) / (2 * h),
          "tau": (L(tv=w["tau"] + h) - L(tv=w["tau"] - h)) / (2 * h)}
    for m in (0, 1, 8):
        e = np.zeros_like(amps)
        e[m] = h
        fd["a%d" % (m + 1)] = (L(am=amps + e) - L(am=amps - e)) / (2 * h)
    print("fd", fd, flush=True)
    for k in fd:
        e64 = abs(res["f64"][k] - fd[k]) / abs(fd[k])
        e32 = abs(res["f32"][k] - fd[k]) / abs(fd[k])
        print("%s: fd %.9e, f64 rel err %.2e, f32 rel err %.2e" % (k, fd[k], e64, e32), flush=True)
        # float64 adjoint: exact gradient of the float64 run (FD truncation
        # error ~1e-8); float32 storage: gradient of the float32 run (adjoint
        # arithmetic in float64), which differs from the float64 run by its
        # rounding.  Both relative to each component itself.
        assert e64 <= 1e-6, ("f64", k, e64)
        assert e32 <= 1e-4, ("f32", k, e32)


def test_parameter_gradients_follow_their_inputs():
    """G and tau given as one-element float32 tensors on the GPU get
    gradients of their own shape and device, equal to the float64 scalar
    case."""
    from paper_1905_09554_amd import autograd as lag
    nx = ny = 16
    nz, R = 32, 4.0
    rv, rl = lbm_inputs.coexistence(-5.0)
    rho0 = torch.from_numpy(lbm_inputs.ligament_density(nx, ny, nz, R, 0.1, 1, rv, rl))
    cfg = dict(collision="mrt", precision="f64", steps=40, segment=16, rho_v=rv, rho_l=rl)
    G1 = torch.tensor(-5.0, dtype=torch.float64, requires_grad=True)
    t1 = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    lag.ligament_rmin(rho0, G1, t1, cfg).backward()
    G2 = torch.tensor([-5.0], dtype=torch.float32, device="cuda:0", requires_grad=True)
    t2 = torch.tensor([1.0], dtype=torch.float32, device="cuda:0", requires_grad=True)
    lag.ligament_rmin(rho0, G2, t2, cfg).backward()
    for a, b in ((G1, G2), (t1, t2)):
        assert b.grad.shape == (1,) and b.grad.device.type == "cuda"
        assert b.grad.dtype == torch.float32
        assert abs(float(b.grad[0]) - float(a.grad)) <= 1e-6 * abs(float(a.grad))
