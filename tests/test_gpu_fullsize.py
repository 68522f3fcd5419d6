"""Full-size runs in the launch configuration the benchmark times, checked on
sampled nodes: the oracle computes each sampled node from a periodic patch of
the same initial field (after k steps a node depends only on nodes within 2k
links, and its u^b on one link more), so the comparison is exact up to
rounding."""
import numpy as np
import pytest
import torch

import lbm_inputs
from tests import gpu_cases as gc

pytestmark = pytest.mark.gpu


def _sample_nodes(shape, tune, rng, count=24):
    nz, ny, nx = shape
    bx, by, zc = tune["block_x"], tune["block_y"], tune["z_chunk"]
    zs = sorted({0, zc - 1, zc % nz, nz - 1, (2 * zc) % nz})
    ys = sorted({0, by - 1, by % ny, ny - 1, (ny // by // 2) * by % ny})
    xs = sorted({0, bx - 1, bx % nx, nx - 1, nx // 2})
    nodes = [(z, y, x) for z in zs for y in ys for x in xs]
    pick = rng.choice(len(nodes), size=min(count, len(nodes)), replace=False)
    out = [nodes[i] for i in sorted(pick)]
    out += [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(8)]
    return out


@pytest.mark.parametrize("name,coll,prec,steps,kR", [
    ("ligament_256x256x1024_mrt_f32", "mrt", "f32", 2, None),
    ("ligament_256x256x1024_mrt_f32", "mrt", "f64", 2, 0.45),
    ("ligament_128x128x512", "bgk", "f64", 2, None),
    ("ligament_128x128x512", "mrt", "f32", 3, None),
])
def test_full_size_sampled(name, coll, prec, steps, kR):
    from paper_1905_09554_amd import lbsc, tuning
    rho0, info = lbm_inputs.workload_density(name, kR=kR)
    nz, ny, nx = rho0.shape
    print("full size %s %s %s kR_eff %.4f: %d nodes" % (name, coll, prec, info["kR_eff"],
                                                       rho0.size), flush=True)
    prm = lbsc.make_params(nx, ny, nz, collision=coll, precision=prec, G=info["G"],
                           tau=info["tau"])
    sim = lbsc.Simulation(rho0, prm)
    tuning.apply(sim, prm)
    sim.step(steps)
    rho, u, _ = sim.moments(want_p=False)
    tune = sim.get_tuning()
    rng = np.random.default_rng(11)
    nodes = _sample_nodes(rho0.shape, tune, rng)
    idx = torch.tensor(nodes, device=rho.device)
    rho_s = rho[idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    u_s = u[:, idx[:, 0], idx[:, 1], idx[:, 2]].cpu().numpy()
    sim.close()
    del rho, u
    torch.cuda.empty_cache()
    rtol = 1e-12 if prec == "f64" else 1e-5
    utol = 1e-12 if prec == "f64" else 1e-6
    for k, node in enumerate(nodes):
        r_ref, u_ref = gc.oracle_at_node(rho0, node, steps, coll, G=info["G"], tau=info["tau"])
        assert abs(rho_s[k] - r_ref) <= rtol * r_ref, (node, rho_s[k], r_ref)
        assert float(np.abs(u_s[:, k] - u_ref).max()) <= utol, (node, u_s[:, k], u_ref)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_two_kernel_form_full_size_bitwise(prec):
    """The benchmark box in the two-kernel form: density and velocity after
    3 steps equal the fused kernel's bitwise (same arithmetic, psi through
    global memory instead of LDS)."""
    from paper_1905_09554_amd import lbsc
    name = "ligament_256x256x1024_mrt_f32"
    rho0, info = lbm_inputs.workload_density(name)
    nz, ny, nx = rho0.shape
    print("two-kernel full size %s %s" % (name, prec), flush=True)
    prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision=prec, G=info["G"],
                           tau=info["tau"])
    out = []
    for two in (0, 1):
        sim = lbsc.Simulation(rho0, prm)
        if two:
            sim.set_tuning(two_kernel=1)
        sim.step(3)
        rho, u, _ = sim.moments(want_p=False)
        torch.cuda.synchronize()
        sim.close()
        out.append((rho, u))
        del sim
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    del out
    torch.cuda.empty_cache()
