"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the float64 oracle on the same seeded input, and line up their
population orders by velocity vector."""
import functools

import numpy as np
import torch

import lbm_inputs
from oracle import lattice, lbm

CONFIG1 = dict(nx=32, ny=32, nz=64, R=8, amp=0.1, mode=1, G=-5.0, tau=1.0)


def population_perm():
    """perm[a] = library index of the oracle's velocity a."""
    from paper_1905_09554_amd import lbsc
    c_lib, _ = lbsc.lattice()
    idx = {tuple(v): i for i, v in enumerate(c_lib.tolist())}
    return [idx[c] for c in lattice.C_INT]


def ligament(nx, ny, nz, R, amp=0.1, mode=1, G=-5.0, noise=0.0, seed=0):
    rv, rl = lbm_inputs.coexistence(G)
    return lbm_inputs.ligament_density(nx, ny, nz, R, amp, mode, rv, rl, noise=noise, seed=seed)


def run_gpu(rho0, steps, collision="bgk", forcing="guo", precision="f64", G=-5.0, tau=1.0,
            s_bulk=1.0, s_ghost=1.2, rho_ref=1.0, tuning=None, want_state=True):
    """Returns dict(state (oracle order, float64), rho, u, p) after `steps`."""
    from paper_1905_09554_amd import lbsc
    nz, ny, nx = rho0.shape
    prm = lbsc.make_params(nx, ny, nz, collision=collision, forcing=forcing,
                           precision=precision, G=G, tau=tau, s_bulk=s_bulk, s_ghost=s_ghost,
                           rho_ref=rho_ref)
    sim = lbsc.Simulation(rho0, prm, device="cuda:0")
    if tuning:
        sim.set_tuning(**tuning)
    sim.step(steps)
    rho, u, p = sim.moments()
    torch.cuda.synchronize()
    out = {"rho": rho.cpu().numpy(), "u": u.cpu().numpy(), "p": p.cpu().numpy(), "sim": sim}
    if want_state:
        st, count = sim.get_state()
        assert count == steps
        st = st.astype(np.float64)
        if precision == "f32":
            _, w = lbsc.lattice()
            st = st + (w * rho_ref)[:, None, None, None]
        out["state"] = st[population_perm()]
    return out


@functools.lru_cache(maxsize=16)
def _oracle_cached(key):
    (shape, rho_bytes, steps, collision, forcing, G, tau, s_bulk, s_ghost) = key
    rho0 = np.frombuffer(rho_bytes, dtype=np.float64).reshape(shape)
    p = lbm.Params(G=G, tau=tau, collision=collision, forcing=forcing, s_bulk=s_bulk,
                   s_ghost=s_ghost)
    f = lbm.run(lbm.init_rest(torch.from_numpy(rho0.copy())), p, steps)
    rho = lbm.density(f)
    ub = lbm.barycentric_velocity(f, p)
    from oracle import diagnostics
    pr = diagnostics.pressure(rho, G)
    return {"state": f.numpy(), "rho": rho.numpy(), "u": ub.numpy(), "p": pr.numpy(), "f": f,
            "params": p}


def run_oracle(rho0, steps, collision="bgk", forcing="guo", G=-5.0, tau=1.0, s_bulk=1.0,
               s_ghost=1.2):
    key = (rho0.shape, np.ascontiguousarray(rho0).tobytes(), steps, collision, forcing, G, tau,
           s_bulk, s_ghost)
    return _oracle_cached(key)


def periodic_patch(field, center, radius):
    """field[(c + d) mod n] for d in [-r, r]^3; field is [nz, ny, nx]."""
    z, y, x = center
    nz, ny, nx = field.shape
    iz = [(z + d) % nz for d in range(-radius, radius + 1)]
    iy = [(y + d) % ny for d in range(-radius, radius + 1)]
    ix = [(x + d) % nx for d in range(-radius, radius + 1)]
    return field[np.ix_(iz, iy, ix)]


def oracle_at_node(rho0, center, steps, collision, G=-5.0, tau=1.0, s_bulk=1.0, s_ghost=1.2):
    """(rho, u^b) of one node after `steps`, from a periodic patch of radius
    2 steps + 2: one step couples nodes at most two links apart (force one
    link, streaming one more), u^b needs the force, hence one link beyond."""
    r = 2 * steps + 2
    patch = periodic_patch(rho0, center, r)
    p = lbm.Params(G=G, tau=tau, collision=collision, s_bulk=s_bulk, s_ghost=s_ghost)
    f = lbm.run(lbm.init_rest(torch.from_numpy(np.ascontiguousarray(patch))), p, steps)
    rho = lbm.density(f)
    ub = lbm.barycentric_velocity(f, p)
    return float(rho[r, r, r]), ub[:, r, r, r].numpy()
