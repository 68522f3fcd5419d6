"""Full-size parity windows against the oracle, in the launch configuration
the benchmark uses: the 128 x 128 x 512 ligament over 200 steps (BGK and MRT
with Guo forcing, and the paper's two operators: BGK with the velocity shift,
MRT with its rate set) and the 256 x 256 x 1024 MRT ligament over 50 steps,
each in float64 and in float32 shifted storage.

The expected values are the oracle's, written by tests/golden/make_fullsize.py
(the whole 128 x 128 x 512 box; for 256 x 256 x 1024 a slab of 208 planes
around the neck plane, which after 50 steps equals the whole box there since
one step couples nodes at most two links apart).  Compared at the stored
sample nodes of one plane: the row and column through the axis and a regular
grid.

Tolerances: float64, density within 1e-12 relative and u^b within 1e-12;
float32 shifted storage, density within 1e-5 relative of the float64 oracle
(the float32 bar) and u^b within 1e-5 (the velocity error is reported).
"""
import os

import numpy as np
import pytest
import torch

import lbm_inputs

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

CASES = {
    "c2_bgk": ("ligament_128x128x512", "bgk"),
    "c2_mrt": ("ligament_128x128x512", "mrt"),
    "c2_srt_shift": ("ligament_128x128x512", "bgk"),
    "c2_mrt_paper": ("ligament_128x128x512", "mrt"),
    "c3_mrt": ("ligament_256x256x1024_mrt_f32", "mrt"),
}


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_full_size_window_against_oracle(case, prec):
    from paper_1905_09554_amd import lbsc, tuning
    workload, coll = CASES[case]
    ref = np.load(os.path.join(GOLDEN, "fullsize_%s.npz" % case))
    steps, z0 = int(ref["steps"]), int(ref["z0"])
    rho0, info = lbm_inputs.workload_density(workload)
    nz, ny, nx = rho0.shape
    print("full-size window %s %s %s: %d steps, plane %d, %d sampled nodes"
          % (case, workload, prec, steps, z0, ref["rho"].size), flush=True)
    if "forcing" in ref.files:
        print("  forcing %s, tau %g, s_bulk %g, s_ghost %g" % (ref["forcing"], ref["tau"],
                                                             ref["s_bulk"], ref["s_ghost"]),
              flush=True)
    # Forcing, tau and MRT rates as the oracle ran them (stored with its values;
    # files without them used Guo forcing, the workload's tau, bulk 1.0, ghost 1.2).
    forcing = str(ref["forcing"]) if "forcing" in ref.files else "guo"
    tau = float(ref["tau"]) if "tau" in ref.files else info["tau"]
    s_bulk = float(ref["s_bulk"]) if "s_bulk" in ref.files else 1.0
    s_ghost = float(ref["s_ghost"]) if "s_ghost" in ref.files else 1.2
    prm = lbsc.make_params(nx, ny, nz, collision=coll, forcing=forcing, precision=prec,
                           G=info["G"], tau=tau, s_bulk=s_bulk, s_ghost=s_ghost)
    sim = lbsc.Simulation(rho0, prm)
    tuning.apply(sim, prm)
    sim.step(steps)
    rho, u, _ = sim.moments(want_p=False)
    ys = torch.from_numpy(ref["y"]).to(rho.device)
    xs = torch.from_numpy(ref["x"]).to(rho.device)
    rho_s = rho[z0][ys, xs].cpu().numpy()
    u_s = u[:, z0][:, ys, xs].cpu().numpy()
    sim.close()
    del rho, u, sim
    torch.cuda.empty_cache()
    e_rho = float((np.abs(rho_s - ref["rho"]) / ref["rho"]).max())
    e_u = float(np.abs(u_s - ref["u"]).max())
    print("  max rel drho %.3e, max |du| %.3e (max |u| %.3e)"
          % (e_rho, e_u, float(np.abs(ref["u"]).max())), flush=True)
    if prec == "f64":
        assert e_rho <= 1e-12 and e_u <= 1e-12
    else:
        assert e_rho <= 1e-5 and e_u <= 1e-5
