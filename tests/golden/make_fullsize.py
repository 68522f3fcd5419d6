"""Writes the oracle's expected values for the full-size parity windows.

Calls only the oracle (float64 CPU) and the input builder.  Run from the
repository root (10-25 minutes per case on 8 cores, up to 20 GB of memory):

    python tests/golden/make_fullsize.py [case ...]

Cases (the ligament inputs of lbm_inputs.WORKLOADS, seed 0):

  c2_bgk, c2_mrt  128 x 128 x 512, R = 32, kR_eff = 0.785, A = 0.05, noise
                  U(+-1e-4); 200 steps of the whole box (one step couples
                  nodes up to two links apart, so 200 steps reach every plane
                  of the 512-plane box).
  c2_srt_shift    the same box and input, BGK with the velocity-shift forcing
                  (the paper's SRT operator), tau = 1; 200 steps, whole box.
  c2_mrt_paper    the same box and input, MRT with the paper's rate set
                  (shear and bulk 1/tau, every other rate 1), tau = 0.8;
                  200 steps, whole box.
  c3_mrt          256 x 256 x 1024 MRT, R = 64, kR_eff = 0.785, noise U(+-1e-4);
                  50 steps.  After k steps a node depends only on the nodes
                  within 2k links, so the oracle runs the slab of planes
                  z0 - 104 .. z0 + 103 around the neck plane z0 = 256 with its
                  own periodic wrap: the wrap's error travels two planes per
                  step from the slab's ends and stays more than 100 planes
                  away from z0 after 50 steps.

Output: tests/golden/fullsize_<case>.npz with the density rho and the
barycentric velocity u^b (Eq. barycentric) after the run at the sampled nodes
of plane z0: the whole row y = ny/2 and column x = nx/2 through the axis, and a
regular grid of every `stride`-th node.  Arrays: z0, y, x (node indices),
rho, u (3 x m), steps.
"""
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lbm_inputs  # noqa: E402
from oracle import lbm  # noqa: E402

CASES = {
    "c2_bgk": dict(workload="ligament_128x128x512", collision="bgk", steps=200, z0=128,
                   slab=None, stride=2),
    "c2_mrt": dict(workload="ligament_128x128x512", collision="mrt", steps=200, z0=128,
                   slab=None, stride=2),
    "c3_mrt": dict(workload="ligament_256x256x1024_mrt_f32", collision="mrt", steps=50, z0=256,
                   slab=104, stride=4),
    "c2_srt_shift": dict(workload="ligament_128x128x512", collision="bgk", forcing="shift",
                         steps=200, z0=128, slab=None, stride=2),
    "c2_mrt_paper": dict(workload="ligament_128x128x512", collision="mrt", tau=0.8,
                         s_bulk=1.0 / 0.8, s_ghost=1.0, steps=200, z0=128, slab=None, stride=2),
}


def case_params(c, info):
    """The oracle's parameters of case c (the workload's G and tau unless the
    case sets its own; MRT ghost 1.2 and bulk 1.0 unless set)."""
    return lbm.Params(G=info["G"], tau=c.get("tau", info["tau"]), collision=c["collision"],
                      forcing=c.get("forcing", "guo"), s_bulk=c.get("s_bulk", 1.0),
                      s_ghost=c.get("s_ghost", 1.2))


def sample_nodes(nx, ny, stride):
    """(y, x) of the row and column through the axis and a strided grid."""
    pts = {(ny // 2, x) for x in range(nx)} | {(y, nx // 2) for y in range(ny)}
    pts |= {(y, x) for y in range(0, ny, stride) for x in range(0, nx, stride)}
    pts = sorted(pts)
    return np.array([p[0] for p in pts]), np.array([p[1] for p in pts])


def run_case(name):
    c = CASES[name]
    rho0, info = lbm_inputs.workload_density(c["workload"])
    nz = rho0.shape[0]
    z0 = c["z0"]
    if c["slab"] is not None:
        planes = [(z0 + d) % nz for d in range(-c["slab"], c["slab"])]
        rho0 = np.ascontiguousarray(rho0[planes])
        zl = c["slab"]
    else:
        zl = z0
    p = case_params(c, info)
    t = time.time()
    f = lbm.init_rest(torch.from_numpy(rho0))
    del rho0
    for k in range(c["steps"]):
        f = lbm.step(f, p)
        if (k + 1) % 10 == 0:
            print("%s: step %d, %.0f s" % (name, k + 1, time.time() - t), flush=True)
    rho = lbm.density(f)[zl]
    ub = lbm.barycentric_velocity(f, p)[:, zl]
    ny, nx = rho.shape
    ys, xs = sample_nodes(nx, ny, c["stride"])
    out = os.path.join(ROOT, "tests", "golden", "fullsize_%s.npz" % name)
    np.savez(out, z0=np.int64(z0), y=ys, x=xs, rho=rho.numpy()[ys, xs],
             u=ub.numpy()[:, ys, xs], steps=np.int64(c["steps"]), tau=np.float64(p.tau),
             s_bulk=np.float64(p.s_bulk), s_ghost=np.float64(p.s_ghost),
             forcing=np.str_(p.forcing))
    print("wrote", out, flush=True)


def main():
    names = sys.argv[1:] or list(CASES)
    for n in names:
        run_case(n)


if __name__ == "__main__":
    main()
