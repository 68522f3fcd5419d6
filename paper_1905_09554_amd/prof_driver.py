"""Short, fixed workload for profiler runs (rocprofv3 kernel traces and HBM
counters).

    python -m paper_1905_09554_amd.prof_driver [--precision f32|f64] [--steps K]

Runs the benchmark box (256 x 256 x 1024 ligament, MRT, the launch shape the
benchmark uses) for a few steps, then a plain device-to-device copy of a known
size whose counters calibrate FETCH_SIZE and WRITE_SIZE.  With --adjoint it
runs the adjoint workload instead (64 x 64 x 256 MRT, 4000 steps, checkpoints
every 200, loss r_min; --adjoint-steps K for a shorter run followed by the
calibration copy): forward, loss gradient and backward, once.  With
--batch it runs the 64-ligament dispersion batch (3.9e8 nodes, FP32 BGK) for
--steps steps with one launch per step, then the same calibration copy (the
persistent cooperative form is timed with HIP events by the benchmark, not
under the profiler).  With --small it runs the 32 x 32 x 64 FP64 BGK box for
1000 steps, one launch per step.
"""
import argparse
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

COPY_BYTES = 1 << 30
WORKLOAD = "ligament_256x256x1024_mrt_f32"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--adjoint", action="store_true",
                    help="run the adjoint workload (forward with checkpoints, backward) instead")
    ap.add_argument("--adjoint-steps", type=int, default=None,
                    help="steps of the adjoint run (default: the workload's 4000); with this "
                         "option the calibration copy follows")
    ap.add_argument("--batch", action="store_true",
                    help="run the 64-ligament batch instead, one launch per step")
    ap.add_argument("--small", action="store_true",
                    help="run the 32 x 32 x 64 FP64 BGK box instead: 1000 steps, one launch each")
    args = ap.parse_args()

    import torch
    import lbm_inputs
    from paper_1905_09554_amd import lbsc, tuning

    if args.small:
        import time
        name = "ligament_32x32x64_bgk_f64"
        rho0, info = lbm_inputs.workload_density(name)
        nz, ny, nx = rho0.shape
        prm = lbsc.make_params(nx, ny, nz, collision="bgk", precision="f64", G=info["G"],
                               tau=info["tau"])
        sim = lbsc.Simulation(rho0, prm)
        sim.step(20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(1000)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        print("small done", name, "%.2f us per step (wall)" % (wall * 1e3), sim.get_tuning(),
              flush=True)
        sim.close()
        return

    if args.batch:
        from paper_1905_09554_amd import dispersion
        sweep = dispersion.make_sweep(seed=0)
        b = dispersion.build_batch(sweep, persistent=0)  # one launch per step, also when
        b.step(args.steps)                               # the tuned shape is persistent
        torch.cuda.synchronize()
        print("batch done", len(sweep["members"]), b.get_tuning(), flush=True)
        b.close()
        del b
        calibration_copy()
        return

    if args.adjoint:
        name = "adjoint_64x64x256_mrt_f32"
        rho0, info = lbm_inputs.workload_density(name)
        nz, ny, nx = rho0.shape
        prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision=args.precision,
                               G=info["G"], tau=info["tau"])
        sim = lbsc.Simulation(rho0, prm)
        steps = info["steps"] if args.adjoint_steps is None else args.adjoint_steps
        sim.adjoint_forward(steps, min(info["checkpoint_every"], steps))
        rhobar, rmin = sim.rmin_gradient(info["rho_v"], info["rho_l"])
        _, dG, dtau = sim.adjoint_backward(rhobar)
        torch.cuda.synchronize()
        print("adjoint done", name, args.precision, steps, rmin, dG, dtau, flush=True)
        sim.close()
        del sim
        if args.adjoint_steps is not None:
            calibration_copy()
        return

    rho0, info = lbm_inputs.workload_density(args.workload)
    nz, ny, nx = rho0.shape
    prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision=args.precision,
                           G=info["G"], tau=info["tau"], rho_ref=1.0)
    sim = lbsc.Simulation(rho0, prm)
    t = tuning.apply(sim, prm)
    sim.step(args.steps)
    torch.cuda.synchronize()
    print("steps done", args.steps, t, flush=True)
    sim.close()
    del sim
    calibration_copy()


def calibration_copy():
    """A plain device copy of COPY_BYTES, whose counters scale the kernel's."""
    import torch
    torch.cuda.empty_cache()
    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print("copy done", COPY_BYTES, flush=True)


if __name__ == "__main__":
    main()
