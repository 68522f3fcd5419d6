"""Throughput of the D3Q19 Shan-Chen step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one full time step of the method (streaming, moments, psi, force
gather, forcing, collision) over the whole box; the interface diagnostics
(minimum radius, mass, momentum) run every 100 steps inside the timed
region.  The workload is a 256 x 256 x 1024 periodic box (67.1 M nodes)
holding a perturbed ligament of radius 64, D3Q19 MRT, Guo forcing, G = -5,
float32 shifted storage; the same box is also run in float64.

Prints one JSON line: MLUPS (million lattice-node updates per second),
the fraction of the HBM roofline reached by the step kernel, and the float64
oracle timed on the host cores on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Measured ceilings on MI355X (hand-written probe,
# paper_1905_09554_amd/csrc/hbm_probe.hip), reported beside the published
# peak: the fastest plain copy (one pass, 16 bytes per lane, one 256-thread
# group per 4 KiB) and the step's own access pattern without its stencil
# (19 pulled loads and 19 stores per node, 1024-thread groups of 256 x 4
# tiles marching 128 planes, populations in blocks of 1024 nodes).
COPY_CEILING_GBS = 6324.0
PULL_PATTERN_GBS = 5294.0
WORKLOAD = "ligament_256x256x1024_mrt_f32"
METRIC = "MLUPS & % HBM peak, D3Q19 Shan-Chen FP32 vs FP64; adjoint/forward cost ratio"
DIAG_EVERY = 100
# Algorithmic bytes per node and step: 19 populations read + 19 written.
BYTES_PER_NODE = {"f32": 19 * 2 * 4, "f64": 19 * 2 * 8}


def kernel_source_hash():
    h = hashlib.sha256()
    for name in ("lbsc_device.hip", "lbsc_api.hip", "lbsc_internal.h"):
        with open(os.path.join(ROOT, "paper_1905_09554_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def launch_shape_entry(workload, precision):
    """The autotuner's launch shape for a single-box workload (None: the
    library default)."""
    import lbm_inputs
    from paper_1905_09554_amd import lbsc, tuning
    w = lbm_inputs.WORKLOADS[workload]
    prm = lbsc.make_params(w["nx"], w["ny"], w["nz"], collision=w["collision"],
                           precision=precision)
    return tuning.lookup(prm)


def measured_traffic(workload, precision):
    """HBM bytes per step-kernel launch from the committed rocprofv3 counter
    runs, or None when absent or taken on different kernel sources or with a
    different launch shape."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (workload, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    if rec.get("launch_shape", "missing") != launch_shape_entry(workload, precision):
        return None
    return rec.get("bytes_per_launch")


def run_gpu(rho0, info, precision, steps, warmup):
    import torch
    from paper_1905_09554_amd import lbsc, tuning

    nz, ny, nx = rho0.shape
    n = rho0.size
    prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision=precision,
                           G=info["G"], tau=info["tau"], rho_ref=1.0)
    sim = lbsc.Simulation(rho0, prm, device="cuda:0")
    tune = tuning.apply(sim, prm)
    stream = sim.stream
    rv, rl = info["rho_v"], info["rho_l"]

    sim.step(warmup)
    mass0 = sim.diagnostics(rv, rl)["mass"]
    torch.cuda.synchronize()

    # Whole-job timing: steps plus diagnostics every DIAG_EVERY steps.
    t0 = time.perf_counter()
    done = 0
    diag = None
    while done < steps:
        k = min(DIAG_EVERY, steps - done)
        sim.step(k)
        done += k
        if done % DIAG_EVERY == 0 or done == steps:
            diag = sim.diagnostics(rv, rl)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0

    # Step-kernel duration: HIP events on the stream the kernels run on.
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    kreps = max(10, min(steps, 200))
    with torch.cuda.stream(stream):
        ev0.record(stream)
        sim.step(kreps)
        ev1.record(stream)
    ev1.synchronize()
    per_launch_s = ev0.elapsed_time(ev1) / 1e3 / kreps
    sim.close()
    del sim
    torch.cuda.empty_cache()

    alg = BYTES_PER_NODE[precision] * n
    achieved = alg / per_launch_s / 1e9
    traffic = measured_traffic(WORKLOAD, precision)
    return {
        "mlups": n * steps / wall / 1e6,
        "ms_per_step": wall / steps * 1e3,
        "kernel_ms": per_launch_s * 1e3,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "tuning": tune,
        "r_min": diag["r_min"] if diag else None,
        "mass": diag["mass"] if diag else None,
        # |M(end) - M(start)| / M(start) over the timed steps, per 1000 steps.
        "mass_drift_per_1000": abs(diag["mass"] - mass0) / mass0 * 1000.0 / steps,
    }


def run_two_kernel(rho0, info, precision, reps=100):
    """The same step in its two-kernel form (psi written to global memory,
    then read back as a stencil by the colliding kernel): HIP-event time per
    step on the library's stream, the unfused baseline beside the fused
    kernel's kernel_ms."""
    import torch
    from paper_1905_09554_amd import lbsc

    nz, ny, nx = rho0.shape
    prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision=precision,
                           G=info["G"], tau=info["tau"], rho_ref=1.0)
    sim = lbsc.Simulation(rho0, prm, device="cuda:0")
    sim.set_tuning(two_kernel=1)
    stream = sim.stream
    sim.step(10)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        ev0.record(stream)
        sim.step(reps)
        ev1.record(stream)
    ev1.synchronize()
    per_step_s = ev0.elapsed_time(ev1) / 1e3 / reps
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"kernel_ms": round(per_step_s * 1e3, 4),
            "mlups": round(rho0.size / per_step_s / 1e6, 1), "steps": reps,
            "values_per_node": 59, "dtype": precision}


def run_accuracy(rho0, info, steps=1000):
    """FP32 shifted storage against FP64 on the benchmark box: both from the
    same input for `steps` steps, then the largest relative density error
    and the largest velocity (u^b) error over all nodes.  The FP64 step is
    the reference (it matches the oracle to 1e-12, on sampled nodes at this
    size)."""
    import torch
    from paper_1905_09554_amd import lbsc

    nz, ny, nx = rho0.shape
    res = {}
    for prec in ("f64", "f32"):
        prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision=prec,
                               G=info["G"], tau=info["tau"], rho_ref=1.0)
        sim = lbsc.Simulation(rho0, prm, device="cuda:0")
        sim.step(steps)
        rho, u, _ = sim.moments(want_p=False)
        torch.cuda.synchronize()
        sim.close()
        del sim
        res[prec] = (rho, u)
    (r64, u64), (r32, u32) = res["f64"], res["f32"]
    out = {"steps": steps, "reference": "f64 step on the GPU",
           "max_rel_drho": float(((r32 - r64).abs() / r64).max()),
           "max_abs_du": float((u32 - u64).abs().max()),
           "max_abs_u": float(u64.abs().max())}
    del res, r64, u64, r32, u32
    torch.cuda.empty_cache()
    return out


def run_batch(steps, warmup):
    """The 64-ligament dispersion sweep (uneven boxes, 3.9e8 nodes) in one
    batch: MLUPS with one launch per step and with one persistent launch."""
    import torch
    from paper_1905_09554_amd import dispersion

    sweep = dispersion.make_sweep(seed=0)
    total = sum(m["rho0"].size for m in sweep["members"])
    out = {"workload": sweep["workload"], "members": len(sweep["members"]), "nodes": total,
           "dtype": sweep["precision"], "collision": sweep["collision"]}
    b = dispersion.build_batch(sweep)
    for mode in (0, 1):
        b.set_tuning(**dict(b.get_tuning(), persistent=mode))
        b.step(warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        key = "persistent" if mode else "per_step_launch"
        out[key] = {"value": round(total * steps / dt / 1e6, 1), "unit": "MLUPS",
                    "ms_per_step": round(dt / steps * 1e3, 4),
                    "hbm_frac_alg": round(total * steps / dt * BYTES_PER_NODE["f32"] / 1e9
                                          / HBM_PEAK_GBS, 4)}
    out["steps"] = steps
    out["tuning"] = b.get_tuning()
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


def run_adjoint():
    """Adjoint of the float32 MRT step on the 64 x 64 x 256 ligament (32
    Fourier modes), loss r_min after 4000 steps, checkpoints every 200:
    time of the forward (with checkpoint saves) and of the backward (segment
    recomputation plus adjoint steps)."""
    import torch
    import lbm_inputs
    from paper_1905_09554_amd import lbsc

    name = "adjoint_64x64x256_mrt_f32"
    rho0, info = lbm_inputs.workload_density(name)
    nz, ny, nx = rho0.shape
    prm = lbsc.make_params(nx, ny, nz, collision=info["collision"], precision="f32",
                           G=info["G"], tau=info["tau"])
    sim = lbsc.Simulation(rho0, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.adjoint_forward(info["steps"], info["checkpoint_every"])
    rhobar, rmin = sim.rmin_gradient(info["rho_v"], info["rho_l"])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, dG, dtau = sim.adjoint_backward(rhobar)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"workload": name, "steps": info["steps"], "checkpoint_every": info["checkpoint_every"],
            "forward_s": round(t1 - t0, 4), "backward_s": round(t2 - t1, 4),
            "ratio": round((t2 - t1) / (t1 - t0), 3), "r_min": rmin, "dL_dG": dG,
            "dL_dtau": dtau}


def run_small_box(steps=1000):
    """The 32 x 32 x 64 float64 BGK ligament (65 536 nodes, 20 MB of state,
    resident in the last-level cache): the whole run of `steps` steps with
    one launch per step and with one persistent cooperative launch, the time
    of one isolated launch (HIP events around it: kernel plus launch latency,
    which back-to-back launches hide)."""
    import torch
    import lbm_inputs
    from paper_1905_09554_amd import lbsc

    name = "ligament_32x32x64_bgk_f64"
    rho0, info = lbm_inputs.workload_density(name)
    nz, ny, nx = rho0.shape
    n = rho0.size
    prm = lbsc.make_params(nx, ny, nz, collision="bgk", precision="f64", G=info["G"],
                           tau=info["tau"])
    out = {"workload": name, "nodes": n, "steps": steps, "dtype": "f64",
           "note": "cache-resident, not HBM-bound"}
    sim = lbsc.Simulation(rho0, prm)
    sim.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(50)]
    for e0, e1 in evs:
        e0.record(sim.stream)
        sim.step(1)
        e1.record(sim.stream)
        torch.cuda.synchronize()
    kern = sum(e0.elapsed_time(e1) for e0, e1 in evs) / len(evs) / 1e3
    sim.close()
    out["per_step_launch"] = {"value": round(n * steps / wall / 1e6, 1), "unit": "MLUPS",
                              "us_per_step": round(wall / steps * 1e6, 2)}
    out["single_launch_us"] = round(kern * 1e6, 2)
    b = lbsc.Batch([rho0], [prm])
    b.set_tuning(**dict(b.get_tuning(), persistent=1))
    b.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    wall_p = time.perf_counter() - t0
    b.close()
    torch.cuda.empty_cache()
    out["persistent"] = {"value": round(n * steps / wall_p / 1e6, 1), "unit": "MLUPS",
                         "us_per_step": round(wall_p / steps * 1e6, 2)}
    return out


def cpu_model():
    """The host CPU's model name, from /proc/cpuinfo where there is one."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def host_threads():
    """Threads the oracle may use: the CPUs this process may run on, within
    the OpenMP thread limit the environment sets (a shared host may grant
    each GPU only a share of its cores)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def cpu_baseline(rho0, info, nz_sample=16, steps=40):
    """The float64 oracle on the host: the first nz_sample planes of the same
    input as a periodic slab, `steps` steps, reported in MLUPS; also on one
    thread, for 4 steps."""
    import torch
    from oracle import lbm

    torch.set_num_threads(host_threads())
    sample = rho0[:nz_sample].copy()
    p = lbm.Params(G=info["G"], tau=info["tau"], collision=info["collision"])
    f = lbm.init_rest(torch.from_numpy(sample))
    f = lbm.step(f, p)
    t0 = time.perf_counter()
    for _ in range(steps):
        f = lbm.step(f, p)
    dt = time.perf_counter() - t0
    out = {"value": round(sample.size * steps / dt / 1e6, 3), "unit": "MLUPS",
           "cores": torch.get_num_threads(), "kind": "oracle", "cpu_model": cpu_model(),
           "host_cpus": os.cpu_count(), "sample": "%dx%dx%d periodic slab (first %d planes of "
           "the benchmark input), %s float64, %d steps, %.1f s" % (
               sample.shape[2], sample.shape[1], nz_sample, nz_sample, info["collision"], steps,
               dt)}
    nthreads = torch.get_num_threads()
    torch.set_num_threads(1)
    f = lbm.step(lbm.init_rest(torch.from_numpy(sample)), p)
    t0 = time.perf_counter()
    for _ in range(4):
        f = lbm.step(f, p)
    dt1 = time.perf_counter() - t0
    torch.set_num_threads(nthreads)
    out["one_thread"] = {"value": round(sample.size * 4 / dt1 / 1e6, 3), "unit": "MLUPS",
                         "steps": 4, "seconds": round(dt1, 2)}
    # A 20-step window of the 128 x 128 x 512 ligament (first 64 planes), BGK.
    import lbm_inputs
    rho2, info2 = lbm_inputs.workload_density("ligament_128x128x512")
    s2 = rho2[:64].copy()
    p2 = lbm.Params(G=info2["G"], tau=info2["tau"], collision="bgk")
    f = lbm.step(lbm.init_rest(torch.from_numpy(s2)), p2)
    t0 = time.perf_counter()
    for _ in range(20):
        f = lbm.step(f, p2)
    dt2 = time.perf_counter() - t0
    out["window_128x128x512"] = {
        "value": round(s2.size * 20 / dt2 / 1e6, 3), "unit": "MLUPS",
        "sample": "128x128x64 periodic slab (first 64 planes), bgk float64, 20 steps, %.1f s" % dt2}
    # The whole 32 x 32 x 64 BGK box (the small-box figure's run): 1000 steps
    # on up to 16 threads, 50 steps on one.
    rho1, info1 = lbm_inputs.workload_density("ligament_32x32x64_bgk_f64")
    p1 = lbm.Params(G=info1["G"], tau=info1["tau"], collision="bgk")
    nthreads = torch.get_num_threads()
    res = {}
    for threads, k in ((nthreads, 1000), (1, 50)):
        torch.set_num_threads(threads)
        f = lbm.step(lbm.init_rest(torch.from_numpy(rho1)), p1)
        t0 = time.perf_counter()
        for _ in range(k):
            f = lbm.step(f, p1)
        dt1 = time.perf_counter() - t0
        res["threads_%d" % threads] = {"value": round(rho1.size * k / dt1 / 1e6, 3),
                                       "unit": "MLUPS", "steps": k, "seconds": round(dt1, 2)}
    torch.set_num_threads(nthreads)
    out["small_box_32x32x64"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # 5000 timed steps of the 256 x 256 x 1024 box by default (about 10 s of
    # FP32 steps); the FP64 figure takes half as many, the batch at most 100.
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 figure")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched sweep figure")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost figure")
    ap.add_argument("--no-small", action="store_true", help="skip the 32x32x64 small-box figure")
    ap.add_argument("--no-two-kernel", action="store_true",
                    help="skip the unfused two-kernel baseline figure")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the FP32-against-FP64 error after 1000 steps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the step is single-GPU; see the design notes "
              "for how it would shard); got --gpus %d" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import lbm_inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)

    rho0, info = lbm_inputs.workload_density(WORKLOAD)
    print("workload %s: %d nodes" % (WORKLOAD, rho0.size), file=sys.stderr, flush=True)
    f32 = run_gpu(rho0, info, "f32", args.steps, args.warmup)
    print("f32 done: %.0f MLUPS" % f32["mlups"], file=sys.stderr, flush=True)
    f64 = None
    if not args.no_fp64:
        f64 = run_gpu(rho0, info, "f64", max(50, args.steps // 2), args.warmup)
        print("f64 done: %.0f MLUPS" % f64["mlups"], file=sys.stderr, flush=True)
    two = None
    if not args.no_two_kernel:
        two = run_two_kernel(rho0, info, "f32")
        two["fused_kernel_ms"] = round(f32["kernel_ms"], 4)
        two["fused_speedup"] = round(two["kernel_ms"] / f32["kernel_ms"], 3)
        print("two-kernel done: %.3f ms per step" % two["kernel_ms"], file=sys.stderr, flush=True)
    acc = None
    if not args.no_accuracy:
        acc = run_accuracy(rho0, info)
        print("accuracy done: max rel drho %.2e" % acc["max_rel_drho"], file=sys.stderr, flush=True)
    batch = None
    if not args.no_batch:
        batch = run_batch(min(100, max(20, args.steps // 5)), 5)
        print("batch done: %.0f MLUPS" % batch["persistent"]["value"], file=sys.stderr, flush=True)
    adj = None if args.no_adjoint else run_adjoint()
    if adj:
        print("adjoint done: ratio %.2f" % adj["ratio"], file=sys.stderr, flush=True)
    small = None
    if not args.no_small:
        small = run_small_box()
        print("small box done: %.0f MLUPS per launch, %.0f persistent"
              % (small["per_step_launch"]["value"], small["persistent"]["value"]),
              file=sys.stderr, flush=True)
    cpu = None if args.no_cpu_baseline else cpu_baseline(rho0, info)

    nz, ny, nx = rho0.shape
    line = {
        "metric": METRIC,
        "value": round(f32["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(f32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "nx": nx, "ny": ny, "nz": nz, "nodes": rho0.size,
                   "collision": info["collision"], "forcing": "guo", "G": info["G"],
                   "tau": info["tau"], "storage": "f32 shifted, rho_ref 1.0",
                   "R": info["R"], "kR_eff": round(info["kR_eff"], 4),
                   "diagnostics_every": DIAG_EVERY, "tuning": f32["tuning"]},
        "roofline": f32["roofline"],
        "copy_ceiling": {"gbs": COPY_CEILING_GBS,
                         "frac": round(f32["roofline"]["achieved"] / COPY_CEILING_GBS, 4)},
        "pull_pattern_ceiling": {"gbs": PULL_PATTERN_GBS,
                                 "frac": round(f32["roofline"]["achieved"] / PULL_PATTERN_GBS, 4)},
        "kernel_ms": round(f32["kernel_ms"], 4),
        # Step kernel alone (HIP events, no diagnostics), and the measured HBM
        # bytes per node-step from the counter runs.
        "value_kernel_only": round(rho0.size / (f32["kernel_ms"] * 1e-3) / 1e6, 1),
        "traffic_bytes_per_node": (round(f32["roofline"]["traffic"] / rho0.size, 2)
                                   if f32["roofline"]["traffic"] else None),
        "hbm_frac_alg": round(f32["mlups"] * 1e6 * BYTES_PER_NODE["f32"] / 1e9 / HBM_PEAK_GBS, 4),
        "cpu_baseline": cpu,
        "mass_drift_per_1000": f32["mass_drift_per_1000"],
    }
    if f64:
        line["fp64"] = {"value": round(f64["mlups"], 1), "unit": "MLUPS", "dtype": "f64",
                        "ms_per_step": round(f64["ms_per_step"], 4),
                        "kernel_ms": round(f64["kernel_ms"], 4), "roofline": f64["roofline"],
                        "value_kernel_only": round(rho0.size / (f64["kernel_ms"] * 1e-3) / 1e6, 1),
                        "mass_drift_per_1000": f64["mass_drift_per_1000"],
                        "tuning": f64["tuning"]}
    if acc:
        line["fp32_vs_fp64"] = acc
    if two:
        line["two_kernel_baseline"] = two
    if batch:
        line["batched"] = batch
    if small:
        line["small_box"] = small
    if adj:
        line["adjoint_forward_cost_ratio"] = adj["ratio"]
        line["adjoint"] = adj
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
