"""Launch-shape search for the fused step, written to tuning_cache.json.

    python -m paper_1905_09554_amd.autotune [--workload NAME | --box NX,NY,NZ]
                                            [--precision f32,f64] [--collision mrt]
                                            [--steps K] [--out FILE]
    python -m paper_1905_09554_amd.autotune --batch [--steps K] [--out FILE]

For one box (a workload of lbm_inputs.WORKLOADS), times the step over a grid
of launch shapes: work-group size, nodes per thread, tile width (whole rows
or multiples of 64 columns), z chunk and the XCD-aware tile order.  Each
candidate runs K steps after a short warm-up, timed with HIP events on the
library's stream.  The fastest shape is stored under the key of
tuning.key(params) together with its MLUPS and the library default's, so
the benchmark and the full-size tests use what was measured fastest.  With
--batch it tunes the dispersion batch instead (work-group size, z chunk,
tile order, and the persistent form), stored under tuning.batch_key.  The
state of the box is the workload's own input; timing does not depend on it
beyond the first steps.
"""
import argparse
import itertools
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def candidates(nx, precision, nodes=None):
    """Launch shapes worth timing for a box of row length nx (and, when
    given, `nodes` in all: boxes under 16 M nodes also try the short
    z-chunks that give them enough work-groups)."""
    # Multiples of 64 columns, whole rows, and the even splits of a row into
    # 2-6 tiles whose width is a multiple of 16 nodes (no ragged last tile,
    # and tile edges on 64-byte lines in float32).
    widths = sorted({nx} | {w for w in (64, 128, 192, 256, 384, 512) if w < nx}
                    | {nx // k for k in range(2, 7)
                       if nx % k == 0 and (nx // k) % 16 == 0 and nx // k >= 64})
    out = []
    for threads, npt in itertools.product((256, 512, 1024), (1, 2)):
        if precision == "f64" and (threads == 1024 or npt == 2):
            continue  # 204 VGPRs: one group per CU at 512 threads already
        cap = threads * npt
        for bx in widths:
            if bx > cap or (bx < nx and 2 * bx > cap):
                continue  # split rows only as tiles of two or more rows
            chunks = (16, 32, 64, 128, 256)
            if nodes is not None and nodes < (1 << 24):
                chunks = (1, 2, 4, 8) + chunks
            for zc in chunks:
                out.append(dict(threads=threads, nodes_per_thread=npt, block_x=bx, z_chunk=zc))
    return out


def time_shape(sim, steps):
    import torch
    sim.step(3)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def box_density(nx, ny, nz):
    """A ligament of radius min(nx, ny) / 4 along z in an nx x ny x nz box
    (G = -5 coexisting densities, one wavelength, amplitude 0.05), for
    tuning boxes that are not one of the named workloads."""
    import lbm_inputs
    rv, rl = lbm_inputs.coexistence(-5.0)
    R = min(nx, ny) / 4.0
    rho0 = lbm_inputs.ligament_density(nx, ny, nz, R, 0.05, 1, rv, rl)
    return rho0, {"G": -5.0, "tau": 1.0}


def tune(workload, precision, collision, steps=20, progress=True, out=None, box=None):
    import torch
    import lbm_inputs
    from . import lbsc, tuning

    if box is not None:
        rho0, info = box_density(*box)
        workload = "box_%dx%dx%d" % box
    else:
        rho0, info = lbm_inputs.workload_density(workload)
    nz, ny, nx = rho0.shape
    n = rho0.size
    prm = lbsc.make_params(nx, ny, nz, collision=collision, precision=precision, G=info["G"],
                           tau=info["tau"], rho_ref=1.0)
    sim = lbsc.Simulation(rho0, prm)
    default_shape = sim.get_tuning()
    tried = []
    for c in candidates(nx, precision, nodes=n):
        for remap in (1, 0):
            try:
                sim.set_tuning(xcd_remap=remap, **c)
            except lbsc.LbscError:
                continue
            t = time_shape(sim, steps)
            shape = sim.get_tuning()
            tried.append((t, shape))
            if progress:
                print("  %s %s %s: %s %.0f MLUPS" % (workload, precision, collision, shape,
                                                     n / t / 1e6), flush=True)
    # Second pass, five times longer, over the four fastest and the default:
    # one short timing per shape favours whichever caught the least noise.
    tried.sort(key=lambda x: x[0])
    finalists = [default_shape] + [shape for _, shape in tried[:4]]
    timed = []
    for shape in finalists:
        sim.set_tuning(**shape)
        timed.append((time_shape(sim, 5 * steps), shape))
    default = timed[0][0]
    best = min(timed, key=lambda x: x[0])
    sim.close()
    del sim
    torch.cuda.empty_cache()
    entry = {"tuning": best[1], "mlups": n / best[0] / 1e6,
             "default": {"tuning": default_shape, "mlups": n / default / 1e6},
             "steps_timed": steps, "candidates": len(tried),
             "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    path = out or tuning._CACHE
    cache = {}
    if os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    cache[tuning.key(prm)] = entry
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return entry


def batch_candidates():
    """Launch shapes worth timing for a batch of small boxes: work-group
    size, z chunk and tile order (tiles are whole rows of each member, the
    default for boxes this narrow)."""
    return [dict(threads=threads, z_chunk=zc, xcd_remap=remap, persistent=0)
            for threads in (256, 512, 1024) for zc in (2, 4, 8, 16, 32, 64)
            for remap in (0, 1)]


def tune_batch(workload=None, steps=5, progress=True, out=None):
    """Times the dispersion batch (every member stepped together) over
    batch_candidates(), then re-times the four fastest, the library default
    and the fastest in the persistent form (one cooperative launch for all
    steps) five times longer, and stores the best under
    tuning.batch_key(workload, precision)."""
    import torch
    from . import dispersion, lbsc, tuning

    workload = workload or dispersion.WORKLOAD
    sweep = dispersion.make_sweep(seed=0, workload=workload)
    params = dispersion.member_params(sweep)
    b = lbsc.Batch([m["rho0"] for m in sweep["members"]], params)
    n = sum(m["nx"] * m["ny"] * m["nz"] for m in sweep["members"])
    default_shape = b.get_tuning()
    tried = []
    for c in batch_candidates():
        try:
            b.set_tuning(**c)
        except lbsc.LbscError:
            continue
        t = time_shape(b, steps)
        shape = b.get_tuning()
        tried.append((t, shape))
        if progress:
            print("  %s: %s %.0f MLUPS" % (workload, shape, n / t / 1e6), flush=True)
    if not tried:
        raise RuntimeError("the library refused every batch launch shape")
    tried.sort(key=lambda x: x[0])
    finalists = [default_shape] + [shape for _, shape in tried[:4]]
    finalists.append(dict(tried[0][1], persistent=1))
    timed = []
    for shape in finalists:
        b.set_tuning(**shape)
        timed.append((time_shape(b, 5 * steps), b.get_tuning()))
        if progress:
            print("  final %s %.0f MLUPS" % (timed[-1][1], n / timed[-1][0] / 1e6), flush=True)
    default = timed[0][0]
    best = min(timed, key=lambda x: x[0])
    b.close()
    del b
    torch.cuda.empty_cache()
    entry = {"tuning": best[1], "mlups": n / best[0] / 1e6,
             "default": {"tuning": default_shape, "mlups": n / default / 1e6},
             "steps_timed": steps, "candidates": len(tried),
             "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    path = out or tuning._CACHE
    cache = {}
    if os.path.exists(path):
        with open(path) as fh:
            cache = json.load(fh)
    cache[tuning.batch_key(workload, sweep["precision"])] = entry
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    return entry


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="ligament_256x256x1024_mrt_f32")
    ap.add_argument("--precision", default="f32,f64")
    ap.add_argument("--collision", default="mrt")
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--out", default=None,
                    help="cache file to update (default: the package's tuning_cache.json)")
    ap.add_argument("--box", default=None,
                    help="nx,ny,nz of a box to tune instead of a named workload")
    ap.add_argument("--batch", action="store_true",
                    help="tune the dispersion batch (all members in one launch) instead")
    args = ap.parse_args()
    if args.batch:
        e = tune_batch(steps=args.steps, out=args.out)
        print(json.dumps({"workload": "batch", "best": e["tuning"], "mlups": round(e["mlups"], 1),
                          "default_mlups": round(e["default"]["mlups"], 1)}), flush=True)
        return
    box = tuple(int(v) for v in args.box.split(",")) if args.box else None
    for prec in args.precision.split(","):
        e = tune(args.workload, prec, args.collision, args.steps, out=args.out, box=box)
        name = "box_%dx%dx%d" % box if box else args.workload
        print(json.dumps({"workload": name, "precision": prec,
                          "collision": args.collision, "best": e["tuning"],
                          "mlups": round(e["mlups"], 1),
                          "default_mlups": round(e["default"]["mlups"], 1)}), flush=True)


if __name__ == "__main__":
    main()
