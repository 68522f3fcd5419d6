"""HBM traffic of the step kernel from two rocprofv3 counter runs.

    python -m paper_1905_09554_amd.traffic --fetch DIR --write DIR \
        --precision f32 [--workload NAME]

DIR are the output folders of
    rocprofv3 --pmc FETCH_SIZE -d DIR -- python -m paper_1905_09554_amd.prof_driver
    rocprofv3 --pmc WRITE_SIZE -d DIR -- python -m paper_1905_09554_amd.prof_driver
Both counters are in KiB per dispatch.  Each is scaled by what it reads for
the driver's plain copy of a known size (1 GiB read, 1 GiB written), and the
per-launch bytes of the step kernel are written to
profiles/traffic_<workload>_<precision>.json together with a hash of the
kernel sources (lbsc_device.hip, lbsc_api.hip, lbsc_internal.h) and the autotuner's launch shape for the box (the benchmark
ignores the file once either changes).
"""
import argparse
import csv
import glob
import json
import os
import statistics

from .prof_driver import COPY_BYTES, WORKLOAD

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rows(folder, counter):
    files = glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError("no counter_collection.csv under %s" % folder)
    out = []
    for path in files:
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") == counter:
                    out.append((row.get("Kernel_Name", ""), float(row["Counter_Value"])))
    return out


def _per_kernel(rows):
    step = [v for name, v in rows if "k_step" in name]
    copy = [v for name, v in rows if "copyBuffer" in name or "elementwise" in name]
    if not step or not copy:
        raise RuntimeError("missing step or copy dispatches in the counter file")
    return statistics.mean(step), copy[-1], len(step)


def reduce_counters(fetch_rows, write_rows, precision, nodes):
    """Per-launch bytes of the step kernel from (kernel name, KiB) rows of the
    two counters, each scaled by its reading for the plain copy."""
    f_step, f_copy, nf = _per_kernel(fetch_rows)
    w_step, w_copy, nw = _per_kernel(write_rows)
    kib = COPY_BYTES / 1024.0
    f_scale, w_scale = kib / f_copy, kib / w_copy
    fetch_b = f_step * f_scale * 1024.0
    write_b = w_step * w_scale * 1024.0
    elem = 4 if precision == "f32" else 8
    alg = 19 * elem * nodes
    return {
        "fetch_kib_raw": f_step, "write_kib_raw": w_step, "dispatches": [nf, nw],
        "copy_fetch_kib": f_copy, "copy_write_kib": w_copy,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "fetch_bytes_per_launch": fetch_b, "write_bytes_per_launch": write_b,
        "bytes_per_launch": fetch_b + write_b,
        "algorithmic_bytes_per_launch": 2 * alg,
        "fetch_over_algorithmic": fetch_b / alg, "write_over_algorithmic": write_b / alg,
    }


def by_kernel(fetch_rows, write_rows, nodes):
    """Mean scaled bytes per dispatch of every kernel in the two counter
    runs (the last copy dispatch calibrates each counter), and per node."""
    _, f_copy, _ = _per_kernel([("k_step", 0.0)] + fetch_rows)
    _, w_copy, _ = _per_kernel([("k_step", 0.0)] + write_rows)
    kib = COPY_BYTES / 1024.0
    out = {}
    for rows, copy, key in ((fetch_rows, f_copy, "fetch"), (write_rows, w_copy, "write")):
        groups = {}
        for name, v in rows:
            short = name.replace("lbsc::(anonymous namespace)::", "").replace("void ", "")
            short = short.split("(")[0]
            groups.setdefault(short, []).append(v)
        for short, vals in groups.items():
            b = statistics.mean(vals) * kib / copy * 1024.0
            e = out.setdefault(short, {"dispatches": len(vals)})
            e[key + "_bytes"] = b
            e[key + "_bytes_per_node"] = b / nodes
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--precision", choices=["f32", "f64"])
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--nodes", type=int, default=256 * 256 * 1024)
    ap.add_argument("--by-kernel", action="store_true",
                    help="print the scaled bytes of every kernel (per dispatch and per node); "
                         "writes no file")
    args = ap.parse_args()

    if args.by_kernel:
        rec = by_kernel(_rows(args.fetch, "FETCH_SIZE"), _rows(args.write, "WRITE_SIZE"), args.nodes)
        print(json.dumps(rec, indent=1))
        return
    if args.precision is None:
        ap.error("--precision is required unless --by-kernel is given")

    import sys
    sys.path.insert(0, ROOT)
    from bench import kernel_source_hash, launch_shape_entry

    rec = {
        "workload": args.workload, "precision": args.precision, "nodes": args.nodes,
        "source_hash": kernel_source_hash(),
        "launch_shape": launch_shape_entry(args.workload, args.precision),
    }
    rec.update(reduce_counters(_rows(args.fetch, "FETCH_SIZE"), _rows(args.write, "WRITE_SIZE"),
                               args.precision, args.nodes))
    out = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (args.workload, args.precision))
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main()
