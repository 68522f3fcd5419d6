"""Launch shapes chosen by the autotuner (autotune.py), keyed by box shape,
precision and collision.  The benchmark and the full-size tests apply the
same choice, so what is timed is what is checked."""
import json
import os

_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_cache.json")


def key(params):
    coll = {0: "bgk", 1: "mrt"}[params.collision]
    prec = {0: "f64", 1: "f32"}[params.precision]
    return "%dx%dx%d/%s/%s" % (params.nx, params.ny, params.nz, prec, coll)


def load():
    if not os.path.exists(_CACHE):
        return {}
    with open(_CACHE) as fh:
        return json.load(fh)


def lookup(params):
    """Tuning dict for these parameters, or None for the library default."""
    entry = load().get(key(params))
    return dict(entry["tuning"]) if entry else None


def apply(sim, params):
    t = lookup(params)
    if t:
        sim.set_tuning(**t)
    return sim.get_tuning()


def batch_key(workload, precision):
    return "batch/%s/%s" % (workload, precision)


def lookup_batch(workload, precision):
    entry = load().get(batch_key(workload, precision))
    return dict(entry["tuning"]) if entry else None
