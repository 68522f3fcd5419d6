"""Dispersion-relation sweeps: many ligaments of uneven radius and wavenumber
stepped together in one batch, with the linear growth rate of each fitted from
its radius profile.

The paper follows the growth of the perturbation in the linear stage
(Sec. 4, Fig. 4a) and compares break-up times with linear stability
analysis (Fig. 3).  Here every member is a periodic box 4R x 4R x L holding
exactly one wavelength L = round(2 pi R / kR) of the perturbation
r(z) = R (1 + A cos(2 pi z / L)).  The mode amplitude
a(t) = (2 / L) sum_z r(z, t) cos(2 pi z / L) (with r(z) the equivalent
radius of the interface diagnostics) grows as exp(omega t) in the linear
stage; omega is fitted by least squares on ln a(t) over the window
2 a(0) <= a <= 0.2 R after a 200-step relaxation of the initial tanh profile.
"""
import math

import numpy as np

import lbm_inputs

from . import lbsc, tuning

WORKLOAD = "batch64_bgk_f32"


def make_sweep(seed=0, n=None, workload=WORKLOAD):
    """Members of the sweep: geometry, physics and initial density."""
    w = dict(lbm_inputs.WORKLOADS[workload])
    if n is not None:
        w["n"] = n
    rv, rl = lbm_inputs.coexistence(w["G"])
    members = []
    for spec in lbm_inputs.batch_ligaments(n=w["n"], seed=seed):
        rho0 = lbm_inputs.ligament_density(spec["nx"], spec["ny"], spec["nz"], spec["R"],
                                           w["amp"], 1, rv, rl)
        members.append(dict(spec, rho0=rho0, G=w["G"], tau=w["tau"], amp=w["amp"]))
    return {"workload": workload, "seed": seed, "rho_v": rv, "rho_l": rl, "members": members,
            "collision": w["collision"], "precision": w["precision"]}


def member_params(sweep):
    return [lbsc.make_params(m["nx"], m["ny"], m["nz"], collision=sweep["collision"],
                             precision=sweep["precision"], G=m["G"], tau=m["tau"])
            for m in sweep["members"]]


def build_batch(sweep, persistent=None):
    """lbsc.Batch of the sweep with the tuned launch shape."""
    params = member_params(sweep)
    b = lbsc.Batch([m["rho0"] for m in sweep["members"]], params)
    t = tuning.lookup_batch(sweep["workload"], sweep["precision"]) or {}
    if persistent is not None:
        t["persistent"] = persistent
    if t:
        b.set_tuning(**t)
    return b


def mode_amplitude(r_of_z):
    nz = len(r_of_z)
    z = np.arange(nz)
    return 2.0 / nz * float(np.sum(r_of_z * np.cos(2.0 * math.pi * z / nz)))


def fit_growth(t, a, R, transient=200, lo_factor=2.0, hi_frac=0.2):
    """Least-squares growth rate of ln a(t) in the linear window; None if the
    window holds fewer than three samples (decaying or saturated modes give
    the rate over all samples after the transient instead)."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    keep = t >= transient
    t, a = t[keep], a[keep]
    if len(t) < 3:
        return None
    a0 = abs(a[0])
    win = (np.abs(a) >= lo_factor * a0) & (np.abs(a) <= hi_frac * R) & (a > 0)
    if win.sum() < 3:
        win = a > 0
    if win.sum() < 3:
        return None
    slope, _ = np.polyfit(t[win], np.log(a[win]), 1)
    return float(slope)


def run_sweep(batch, sweep, steps=3000, every=50):
    """Steps the batch, samples every member's radius profile every `every`
    steps, returns per-member growth rates (1 / step) and the time series."""
    rv, rl = sweep["rho_v"], sweep["rho_l"]
    n = len(sweep["members"])
    times, amps = [], [[] for _ in range(n)]

    def sample():
        times.append(batch.step_count)
        for i in range(n):
            d = batch.diagnostics(i, rv, rl)
            amps[i].append(mode_amplitude(d["r_of_z"]))

    sample()
    done = 0
    while done < steps:
        k = min(every, steps - done)
        batch.step(k)
        done += k
        sample()
    rates = [fit_growth(times, amps[i], m["R"]) for i, m in enumerate(sweep["members"])]
    return {"t": times, "amplitude": amps, "rate": rates,
            "kR": [m["kR_eff"] for m in sweep["members"]],
            "R": [m["R"] for m in sweep["members"]]}
