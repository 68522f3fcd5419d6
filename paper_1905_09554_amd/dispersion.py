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
stage.  A mode released from rest is the sum of the growing root and a
decaying one of the dispersion relation, so ln a(t) reaches its asymptotic
slope only after a few capillary times; omega is therefore fitted by least
squares on ln a(t) over t >= 3 t_cap (t_cap = sqrt(rho_l R^3 / sigma),
Eq. Oh_Tcap) and a <= 0.15 R, before nonlinear pinching sets in.
"""
import math

import numpy as np

import lbm_inputs

from . import lbsc, tuning

WORKLOAD = "batch64_bgk_f32"


def make_sweep(seed=0, n=None, workload=WORKLOAD, select=None):
    """Members of the sweep: geometry, physics and initial density.

    `select(spec) -> bool` keeps a subset of the drawn ligaments (the draw
    itself, and so every member's geometry, does not depend on it)."""
    w = dict(lbm_inputs.WORKLOADS[workload])
    if n is not None:
        w["n"] = n
    rv, rl = lbm_inputs.coexistence(w["G"])
    members = []
    for spec in lbm_inputs.batch_ligaments(n=w["n"], seed=seed):
        if select is not None and not select(spec):
            continue
        rho0 = lbm_inputs.ligament_density(spec["nx"], spec["ny"], spec["nz"], spec["R"],
                                           w["amp"], 1, rv, rl)
        members.append(dict(spec, rho0=rho0, G=w["G"], tau=w["tau"], amp=w["amp"]))
    return {"workload": workload, "seed": seed, "rho_v": rv, "rho_l": rl,
            "sigma": lbm_inputs.surface_tension(w["G"]), "members": members,
            "collision": w["collision"], "precision": w["precision"]}


def capillary_time(sweep, m):
    """t_cap = sqrt(rho_l R^3 / sigma) of member m (Eq. Oh_Tcap)."""
    return math.sqrt(sweep["rho_l"] * m["R"] ** 3 / sweep["sigma"])


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


def fit_growth(t, a, R, t_start, hi_frac=0.15, min_points=4):
    """Least-squares slope of ln a(t) over t >= t_start, 0 < a <= hi_frac R;
    None if that window holds fewer than min_points samples."""
    t = np.asarray(t, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    win = (t >= t_start) & (a > 0) & (a <= hi_frac * R)
    if win.sum() < min_points:
        return None
    slope, _ = np.polyfit(t[win], np.log(a[win]), 1)
    return float(slope)


def run_sweep(batch, sweep, steps=3000, every=50, transient_tcap=3.0):
    """Steps the batch, samples every member's radius profile every `every`
    steps, returns per-member growth rates (1 / step and omega t_cap; None
    where the run ends before the fit window holds enough samples) and the
    time series."""
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
    tcap = [capillary_time(sweep, m) for m in sweep["members"]]
    rates = [fit_growth(times, amps[i], m["R"], transient_tcap * tcap[i])
             for i, m in enumerate(sweep["members"])]
    return {"t": times, "amplitude": amps, "rate": rates, "t_cap": tcap,
            "rate_tcap": [None if r is None else r * tc for r, tc in zip(rates, tcap)],
            "kR": [m["kR_eff"] for m in sweep["members"]],
            "R": [m["R"] for m in sweep["members"]]}
