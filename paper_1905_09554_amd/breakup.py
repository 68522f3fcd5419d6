"""Break-up time of a perturbed ligament (Sec. 4, Fig. 2b and Fig. 3 of the
paper): run until the neck pinches off and report T_break / t_cap.

Operators as in the paper (Sec. 2): "srt" is BGK with the velocity-shift
forcing of Eq. vel_shift; "mrt" is MRT with Guo-like forcing and the paper's
rate set (bulk and shear rates 1/tau, every other rate 1).

Break-up criterion (the paper does not state one): the first sampled step at
which some z-slice holds no node denser than the mid density
(rho_l + rho_v) / 2, i.e. the liquid column is cut.  Sampling every `every`
steps bounds the resolution of T_break to every / t_cap.

`Recorder` samples the observables of Sec. 4 along the run (perturbation
growth, silhouettes, minimum radius, velocity magnitude maps).
"""
import numpy as np
import torch

import lbm_inputs

from . import lbsc, tuning


def params_for(info, operator, precision="f32"):
    if operator == "srt":
        return lbsc.make_params(info["nx"], info["ny"], info["nz"], collision="bgk",
                                forcing="shift", precision=precision, G=info["G"],
                                tau=info["tau"])
    return lbsc.make_params(info["nx"], info["ny"], info["nz"], collision="mrt", forcing="guo",
                            precision=precision, G=info["G"], tau=info["tau"],
                            s_bulk=1.0 / info["tau"], s_ghost=1.0)


def neck_cut(sim, rho_mid):
    """True if some z-slice has no node above rho_mid."""
    return bool((slice_max(sim) <= rho_mid).any())


def slice_max(sim):
    """Densest node of every z-slice, float64 numpy [nz]."""
    rho, _, _ = sim.moments(want_u=False, want_p=False)
    return rho.amax(dim=(1, 2)).cpu().numpy()


def drops(smax, rho_mid, r_of_z=None):
    """Liquid bodies along the periodic axis: maximal runs of slices whose
    densest node exceeds rho_mid.  Returns a list of (first slice, length,
    volume) with volume = sum of pi r(z)^2 over the run when r(z) is given."""
    wet = np.asarray(smax) > rho_mid
    nz = len(wet)
    if wet.all():
        return [(0, nz, float(np.pi * np.sum(np.asarray(r_of_z) ** 2)) if r_of_z is not None
                 else None)]
    if not wet.any():
        return []
    start = int(np.argmin(wet))  # a dry slice: runs never wrap across it
    out = []
    z = 0
    while z < nz:
        k = (start + z) % nz
        if wet[k]:
            n = 0
            while z + n < nz and wet[(start + z + n) % nz]:
                n += 1
            idx = [(k + i) % nz for i in range(n)]
            vol = float(np.pi * np.sum(np.asarray(r_of_z)[idx] ** 2)) if r_of_z is not None else None
            out.append((k, n, vol))
            z += n
        else:
            z += 1
    return out


class Recorder:
    """Observables of Sec. 4 sampled along a run (every `every` steps):

    * r(z, t), the equivalent radius of each slice (interface diagnostics);
      from it the minimum radius h_min(t) / R0 (Fig. 5) and the perturbation
      at the first neck z = nz / (2 m) of the m wavelengths in the box
      (info["wavelengths"], default 2: L/4) and at the crest z = 0, each
      normalised by its initial value (Fig. 4a: our cos profile puts the neck
      at L/4 where the paper's sin profile has it at 3 L/8);
    * silhouettes r(z) at the requested t* = t / t_cap (Fig. 4b: 7, 8, 9);
    * v* = |u^b| / (R0 / t_cap) on the plane through the axis (y = ny/2) at
      the requested t* (Fig. 6), float32 [nz, nx].
    """

    def __init__(self, info, silhouette_tstar=(7.0, 8.0, 9.0), velocity_tstar=(7.0, 8.0, 9.0)):
        self.info = info
        self.t, self.r = [], []
        self.sil_t = sorted(silhouette_tstar)
        self.vel_t = sorted(velocity_tstar)
        self.silhouettes, self.velocity = {}, {}

    def sample(self, sim, steps, last=False):
        info = self.info
        tstar = steps / info["t_cap"]
        d = sim.diagnostics(info["rho_v"], info["rho_l"])
        self.t.append(steps)
        self.r.append(np.asarray(d["r_of_z"], dtype=np.float64))
        for ts in self.sil_t:
            if ts not in self.silhouettes and tstar >= ts:
                self.silhouettes[ts] = (steps, self.r[-1].copy())
        for ts in self.vel_t:
            if ts not in self.velocity and (tstar >= ts or last):
                _, u, _ = sim.moments(want_u=True, want_p=False)
                mid = info["ny"] // 2
                vmag = torch.sqrt((u[:, :, mid, :] ** 2).sum(0))
                v = (vmag / (info["R0"] / info["t_cap"])).float().cpu().numpy()
                self.velocity[ts] = (steps, v)
                break

    def result(self):
        info = self.info
        r = np.stack(self.r)
        t = np.asarray(self.t, dtype=np.float64)
        nz = r.shape[1]
        rbar = r[0].mean()
        neck, crest = nz // (2 * info.get("wavelengths", 2)), 0
        return {
            "t_star": t / info["t_cap"],
            "h_min_over_R0": r.min(axis=1) / info["R0"],
            "neck_perturbation": (rbar - r[:, neck]) / (rbar - r[0, neck]),
            "crest_perturbation": (r[:, crest] - rbar) / (r[0, crest] - rbar),
            "r_of_z": r,
            "silhouettes": {k: v for k, v in self.silhouettes.items()},
            "velocity": {k: v for k, v in self.velocity.items()},
        }


def break_time(R0, operator, eps=0.1, every=25, max_tcap=16.0, precision="f32", progress=False,
               record=None, after_tcap=0.0, wavelengths=2):
    """(T_break / t_cap, steps, info) for the paper's run at radius R0.
    With record = a Recorder (or True for the default one), info["record"]
    holds the observables it sampled.  With after_tcap > 0 the run goes on
    for that many capillary times after the break-up and info["drops"] holds
    the liquid bodies along the axis at every sample (see `satellites`); a
    state that turns non-finite ends the continuation and is reported as
    info["diverged_after_tcap"].  wavelengths = 1 runs half the paper's
    box along the axis (one wavelength of the perturbation), which holds the
    same periodic solution at half the cost."""
    rho0, info = lbm_inputs.paper_ligament(R0, operator, eps, wavelengths)
    return run_to_breakup(rho0, info, operator, every=every, max_tcap=max_tcap,
                          precision=precision, progress=progress, record=record,
                          after_tcap=after_tcap)


def run_to_breakup(rho0, info, operator, every=25, max_tcap=16.0, precision="f32",
                   progress=False, record=None, after_tcap=0.0):
    """The run of break_time from any initial density: info holds the box
    (nx, ny, nz), G, tau, rho_l, rho_v, t_cap and R0 (and eps for the
    progress lines).  Same return values."""
    R0, eps = info["R0"], info.get("eps", float("nan"))
    prm = params_for(info, operator, precision)
    sim = lbsc.Simulation(rho0, prm)
    tuning.apply(sim, prm)  # a measured launch shape for this box, if one is cached
    rec = Recorder(info) if record is True else (record or None)
    rho_mid = 0.5 * (info["rho_l"] + info["rho_v"])
    max_steps = int(max_tcap * info["t_cap"])
    steps = 0
    broke = False
    if rec is not None:
        rec.sample(sim, 0)
    while steps < max_steps:
        sim.step(every)
        steps += every
        cut = neck_cut(sim, rho_mid)
        if rec is not None:
            rec.sample(sim, steps, last=cut)
        if cut:
            broke = True
            break
        if progress and steps % 2000 == 0:
            print("  R0=%d %s eps=%.4f: %d steps (%.2f t_cap)" % (R0, operator, eps, steps,
                                                                 steps / info["t_cap"]),
                  flush=True)
    history = []
    diverged = None
    if broke and after_tcap > 0:
        end = steps + int(after_tcap * info["t_cap"])
        t = steps
        while t < end:
            sim.step(every)
            t += every
            try:
                d = sim.diagnostics(info["rho_v"], info["rho_l"])
            except lbsc.LbscError as e:
                if e.code != lbsc.LBSC_ENONFINITE:
                    raise
                diverged = t  # the state holds NaN or Inf: stop here
                break
            history.append((t, drops(slice_max(sim), rho_mid, d["r_of_z"])))
    torch.cuda.synchronize()
    sim.close()
    info = dict(info, steps=steps, broke=broke, every=every)
    if diverged is not None:
        info["diverged_after_tcap"] = (diverged - steps) / info["t_cap"]
    if rec is not None:
        info["record"] = rec.result()
    if history:
        info["drops"] = history
        info["satellites"] = satellites(history, info)
    return (steps / info["t_cap"] if broke else float("nan")), steps, info


def satellites(history, info, frac=0.25):
    """Satellite droplets after the break-up: bodies whose volume is below
    `frac` of the largest body's.  Returns the largest number of them seen
    at one time, the number left at the end, and the longest unbroken
    stretch (in capillary times) during which at least one was present (the
    paper calls satellites stable when they live at least one capillary
    time)."""
    counts = []
    for t, bodies in history:
        vols = [b[2] for b in bodies]
        big = max(vols) if vols else 0.0
        counts.append((t, sum(1 for v in vols if v < frac * big)))
    if not counts:
        return {"max": 0, "final": 0, "life_tcap": 0.0, "bodies_final": 0}
    longest, start = 0.0, None
    for t, c in counts:
        if c > 0 and start is None:
            start = t
        if c == 0 and start is not None:
            longest = max(longest, t - start)
            start = None
    if start is not None:
        longest = max(longest, counts[-1][0] - start)
    return {"max": max(c for _, c in counts), "final": counts[-1][1],
            "life_tcap": longest / info["t_cap"], "bodies_final": len(history[-1][1])}


def save_record(path, info):
    """Writes the observables of one run to an .npz file."""
    r = info["record"]
    arrays = {k: r[k] for k in ("t_star", "h_min_over_R0", "neck_perturbation",
                                "crest_perturbation")}
    arrays["r_of_z"] = r["r_of_z"].astype(np.float32)
    for ts, (st, prof) in r["silhouettes"].items():
        arrays["silhouette_t%g" % ts] = prof
    for ts, (st, v) in r["velocity"].items():
        arrays["vstar_t%g_step%d" % (ts, st)] = v
    np.savez_compressed(path, **arrays)


def main():
    import argparse
    import json
    import os
    ap = argparse.ArgumentParser()
    ap.add_argument("--radii", default="14,28,42,56")
    ap.add_argument("--operators", default="mrt,srt")
    ap.add_argument("--eps", default="0.1", help="comma-separated delta / R0 values")
    ap.add_argument("--every", type=int, default=25)
    ap.add_argument("--record", default=None,
                    help="folder for per-run .npz files of the observables (Figs. 4-6)")
    ap.add_argument("--after", type=float, default=0.0,
                    help="capillary times to keep running after the break-up (satellites)")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--wavelengths", type=int, default=2, choices=[1, 2],
                    help="1: half the paper's box along the axis (one wavelength, same solution)")
    args = ap.parse_args()
    out = []
    for op in args.operators.split(","):
        for R0 in (int(r) for r in args.radii.split(",")):
            for eps in (float(e) for e in args.eps.split(",")):
                t, steps, info = break_time(R0, op, eps, args.every, precision=args.precision,
                                            progress=True, record=bool(args.record),
                                            after_tcap=args.after, wavelengths=args.wavelengths)
                rec = {"operator": op, "R0": R0, "eps": eps, "precision": args.precision,
                       "wavelengths": args.wavelengths,
                       "T_break_over_tcap": t,
                       "steps": steps, "box": [info["nx"], info["ny"], info["nz"]]}
                if "diverged_after_tcap" in info:
                    rec["diverged_after_tcap"] = info["diverged_after_tcap"]
                if "satellites" in info:
                    rec["satellites"] = info["satellites"]
                    rec["bodies_after"] = [[round(b[2], 1) for b in bodies]
                                           for _, bodies in info["drops"][::10]]
                if args.record:
                    os.makedirs(args.record, exist_ok=True)
                    path = os.path.join(args.record, "breakup_%s_R%d_eps%.4f.npz" % (op, R0, eps))
                    save_record(path, info)
                    rec["record"] = path
                print(json.dumps(rec), flush=True)
                out.append(rec)
    return out


if __name__ == "__main__":
    main()
