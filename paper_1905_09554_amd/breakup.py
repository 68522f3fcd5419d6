"""Break-up time of a perturbed ligament (Sec. 4, Fig. 2b and Fig. 3 of the
paper): run until the neck pinches off and report T_break / t_cap.

Operators as in the paper (Sec. 2): "srt" is BGK with the velocity-shift
forcing of Eq. vel_shift; "mrt" is MRT with Guo-like forcing and the paper's
rate set (bulk and shear rates 1/tau, every other rate 1).

Break-up criterion (the paper does not state one): the first sampled step at
which some z-slice holds no node denser than the mid density
(rho_l + rho_v) / 2, i.e. the liquid column is cut.  Sampling every `every`
steps bounds the resolution of T_break to every / t_cap.
"""
import numpy as np
import torch

import lbm_inputs

from . import lbsc


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
    rho, _, _ = sim.moments(want_u=False, want_p=False)
    slice_max = rho.amax(dim=(1, 2))
    return bool((slice_max <= rho_mid).any())


def break_time(R0, operator, eps=0.1, every=25, max_tcap=12.0, precision="f32", progress=False):
    """(T_break / t_cap, steps, info) for the paper's run at radius R0."""
    rho0, info = lbm_inputs.paper_ligament(R0, operator, eps)
    sim = lbsc.Simulation(rho0, params_for(info, operator, precision))
    rho_mid = 0.5 * (info["rho_l"] + info["rho_v"])
    max_steps = int(max_tcap * info["t_cap"])
    steps = 0
    broke = False
    while steps < max_steps:
        sim.step(every)
        steps += every
        if neck_cut(sim, rho_mid):
            broke = True
            break
        if progress and steps % 2000 == 0:
            print("  R0=%d %s: %d steps (%.2f t_cap)" % (R0, operator, steps,
                                                       steps / info["t_cap"]), flush=True)
    torch.cuda.synchronize()
    sim.close()
    info = dict(info, steps=steps, broke=broke, every=every)
    return (steps / info["t_cap"] if broke else float("nan")), steps, info


def main():
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--radii", default="14,28,42,56")
    ap.add_argument("--operators", default="mrt,srt")
    ap.add_argument("--eps", type=float, default=0.1)
    ap.add_argument("--every", type=int, default=25)
    args = ap.parse_args()
    out = []
    for op in args.operators.split(","):
        for R0 in (int(r) for r in args.radii.split(",")):
            t, steps, info = break_time(R0, op, args.eps, args.every, progress=True)
            rec = {"operator": op, "R0": R0, "eps": args.eps, "T_break_over_tcap": t,
                   "steps": steps, "box": [info["nx"], info["ny"], info["nz"]]}
            print(json.dumps(rec), flush=True)
            out.append(rec)
    return out


if __name__ == "__main__":
    main()
