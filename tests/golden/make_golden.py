"""Writes the stored values that tests and input builders read.

Calls only the oracle (float64 CPU).  Run from the repository root:

    python tests/golden/make_golden.py

Outputs
  lbm_inputs/coexistence.json   rho_v, rho_l of the flat-interface run for the
                                interaction strengths used by the workloads
                                (Sec. 3: flat-interface simulations provide the
                                liquid and vapour densities), and sigma from
                                the Laplace law of static cylinders (Sec. 3,
                                the Laplace test).
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import coexistence, lbm, physics  # noqa: E402


def flat_run(G):
    rv0, rl0, _ = coexistence.equal_area_rule(G)
    p = lbm.Params(G=G, tau=1.0, collision="bgk", forcing="guo")
    rv, rl, steps, _ = coexistence.flat_interface(p, nz=32, half_width=8,
                                                  rho_guess=(rv0, rl0), tol=1e-10)
    return {"rho_v": rv, "rho_l": rl, "steps": steps, "box": "1x1x32", "half_width": 8,
            "collision": "bgk", "tau": 1.0, "forcing": "guo", "tol": 1e-10,
            "equal_area_rule": {"rho_v": rv0, "rho_l": rl0}}


def main():
    out = {}
    for G in (-5.0, -5.3):
        out["%.4f" % G] = flat_run(G)
        rec = out["%.4f" % G]
        # Surface tension from the Laplace law of static cylinders (MRT).
        sigma, icpt, _ = physics.laplace_sigma(G, rec["rho_v"], rec["rho_l"])
        rec["sigma_laplace"] = {"sigma": sigma, "intercept": icpt, "radii": [8, 12, 16],
                                "box": "64x64x1", "collision": "mrt", "tau": 1.0}
        print(G, rec)
    with open(os.path.join(ROOT, "lbm_inputs", "coexistence.json"), "w") as fh:
        json.dump(out, fh, indent=1, sort_keys=True)
        fh.write("\n")


if __name__ == "__main__":
    main()
