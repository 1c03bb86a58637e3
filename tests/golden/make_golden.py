"""Write tests/golden/alphas.json: step sizes alpha = 1/lambda_max of
p * A^T A (radial ramp filter, and no filter) for the 128^3 workload's
grids 0-1 and for the 64^3 crop of the 512^3 workload (grids 0-2), computed
by the FP64 oracle's power iteration (30 products, SplitMix64 start vector,
seed 0).

Only the oracle is called.  Usage:  python tests/golden/make_golden.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
from gpu_common import workload  # noqa: E402


def crop_geom():
    """Geometry of the central 64^3 box of the 512^3 workload on a 96^2
    detector (pixel 72/768) with all 1440 views."""
    import synth
    cfg = synth.CONFIGS["c2"]
    views = synth.trajectory(cfg.n_views, cfg.z_levels, cfg.pixel)
    return oracle.Geom(64, 64, 64, cfg.h, (0, 0, 0), 96, 96, views)


def main():
    path = os.path.join(HERE, "alphas.json")
    out = json.load(open(path)) if os.path.exists(path) else {}
    out["note"] = "alpha = 1/lambda, lambda from oracle.power_iteration(iters=30, seed=0)"
    if "c1" not in out:
        g = workload("c1")
        table, rho_max = oracle.radial_table(g.nx)
        filt = oracle.filter_radial(table, rho_max)
        out["c1"] = {"radial_ramp": [], "identity": []}
        for lv in (0, 1):
            gl = g.level(lv)
            out["c1"]["radial_ramp"].append(1.0 / oracle.power_iteration(gl, filt, iters=30, seed=0))
            out["c1"]["identity"].append(1.0 / oracle.power_iteration(gl, None, iters=30, seed=0))
            print("c1", lv, out["c1"]["radial_ramp"][-1], out["c1"]["identity"][-1], flush=True)
    if "c2_crop" not in out:
        g = crop_geom()
        table, rho_max = oracle.radial_table(g.nx)
        filt = oracle.filter_radial(table, rho_max)
        out["c2_crop"] = {"radial_ramp": []}
        for lv in (0, 1, 2):
            out["c2_crop"]["radial_ramp"].append(1.0 / oracle.power_iteration(g.level(lv), filt, iters=30, seed=0))
            print("c2_crop", lv, out["c2_crop"]["radial_ramp"][-1], flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
