"""Write tests/golden/alphas.json: step sizes alpha = 1/lambda_max of
p * A^T A for the 128^3 workload, computed by the FP64 oracle's power
iteration (30 products, SplitMix64 start vector, seed 0).

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


def main():
    g = workload("c1")
    table, rho_max = oracle.radial_table(g.nx)
    filt = oracle.filter_radial(table, rho_max)
    out = {"note": "alpha = 1/lambda, lambda from oracle.power_iteration(iters=30, seed=0)",
           "c1": {"radial_ramp": [], "identity": []}}
    for lv in (0, 1):
        gl = g.level(lv)
        out["c1"]["radial_ramp"].append(1.0 / oracle.power_iteration(gl, filt, iters=30, seed=0))
        out["c1"]["identity"].append(1.0 / oracle.power_iteration(gl, None, iters=30, seed=0))
        print(lv, out["c1"]["radial_ramp"][-1], out["c1"]["identity"][-1], flush=True)
    with open(os.path.join(HERE, "alphas.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
