"""Benchmark: preconditioned multigrid Landweber reconstruction on one MI355X.

Workload (synthetic, seeded): 128^3 volume, 360 views of 192x192 on the
golden-angle + 8-level height-lattice trajectory, 60 random ellipsoids,
Poisson noise at I0 = 1e4.  One step = one full iteration of Algorithm 1
with 3 grids (restrict, OS-EMTR on the coarsest grid, prolongate, and on the
two finer grids a radially preconditioned Landweber step, soft threshold and
bilateral filter).  Inputs are resident in HBM before timing starts.

value = fine-grid voxel*views of one A + A^T pair per step (128^3 * 360) per
second of whole-step time: the paper prices one such iteration at about one
SIRT iteration.  The JSON line also carries the dominant kernel's roofline
(measured with HIP events inside the library), the time-to-residual against
plain SIRT on the same GPU, and the FP64 oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "c1"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sirt", action="store_true")
    ap.add_argument("--sirt-cap", type=int, default=1000)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (views would shard across "
              "GPUs with one sum-exchange of A^T per step; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2103_10329_amd as mg
    import synth

    cfg = synth.CONFIGS[WORKLOAD]
    n, V, nu, nv = cfg.n, cfg.n_views, cfg.nu, cfg.nv
    t0 = time.time()
    d = synth.make_dataset(WORKLOAD, truth=False)
    log("data %.1fs" % (time.time() - t0))
    views = d["views"]

    ctx = mg.Context(0)
    ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), nu, nv, views)
    b = torch.from_numpy(d["b"].astype(np.float32)).cuda()
    table = np.maximum(np.linspace(0, np.sqrt(3), 4097), 2.0 / n)
    filt = mg.filter_radial(table, np.sqrt(3))
    levels = cfg.levels
    lam, bil = 1e-3, (1.0, 0.05)

    # step sizes (once per geometry and filter): power iteration on the GPU
    torch.cuda.synchronize()
    t0 = time.time()
    alphas = [ctx.estimate_step(filt, level=g, iters=30, seed=0) for g in range(levels - 1)]
    torch.cuda.synchronize()
    t_alpha = time.time() - t0
    log("alphas", alphas, "%.3fs" % t_alpha)

    def step(vol):
        ctx.multigrid_solve(vol, b, levels, 1, filt, alphas=alphas, lam=lam, bilateral=bil, want_hist=False)

    vol = torch.zeros((n, n, n), device="cuda")
    for _ in range(args.warmup):
        step(vol)
    torch.cuda.synchronize()
    ctx.kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(vol)
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ctx.kernel_timing(False)
    ms_step = t_steps / args.steps * 1e3
    value = n ** 3 * V / (t_steps / args.steps) / 1e9

    kt = {}
    names = {mg.MGCT_OP_PROJECT: "project", mg.MGCT_OP_BACKPROJECT: "backproject",
             mg.MGCT_OP_PRECONDITION: "precondition", mg.MGCT_OP_VOLUME_TRANSPOSE: "volume_transpose",
             mg.MGCT_OP_DATA_PRESCALE: "data_prescale"}
    for op, name in names.items():
        for g in range(levels):
            ms, cnt = ctx.kernel_time(op, g)
            if cnt:
                kt["%s@%d" % (name, g)] = {"ms_avg": ms / cnt, "launches": cnt}
    # per-view-stream bytes of one fine-grid application (FP32 volume and data)
    bytes_per_launch = V * (n ** 3 * 4 + nu * nv * 4)
    tA = kt["project@0"]["ms_avg"]
    tB = kt["backproject@0"]["ms_avg"]
    dom = "backproject@0" if tB >= tA else "project@0"
    t_dom = kt[dom]["ms_avg"] * 1e-3
    achieved = bytes_per_launch / t_dom / 1e9
    roofline = {"kernel": "k_backproject_sep" if dom.startswith("back") else "k_project",
                "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": kt[dom]["ms_avg"]}
    a_at = n ** 3 * V / ((tA + tB) * 1e-3) / 1e9

    out = {
        "metric": "A+Aᵀ Gvoxel·views/s (% HBM roofline); time-to-residual vs plain SIRT",
        "value": value, "unit": "Gvoxel·views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "pmg-128^3-360x192^2-L3-radial", "volume": [n, n, n], "views": V,
                   "detector": [nv, nu], "levels": levels, "filter": "radial ramp max(rho,2/N)",
                   "soft_threshold": lam, "bilateral": list(bil), "coarse": "OS-EMTR M=8 x2"},
        "roofline": roofline,
        "a_plus_at_kernels_gvox_views_s": a_at,
        "kernels_ms": kt,
        "step_size_estimate_s": t_alpha,
    }

    # time-to-residual: 2 PMG iterations from zero vs plain SIRT from zero
    if not args.no_sirt:
        def resid(v):
            p = ctx.project(v)
            return float(torch.linalg.vector_norm((b - p).double()).item())

        bnorm = float(torch.linalg.vector_norm(b.double()).item())
        v = torch.zeros((n, n, n), device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            step(v)
        torch.cuda.synchronize()
        t_pmg = time.perf_counter() - t0
        r_pmg = resid(v)
        a_sirt = ctx.estimate_step(None, level=0, iters=30, seed=0)
        vs = torch.zeros((n, n, n), device="cuda")
        k, t_sirt, r_s = 0, 0.0, None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while k < args.sirt_cap:
            r_before = ctx.landweber_step(vs, b, a_sirt, None, want_norm=True)  # ||b - A mu_k||
            if r_before <= r_pmg:
                break
            k += 1
        torch.cuda.synchronize()
        t_sirt = time.perf_counter() - t0
        out["time_to_residual"] = {
            "target_rel_residual": r_pmg / bnorm, "pmg_iterations": 2, "pmg_s": t_pmg,
            "sirt_iterations": k if k < args.sirt_cap else None, "sirt_cap": args.sirt_cap,
            "sirt_s": t_sirt, "sirt_alpha": a_sirt,
            "speedup": (t_sirt / t_pmg) if k < args.sirt_cap else None}
        log("time-to-residual", out["time_to_residual"])

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, views, alphas, lam, bil)
    print(json.dumps(out), flush=True)
    ctx.close()


def cpu_baseline(d, views, alphas, lam, bil):
    """The FP64 oracle, as it stands, on the host cores: one full iteration of
    Algorithm 1 on the same workload (same data, steps and parameters)."""
    import oracle
    import synth
    cfg = synth.CONFIGS[WORKLOAD]
    n = cfg.n
    g = oracle.Geom(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views)
    table, rho_max = oracle.radial_table(n)
    f = oracle.filter_radial(table, rho_max)
    t0 = time.perf_counter()
    oracle.multigrid(g, np.zeros(g.vol_shape), d["b"], cfg.levels, 1, f, alphas, lam=lam, bilateral_on=True,
                     sigma_s=bil[0], sigma_r=bil[1])
    t = time.perf_counter() - t0
    return {"value": n ** 3 * cfg.n_views / t / 1e9, "unit": "Gvoxel·views/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": t,
            "sample": "one full iteration of Algorithm 1 (3 grids, same 128^3 x 360-view data) by the FP64 oracle"}


if __name__ == "__main__":
    main()
