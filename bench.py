"""Benchmark: preconditioned multigrid Landweber reconstruction on one MI355X.

Workload (synthetic, seeded): 512^3 volume, 1440 views of 768x768 on the
golden-angle + 8-level height-lattice trajectory, 400 random ellipsoids plus
5 % cubic inclusions, Poisson noise at I0 = 5e3 (generated on the device from
the same definitions as the CPU generator).  One step = one full iteration
of Algorithm 1 with 4 grids (restrict, OS-EMTR on the coarsest 64^3 grid,
prolongate, and on the three finer grids a radially preconditioned Landweber
step, soft threshold and bilateral filter), FP32 storage.  Inputs are
resident in HBM before timing starts.

value = fine-grid voxel*views of one A + A^T pair per step (512^3 * 1440) per
second of whole-step time: the paper prices one such iteration at about one
SIRT iteration.  The JSON line also carries the dominant kernel's roofline
(HIP events recorded inside the library on the launch stream), the same
operators with BF16 volume / FP16 stack storage, time-to-residual and image
error against plain SIRT on the same data, the 128^3 workload's
time-to-residual against SIRT and OS-EMTR (with the learned and derived
preconditioners), and the FP64 oracle timed on the host cores.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--workload c2|c1]
                    [--no-cpu-baseline] [--no-quality]
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
WORKLOAD_NAMES = {
    "c2": "pmg-512^3-1440x768^2-L4-radial",
    "c1": "pmg-128^3-360x192^2-L3-radial",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOAD_NAMES), default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-quality", action="store_true")
    ap.add_argument("--sirt-cap", type=int, default=60)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales the HBM byte counters)")
    ap.add_argument("--paper-shaped", action="store_true",
                    help="only run the 640x640x2304 / 3600 x 760^2 workload (prints its own JSON line)")
    ap.add_argument("--quality-sweep", action="store_true",
                    help="only run the 128^3 image-error sweep over the regularisation readings and iteration "
                         "counts of Algorithm 1 (prints its own JSON line)")
    ap.add_argument("--oracle-solves", action="store_true",
                    help="only time whole solves of the FP64 oracle on all host threads beside the library: 20 SIRT "
                         "iterations on the 32^3 workload, 2 iterations of Algorithm 1 on the 128^3 one "
                         "(prints its own JSON line)")
    ap.add_argument("--view-share", type=int, metavar="K",
                    help="only time A and A^T on each share of a round-robin split of the 512^3 workload's views "
                         "into K (what one of K GPUs would run), check that the shares compose to the whole, and "
                         "model the sum exchange (prints its own JSON line)")
    ap.add_argument("--cnn-forward", type=int, metavar="N",
                    help="only time the learned preconditioner's forward pass on an N^3 grid, --warmup untimed "
                         "and --steps timed passes (prints its own JSON line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the views would shard across "
              "GPUs, with one sum-exchange of the A^T partial volumes per step).", file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return
    if args.paper_shaped:
        paper_shaped()
        return
    if args.cnn_forward:
        cnn_forward_timing(args.cnn_forward, args.steps, args.warmup)
        return
    if args.view_share:
        view_share(args.view_share, args.steps)
        return
    if args.quality_sweep:
        quality_sweep()
        return
    if args.oracle_solves:
        oracle_solves()
        return

    import torch

    import paper_2103_10329_amd as mg
    import synth
    from paper_2103_10329_amd import learned as lrn

    wl = args.workload
    cfg = synth.CONFIGS[wl]
    idx = int(wl[1:])
    n, V, nu, nv = cfg.n, cfg.n_views, cfg.nu, cfg.nv
    views = synth.trajectory(V, cfg.z_levels, cfg.pixel)
    ctx = mg.Context(0)
    ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), nu, nv, views)
    # data on the device: phantom seed 1000 + k, noise seed 2000 + k
    t0 = time.time()
    ph = synth.random_phantom(cfg, 1000 + idx)
    gen = torch.Generator(device="cuda").manual_seed(2000 + idx)
    b = lrn.poisson_data(ctx.synth_line_integrals(ph), cfg.noise_level, gen)
    torch.cuda.synchronize()
    log("data %.1fs" % (time.time() - t0))
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
    log("alphas", alphas, "%.1fs" % t_alpha)

    def step(vol):
        ctx.multigrid_solve(vol, b, levels, 1, filt, alphas=alphas, lam=lam, bilateral=bil, want_hist=False)

    vol = torch.zeros((n, n, n), device="cuda")
    for _ in range(args.warmup):
        step(vol)
    torch.cuda.synchronize()
    # inside the timed region only the fine grid's A and A^T launches are
    # bracketed by events (each event is a command on the stream)
    ctx.kernel_timing(True, ops=(mg.MGCT_OP_PROJECT, mg.MGCT_OP_BACKPROJECT), levels=(0,))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(vol)
        if wl == "c2":
            torch.cuda.synchronize()
            log("step %d/%d %.3fs" % (k + 1, args.steps, time.perf_counter() - t0))
    torch.cuda.synchronize()
    t_steps = time.perf_counter() - t0
    ctx.kernel_timing(False)
    ms_step = t_steps / args.steps * 1e3
    value = n ** 3 * V / (t_steps / args.steps) / 1e9

    names = {mg.MGCT_OP_PROJECT: "project", mg.MGCT_OP_BACKPROJECT: "backproject",
             mg.MGCT_OP_PRECONDITION: "precondition", mg.MGCT_OP_VOLUME_TRANSPOSE: "volume_transpose",
             mg.MGCT_OP_DATA_PRESCALE: "data_prescale"}

    def collect(ops, grids):
        out = {}
        for op in ops:
            name = names[op]
            for g in grids:
                ms, cnt = ctx.kernel_time(op, g)
                if cnt:
                    e = {"ms_avg": ms / cnt, "launches": cnt}
                    if name in ("project", "backproject"):
                        e["gvox_views_s"] = (n >> g) ** 3 * V / (ms / cnt * 1e-3) / 1e9
                    out["%s@%d" % (name, g)] = e
        return out

    live = collect((mg.MGCT_OP_PROJECT, mg.MGCT_OP_BACKPROJECT), (0,))
    # every instrumented kernel on every grid, from one further step after the
    # timed region; the fine grid's A and A^T keep their timed-region figures
    ctx.kernel_timing(True)
    step(vol)
    torch.cuda.synchronize()
    ctx.kernel_timing(False)
    kt = collect(names.keys(), range(levels))
    kt.update(live)
    # per-view-stream bytes of one fine-grid application (FP32 volume and data)
    bytes_per_launch = V * (n ** 3 * 4 + nu * nv * 4)
    tA = kt["project@0"]["ms_avg"]
    tB = kt["backproject@0"]["ms_avg"]
    dom = "backproject@0" if tB >= tA else "project@0"
    roofline = make_roofline(dom, kt[dom]["ms_avg"], bytes_per_launch, n ** 3 * V, wl)
    a_at = n ** 3 * V / ((tA + tB) * 1e-3) / 1e9
    a_at_grid = {}
    for g in range(levels):
        ka, kb = kt.get("project@%d" % g), kt.get("backproject@%d" % g)
        if ka and kb:
            a_at_grid[str(g)] = (n >> g) ** 3 * V / ((ka["ms_avg"] + kb["ms_avg"]) * 1e-3) / 1e9

    out = {
        "metric": "A+Aᵀ Gvoxel·views/s (% HBM roofline); time-to-residual vs plain SIRT",
        "value": value, "unit": "Gvoxel·views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[wl], "volume": [n, n, n], "views": V,
                   "detector": [nv, nu], "levels": levels, "filter": "radial ramp max(rho,2/N)",
                   "soft_threshold": lam, "bilateral": list(bil), "coarse": "OS-EMTR M=8 x2",
                   "phantom": "%d ellipsoids%s, Poisson I0=%g" % (
                       cfg.n_ellipsoids, " + %g%% cubes" % (100 * cfg.cube_fraction) if cfg.cube_fraction else "",
                       cfg.noise_level)},
        "roofline": roofline,
        "in_cone_fraction": in_cone_fraction(views, n, n, n, cfg.h, nu, nv),
        "a_plus_at_kernels_gvox_views_s": a_at,
        "a_plus_at_hbm_frac": 2 * bytes_per_launch / ((tA + tB) * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels_ms": kt,
        "a_plus_at_gvox_views_s_by_grid": a_at_grid,
        "step_size_estimate_s": t_alpha,
    }
    out["mixed_precision"] = mixed_precision(ctx, mg, b, n, V, step, bytes_per_launch)
    torch.cuda.synchronize()

    if not args.no_quality:
        out["time_to_residual"] = time_to_residual(ctx, mg, synth, ph, b, cfg, levels, filt, alphas, lam, bil,
                                                   args.sirt_cap)
        if os.path.exists(lrn.DEFAULT_WEIGHTS):
            # the learned preconditioner's network alone on this grid (what its step adds)
            out["cnn_forward"] = time_cnn_forward(ctx, n, 5, 1)
        if wl != "c1":
            ctx.close()
            del b, vol
            torch.cuda.empty_cache()
            out["c1"] = quality_c1(args)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, views)
    print(json.dumps(out), flush=True)


# HBM-side traffic of the dominant kernels from rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes (KiB per dispatch), scaled by the same counters on a plain
# 1 GiB copy (fetch x2.0, write x1.0), per launch, with their VALU and LDS
# issue fractions (wave-instructions per CU cycle), L2 hit rates and VALU
# instructions per voxel*view from the SQ/TCC pass; valid only for the kernel
# source they were measured on (the fine grid of the 512^3 workload, one
# Algorithm 1 step: A with the residual epilogue, A^T from the FP32 stack).
TRAFFIC = {
    ("k_project_lds", "c2"): {
        "source_sha256": "406188f30e88d0bd7c61982b100bcdc435ecdff2f354cafe3be849eccf83db63",
        "bytes_per_launch": 1.447e12, "fetch_kib": 6.818e8, "write_kib": 4.927e7,
        "valu_issue": 0.774, "lds_issue": 0.104, "l2_hit": 0.125, "valu_insts_per_voxel_view": 35.4,
        "profile": "profiles/project_backproject_512cube_1440x768_counters.md"},
    ("k_backproject_pl", "c2"): {
        "source_sha256": "406188f30e88d0bd7c61982b100bcdc435ecdff2f354cafe3be849eccf83db63",
        "bytes_per_launch": 4.983e11, "fetch_kib": 2.424e8, "write_kib": 1.765e6,
        "valu_issue": 0.877, "lds_issue": 0.119, "l2_hit": 0.077, "valu_insts_per_voxel_view": 35.8,
        "profile": "profiles/project_backproject_512cube_1440x768_counters.md"},
}


def measured_counters(kernel, workload):
    """The committed counter figures for `kernel` on `workload`, or None when
    the source has changed since they were taken."""
    import hashlib
    t = TRAFFIC.get((kernel, workload))
    if not t:
        return None
    src = os.path.join(ROOT, "paper_2103_10329_amd", "csrc", "joseph.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
            return None
    return t


# Algorithmic FP32 operations per voxel*view, FMA counted as two: A does
# about 12 per Joseph sample (two z interpolations and the in-plane blend with
# the fixed-point step) at 1.45 samples per voxel*view on these trajectories;
# A^T forms about 6 non-zero (ray, voxel) weights per voxel*view, each a hat
# product and a multiply-add (about 24 in all).
ALG_OPS = {"project@0": 1.45 * 12, "backproject@0": 24.0}


def make_roofline(dom, ms_avg, bytes_per_launch, voxel_views, workload):
    """Roofline of the dominant kernel.  The metric's HBM model is the
    per-view-stream bytes V (N^3 s_vol + U W s_det) per launch; the measured
    counters (when present for this source) decide which unit binds: HBM
    (counter bytes per second against 8 TB/s) or the vector ALUs (VALU issue
    against one wave-instruction per CU cycle)."""
    kname = "k_backproject_pl" if dom.startswith("back") else "k_project_lds"
    t = ms_avg * 1e-3
    hbm_achieved = bytes_per_launch / t / 1e9
    cnt = measured_counters(kname, workload)
    r = {"kernel": kname, "bound": "hbm", "achieved": hbm_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": hbm_achieved / HBM_PEAK_GBS, "traffic": cnt["bytes_per_launch"] if cnt else None,
         "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": ms_avg,
         "per_view_stream_frac": hbm_achieved / HBM_PEAK_GBS}
    if cnt:
        hbm_util = cnt["bytes_per_launch"] / t / 1e9 / HBM_PEAK_GBS
        r.update({"valu_issue": cnt["valu_issue"], "lds_issue": cnt.get("lds_issue"), "l2_hit": cnt["l2_hit"],
                  "hbm_util_measured": hbm_util, "valu_insts_per_voxel_view": cnt["valu_insts_per_voxel_view"],
                  "counters": cnt["profile"]})
        if cnt["valu_issue"] > hbm_util:
            ops = ALG_OPS[dom] * voxel_views
            ach = ops / t / 1e12
            r.update({"bound": "alu", "achieved": ach, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                      "frac": ach / FP32_VECTOR_PEAK_TFLOPS, "algorithmic_ops_per_launch": ops})
    return r


def mixed_precision(ctx, mg, b, n, V, step, bytes_fp32):
    """The same operators with BF16 volume copies and FP16 stacks (FP32
    accumulation): one A from a BF16 volume to an FP16 stack, one A^T from an
    FP16 stack, one Algorithm 1 iteration with mixed storage."""
    import torch
    x = torch.rand((n, n, n), device="cuda", generator=torch.Generator(device="cuda").manual_seed(7))
    xb = x.to(torch.bfloat16)
    y = b.half()
    p = ctx.project(xb, out_dtype=torch.float16)
    q = ctx.backproject(y)
    torch.cuda.synchronize()
    ctx.kernel_timing(True, ops=(mg.MGCT_OP_PROJECT, mg.MGCT_OP_BACKPROJECT), levels=(0,))
    ctx.project(xb, out=p)
    ctx.backproject(y, out=q)
    torch.cuda.synchronize()
    ctx.kernel_timing(False)
    tA = ctx.kernel_time(mg.MGCT_OP_PROJECT, 0)[0]
    tB = ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, 0)[0]
    ctx.set_precision("bfloat16", "float16")
    v = torch.zeros((n, n, n), device="cuda")
    step(v)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step(v)
    torch.cuda.synchronize()
    t_step = time.perf_counter() - t0
    ctx.set_precision("float32", "float32")
    bytes_mixed = V * (n ** 3 * 2 + b[0].numel() * 2)
    del x, xb, y, p, q, v
    return {"storage": "BF16 volume copies, FP16 stacks, FP32 accumulation",
            "A_ms": tA, "At_ms": tB, "A_gvox_views_s": n ** 3 * V / (tA * 1e-3) / 1e9,
            "At_gvox_views_s": n ** 3 * V / (tB * 1e-3) / 1e9,
            "a_plus_at_gvox_views_s": n ** 3 * V / ((tA + tB) * 1e-3) / 1e9,
            "per_view_stream_frac_A": bytes_mixed / (tA * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "step_ms": t_step * 1e3, "step_gvox_views_s": n ** 3 * V / t_step / 1e9}


def time_to_residual(ctx, mg, synth, ph, b, cfg, levels, filt, alphas, lam, bil, cap):
    """Two iterations of Algorithm 1 from zero against plain SIRT (eq. 2, its
    own power-iteration step) from zero until it reaches the same relative
    residual ||b - A mu|| / ||b||, on the same GPU; masked image error against
    the voxelised phantom after 2 iterations of each."""
    import torch
    n = cfg.n
    truth = ctx.synth_voxelize(ph, ss=2)
    mask = torch.from_numpy(synth.evaluation_mask(n, cfg.h)).cuda()
    tm = truth[mask].double()

    def err(v):
        return float(torch.linalg.vector_norm(v[mask].double() - tm) / torch.linalg.vector_norm(tm))

    def resid(v):
        return float(torch.linalg.vector_norm((b - ctx.project(v)).double()).item())

    bnorm = float(torch.linalg.vector_norm(b.double()).item())
    v = torch.zeros((n, n, n), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.multigrid_solve(v, b, levels, 2, filt, alphas=alphas, lam=lam, bilateral=bil, want_hist=False)
    torch.cuda.synchronize()
    t_pmg = time.perf_counter() - t0
    r_pmg = resid(v)
    e_pmg = err(v)
    del v
    a_sirt = ctx.estimate_step(None, level=0, iters=30, seed=0)
    vs = torch.zeros((n, n, n), device="cuda")
    k, e_sirt2 = 0, None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while k < cap:
        if ctx.landweber_step(vs, b, a_sirt, None, want_norm=True) <= r_pmg:  # ||b - A mu_k||
            break
        k += 1
        if k == 2:
            torch.cuda.synchronize()
            t_pause = time.perf_counter()
            e_sirt2 = err(vs)
            t0 += time.perf_counter() - t_pause
    torch.cuda.synchronize()
    t_sirt = time.perf_counter() - t0
    out = {"target_rel_residual": r_pmg / bnorm, "pmg": {"iterations": 2, "seconds": t_pmg,
                                                        "image_error_masked": e_pmg},
           "sirt_iterations": k if k < cap else None, "sirt_cap": cap, "sirt_s": t_sirt, "sirt_alpha": a_sirt,
           "sirt_image_error_masked_2": e_sirt2,
           "speedup_vs_sirt": (t_sirt / t_pmg) if k < cap else None}
    log("time-to-residual", out)
    del vs, truth
    return out


def quality_c1(args):
    """The 128^3 workload's time-to-residual and image errors (plain, learned
    and derived preconditioners; SIRT and OS-EMTR), on a context of its own."""
    import torch

    import paper_2103_10329_amd as mg
    import synth
    cfg = synth.CONFIGS["c1"]
    n = cfg.n
    d = synth.make_dataset("c1", truth=True)
    ctx = mg.Context(0)
    ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, d["views"])
    b = torch.from_numpy(d["b"].astype(np.float32)).cuda()
    table = np.maximum(np.linspace(0, np.sqrt(3), 4097), 2.0 / n)
    filt = mg.filter_radial(table, np.sqrt(3))
    lam, bil = 1e-3, (1.0, 0.05)
    alphas = [ctx.estimate_step(filt, level=g, iters=30, seed=0) for g in range(cfg.levels - 1)]

    def step(vol):
        ctx.multigrid_solve(vol, b, cfg.levels, 1, filt, alphas=alphas, lam=lam, bilateral=bil, want_hist=False)

    vol = torch.zeros((n, n, n), device="cuda")
    step(vol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(10):
        step(vol)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 10 * 1e3
    res = quality(ctx, mg, b, d, step, cfg.levels, filt, alphas, lam, bil, args)
    res["workload"] = WORKLOAD_NAMES["c1"]
    res["ms_per_step"] = ms
    res["value_gvox_views_s"] = n ** 3 * cfg.n_views / (ms * 1e-3) / 1e9
    ctx.close()
    return res


def quality_sweep():
    """Masked image error on the 128^3 workload (the same data, mask and
    radial filter as quality_c1) of Algorithm 1 from zero after 1, 2, 4 and 10
    iterations for the soft-threshold weight lambda in {0, 1e-3, 1e-2} with
    and without the bilateral filter (sigma_s 1, sigma_r 0.05), and of
    full-resolution OS-EMTR (8 subsets) after 2, 4 and 10 iterations."""
    import torch

    import paper_2103_10329_amd as mg
    import synth
    cfg = synth.CONFIGS["c1"]
    n = cfg.n
    d = synth.make_dataset("c1", truth=True)
    ctx = mg.Context(0)
    ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, d["views"])
    b = torch.from_numpy(d["b"].astype(np.float32)).cuda()
    table = np.maximum(np.linspace(0, np.sqrt(3), 4097), 2.0 / n)
    filt = mg.filter_radial(table, np.sqrt(3))
    alphas = [ctx.estimate_step(filt, level=g, iters=30, seed=0) for g in range(cfg.levels - 1)]
    truth = torch.from_numpy(d["mu"].astype(np.float32)).cuda()
    mask = torch.from_numpy(synth.evaluation_mask(n, cfg.h)).cuda()
    tm = truth[mask].double()

    def err(v):
        return float(torch.linalg.vector_norm(v[mask].double() - tm) / torch.linalg.vector_norm(tm))

    rows = []
    for lam in (0.0, 1e-3, 1e-2):
        for bil in (None, (1.0, 0.05)):
            e = {}
            for it in (1, 2, 4, 10):
                v = torch.zeros((n, n, n), device="cuda")
                ctx.multigrid_solve(v, b, cfg.levels, it, filt, alphas=alphas, lam=lam, bilateral=bil,
                                    want_hist=False)
                e[it] = err(v)
            rows.append({"lambda": lam, "bilateral": list(bil) if bil else None, "masked_error": e})
    vo = torch.zeros((n, n, n), device="cuda")
    os_err = {}
    for k in range(1, 11):
        ctx.osemtr(vo, b, subsets=8, passes=1, level=0)
        if k in (2, 4, 10):
            os_err[k] = err(vo)
    ctx.close()
    print(json.dumps({"quality_sweep": {"workload": WORKLOAD_NAMES["c1"], "algorithm1": rows,
                                        "osemtr_8_subsets": os_err}}), flush=True)


def quality(ctx, mg, b, d, step, levels, filt, alphas, lam, bil, args):
    """Time-to-residual and image error.  Target: the relative residual
    ||b - A mu|| / ||b|| of 2 iterations of Algorithm 1 from zero.  Plain SIRT
    (unfiltered Landweber, eq. 2) and full-resolution OS-EMTR (eq. 3, 8
    subsets per iteration) run from zero until they reach it.  Image error:
    masked relative L2 error against the phantom (cylinder of radius 14.4,
    |z| <= 12) for SIRT after 2 and 10 iterations, OS-EMTR after 2 and 10,
    Algorithm 1 after 2 plain, with the preconditioner derived from the scan's
    point-spread function, and, with trained weights present, learned."""
    import torch

    import synth
    from paper_2103_10329_amd import learned as lrn
    cfg = synth.CONFIGS["c1"]
    n = cfg.n
    truth = torch.from_numpy(d["mu"].astype(np.float32)).cuda()
    mask = torch.from_numpy(synth.evaluation_mask(n, cfg.h)).cuda()
    tm = truth[mask].double()

    def err(v):
        return float(torch.linalg.vector_norm(v[mask].double() - tm) / torch.linalg.vector_norm(tm))

    def resid(v):
        return float(torch.linalg.vector_norm((b - ctx.project(v)).double()).item())

    bnorm = float(torch.linalg.vector_norm(b.double()).item())
    v = torch.zeros((n, n, n), device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        step(v)
    torch.cuda.synchronize()
    t_pmg = time.perf_counter() - t0
    r_pmg = resid(v)
    errors = {"pmg_plain_2": err(v)}
    pmg = {"iterations": 2, "seconds": t_pmg, "rel_residual": r_pmg / bnorm}

    # learned step (weights trained by paper_2103_10329_amd.learned on the
    # same phantom distribution), same parameters otherwise
    if os.path.exists(lrn.DEFAULT_WEIGHTS):
        ctx.cnn_set_weights(lrn.load_weights())
        vl = torch.zeros((n, n, n), device="cuda")
        ctx.multigrid_solve(vl, b, levels, 1, filt, alphas=alphas, lam=lam, bilateral=bil,
                            want_hist=False, learned=True)  # warm-up of the network buffers
        vl.zero_()
        ctx.learned_stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.multigrid_solve(vl, b, levels, 2, filt, alphas=alphas, lam=lam, bilateral=bil,
                            want_hist=False, learned=True)
        torch.cuda.synchronize()
        t_l = time.perf_counter() - t0
        acc, rej = ctx.learned_stats()
        errors["pmg_learned_2"] = err(vl)
        pmg["learned"] = {"seconds": t_l, "rel_residual": resid(vl) / bnorm, "accepted": acc, "rejected": rej}

    # the preconditioner derived from the scan's own point-spread function
    # (anisotropic 1/max(T(k), 0.03 T(0)) per grid), same parameters otherwise
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fd = ctx.derived_filter(levels - 1)
    alphas_d = [ctx.estimate_step(fd, level=g, iters=30, seed=0) for g in range(levels - 1)]
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    vd = torch.zeros((n, n, n), device="cuda")
    ctx.multigrid_solve(vd, b, levels, 1, fd, alphas=alphas_d, lam=lam, bilateral=bil, want_hist=False)
    vd.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.multigrid_solve(vd, b, levels, 2, fd, alphas=alphas_d, lam=lam, bilateral=bil, want_hist=False)
    torch.cuda.synchronize()
    t_d = time.perf_counter() - t0
    errors["pmg_derived_2"] = err(vd)
    pmg["derived_filter"] = {"seconds": t_d, "rel_residual": resid(vd) / bnorm, "setup_s": t_setup,
                             "filter": "anisotropic 1/max(T(k), 0.03 T(0)) from A^T A's impulse response"}

    # SIRT: from zero until ||b - A mu_k|| <= target
    a_sirt = ctx.estimate_step(None, level=0, iters=30, seed=0)
    vs = torch.zeros((n, n, n), device="cuda")
    k = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cap1 = 1000
    while k < cap1:
        if ctx.landweber_step(vs, b, a_sirt, None, want_norm=True) <= r_pmg:  # ||b - A mu_k||
            break
        k += 1
    torch.cuda.synchronize()
    t_sirt = time.perf_counter() - t0
    vs.zero_()
    for it in range(1, 11):
        ctx.landweber_step(vs, b, a_sirt, None, want_norm=False)
        if it in (2, 10):
            errors["sirt_%d" % it] = err(vs)

    # OS-EMTR at full resolution, 8 subsets per iteration
    vo = torch.zeros((n, n, n), device="cuda")
    cap_os = 200
    reached, t_os = None, 0.0
    for ko in range(1, cap_os + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.osemtr(vo, b, subsets=8, passes=1, level=0)
        torch.cuda.synchronize()
        t_os += time.perf_counter() - t0
        if ko in (2, 10):
            errors["osemtr_%d" % ko] = err(vo)
        if reached is None and resid(vo) <= r_pmg:
            reached = (ko, t_os)
        if reached is not None and ko >= 10:
            break
    ttr = {"target_rel_residual": r_pmg / bnorm, "pmg": pmg,
           "sirt_iterations": k if k < cap1 else None, "sirt_cap": cap1,
           "sirt_s": t_sirt, "sirt_alpha": a_sirt,
           "speedup_vs_sirt": (t_sirt / t_pmg) if k < cap1 else None,
           "osemtr_iterations": reached[0] if reached else None, "osemtr_s": reached[1] if reached else None,
           "osemtr_cap": cap_os}
    log("time-to-residual", ttr)
    log("masked image error", errors)
    return {"time_to_residual": ttr, "image_error_masked": errors}


def paper_shaped():
    """The paper's data shape on one GPU (Sec. 2: 3600 radiographs of 760^2,
    a 640 x 640 x 2304 volume), FP32: one A and one A^T over all views, then
    two iterations of Algorithm 1 on 4 grids with eq. 5's stencil (the FFT
    filter needs power-of-two edges), a synthetic tall phantom and Poisson
    data.  Step sizes: power iteration on every 10th view, scaled by the view
    ratio (A^T A sums over views) and by 0.95.  Image error per height band
    inside the evaluation cylinder shows the sample's ends, seen by fewer
    views, reconstructing worse."""
    import torch

    import paper_2103_10329_amd as mg
    import synth
    cfg = synth.PAPER_SHAPED
    nx, nz, V = cfg.n, synth.PAPER_SHAPED_NZ, cfg.n_views
    views = synth.helix_trajectory(V, cfg.pixel)
    ctx = mg.Context(0)
    ctx.set_geometry(nx, nx, nz, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views)
    t0 = time.time()
    ph = synth.random_phantom(cfg, 5000, extent=(32.0, 32.0, nz * cfg.h))
    truth = ctx.synth_voxelize(ph, ss=2)
    gen = torch.Generator(device="cuda").manual_seed(6000)
    b_true = ctx.synth_line_integrals(ph)
    counts = torch.poisson(cfg.noise_level * torch.exp(-b_true.double()), generator=gen)
    b = torch.log(cfg.noise_level / torch.clamp(counts, min=1.0)).float()
    del counts, b_true
    torch.cuda.synchronize()
    log("paper-shaped data %.1fs" % (time.time() - t0))
    frac_in = in_cone_fraction(views, nx, nx, nz, cfg.h, cfg.nu, cfg.nv)
    out = {"workload": "paper-shaped 640x640x2304, 3600 views of 760^2, FP32", "voxel_views": nx * nx * nz * V,
           "in_cone_fraction": frac_in, "voxel_views_in_cone": nx * nx * nz * V * frac_in}
    # one A and one A^T (after a warm-up of each), HIP-event kernel times
    vol = truth.clone()
    p = ctx.project(vol)
    ctx.backproject(p)
    torch.cuda.synchronize()
    ctx.kernel_timing(True)
    ctx.project(vol, out=p)
    q = ctx.backproject(p)
    torch.cuda.synchronize()
    ctx.kernel_timing(False)
    tA = ctx.kernel_time(mg.MGCT_OP_PROJECT, 0)[0]
    tB = ctx.kernel_time(mg.MGCT_OP_BACKPROJECT, 0)[0]
    n4 = out["voxel_views_in_cone"]  # rates count in-cone voxel*views only
    out["A_ms"], out["At_ms"] = tA, tB
    out["A_gvox_views_s"] = n4 / (tA * 1e-3) / 1e9
    out["At_gvox_views_s"] = n4 / (tB * 1e-3) / 1e9
    out["a_plus_at_gvox_views_s"] = n4 / ((tA + tB) * 1e-3) / 1e9
    log("paper-shaped A %.1f ms, A^T %.1f ms" % (tA, tB))
    del p, q
    # step sizes from every 10th view
    filt = mg.filter_eq5()
    sub = mg.Context(0)
    sub.set_geometry(nx, nx, nz, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views[::10])
    alphas = [0.95 * sub.estimate_step(filt, level=g, iters=10, seed=0) / 10.0 for g in range(cfg.levels - 1)]
    sub.close()
    out["alphas"] = alphas
    log("paper-shaped alphas", alphas)
    # two iterations of Algorithm 1 from zero
    xc = (np.arange(nx) - (nx - 1) / 2.0) * cfg.h
    mask = torch.from_numpy(xc[None, :] ** 2 + xc[:, None] ** 2 <= 14.4 ** 2).cuda()[None]  # cylinder, [1][y][x]
    zc = torch.from_numpy((np.arange(nz) - (nz - 1) / 2.0) * cfg.h).cuda()
    # a height z is seen from source heights within ~17.6 of it (the detector's
    # half-height at the axis) inside [-48, 48]: every view angle for |z| <= 30,
    # about 70-55 % of them at 36 <= |z| <= 46 (the phantom reaches |z| ~ 44)
    bands = {"middle |z|<=20": zc.abs() <= 20.0, "ends 36<=|z|<=46": (zc.abs() >= 36.0) & (zc.abs() <= 46.0)}
    bn = float(torch.linalg.vector_norm(b.double()))
    vol.zero_()
    iters = []
    for it in range(2):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.multigrid_solve(vol, b, cfg.levels, 1, filt, alphas=alphas, want_hist=False)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        r = float(torch.linalg.vector_norm((b - ctx.project(vol)).double())) / bn
        errs = {}
        for name, zb in bands.items():
            m = mask & zb[:, None, None]
            t = truth[m].double()
            errs[name] = float(torch.linalg.vector_norm(vol[m].double() - t) / torch.linalg.vector_norm(t))
        iters.append({"seconds": dt, "rel_residual": r, "masked_error": errs})
        log("paper-shaped iteration", it + 1, iters[-1])
    out["pmg_iterations"] = iters
    print(json.dumps(out), flush=True)
    ctx.close()


def view_share(k, steps):
    """One GPU's part of a K-GPU view sharding of the 512^3 / 1440-view
    workload, FP32: views r, r + K, r + 2K, ... go to GPU r.  For every share
    r the fine-grid A and A^T are timed (HIP events, `steps` launches each
    after one untimed launch) on a context holding only that share's views;
    the share's A must equal the matching rows of the full A bit for bit and
    the shares' A^T must add up to the full A^T.  A K-GPU step would then take
    the slowest share's A + A^T plus one sum exchange of the A^T partial
    volumes, modelled as a ring all-reduce over xGMI (one 153 GB/s link per
    direction: 2 (K - 1)/K x volume bytes / 153 GB/s), without overlap."""
    import torch

    import paper_2103_10329_amd as mg
    import synth
    cfg = synth.CONFIGS["c2"]
    n, V = cfg.n, cfg.n_views
    views = synth.trajectory(V, cfg.z_levels, cfg.pixel)
    gen = torch.Generator(device="cuda").manual_seed(31)
    x = torch.rand((n, n, n), device="cuda", generator=gen)
    y = torch.rand((V, cfg.nv, cfg.nu), device="cuda", generator=gen)
    full = mg.Context(0)
    full.set_geometry(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views)
    a_full = full.project(x)
    b_full = full.backproject(y)
    full.kernel_timing(True, ops=(mg.MGCT_OP_PROJECT, mg.MGCT_OP_BACKPROJECT), levels=(0,))
    for _ in range(steps):
        full.project(x, out=a_full)
        full.backproject(y, out=b_full)
    torch.cuda.synchronize()
    full.kernel_timing(False)
    tA_full = full.kernel_time(mg.MGCT_OP_PROJECT, 0)
    tB_full = full.kernel_time(mg.MGCT_OP_BACKPROJECT, 0)
    full.close()
    acc = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    shares, identical = [], True
    for r in range(k):
        c = mg.Context(0)
        c.set_geometry(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, views[r::k])
        yr = y[r::k].contiguous()
        p = c.project(x)
        q = c.backproject(yr)
        torch.cuda.synchronize()
        identical &= bool(torch.equal(p, a_full[r::k]))
        acc += q.double()
        c.kernel_timing(True, ops=(mg.MGCT_OP_PROJECT, mg.MGCT_OP_BACKPROJECT), levels=(0,))
        for _ in range(steps):
            c.project(x, out=p)
            c.backproject(yr, out=q)
        torch.cuda.synchronize()
        c.kernel_timing(False)
        tA = c.kernel_time(mg.MGCT_OP_PROJECT, 0)
        tB = c.kernel_time(mg.MGCT_OP_BACKPROJECT, 0)
        shares.append({"views": len(views[r::k]), "A_ms": tA[0] / tA[1], "At_ms": tB[0] / tB[1]})
        log("view share", r, shares[-1])
        c.close()
        del p, q, yr
    err = float(torch.linalg.vector_norm(acc - b_full.double()) / torch.linalg.vector_norm(b_full.double()))
    vol_bytes = n ** 3 * 4
    allreduce_ms = 2.0 * (k - 1) / k * vol_bytes / 153e9 * 1e3
    slowest = max(s["A_ms"] + s["At_ms"] for s in shares)
    full_ms = tA_full[0] / tA_full[1] + tB_full[0] / tB_full[1]
    out = {"workload": "pmg-512^3-1440x768^2 view shares, FP32", "shares": k, "share_kernels": shares,
           "one_gpu_a_plus_at_ms": full_ms, "share_A_rows_identical": identical,
           "sum_of_share_At_rel_l2": err, "partial_volume_bytes": vol_bytes,
           "ring_allreduce_ms_model": allreduce_ms, "slowest_share_a_plus_at_ms": slowest,
           "k_gpu_a_plus_at_ms_model": slowest + allreduce_ms,
           "k_gpu_speedup_model": full_ms / (slowest + allreduce_ms)}
    print(json.dumps(out), flush=True)


def in_cone_fraction(views, nx, ny, nz, h, nu, nv, sub=4, chunk=8):
    """Fraction of (voxel, view) pairs whose voxel centre projects onto the
    detector (inside the outer pixel edges), on every sub-th voxel per axis,
    evaluated on the device.  views: (V, 12) rows s, d, u, v as the library
    takes them (pixel (a, b) centred at d + (a - (nu-1)/2) u + (b - (nv-1)/2) v)."""
    import torch
    dev = "cuda"
    ax = [(torch.arange(0, m, sub, device=dev, dtype=torch.float64) - (m - 1) / 2.0) * h for m in (nx, ny, nz)]
    X, Y, Z = torch.meshgrid(ax[0], ax[1], ax[2], indexing="ij")
    P = torch.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], 1)  # [n, 3]
    vw = torch.from_numpy(np.ascontiguousarray(views)).to(dev)
    inside = 0
    for v0 in range(0, len(views), chunk):
        w = vw[v0:v0 + chunk]
        s, d, u, v = w[:, 0:3], w[:, 3:6], w[:, 6:9], w[:, 9:12]
        nrm = torch.linalg.cross(u, v)
        r = P[None, :, :] - s[:, None, :]                                   # [c, n, 3]
        t = ((d - s) * nrm).sum(1)[:, None] / (r * nrm[:, None, :]).sum(2)  # ray parameter at the detector
        q = s[:, None, :] + t[..., None] * r - d[:, None, :]
        a = (q * u[:, None, :]).sum(2) / (u * u).sum(1)[:, None] + (nu - 1) / 2.0
        b = (q * v[:, None, :]).sum(2) / (v * v).sum(1)[:, None] + (nv - 1) / 2.0
        ok = (t > 0) & (a >= -0.5) & (a <= nu - 0.5) & (b >= -0.5) & (b <= nv - 0.5)
        inside += int(ok.sum())
    return inside / (P.shape[0] * len(views))


# multiply-adds per voxel of the learned preconditioner's four 3x3x3 layers
# (1 -> 16 -> 32 -> 32 -> 1 channels), two operations each
CNN_FLOPS_PER_VOXEL = 2 * 27 * (1 * 16 + 16 * 32 + 32 * 32 + 32 * 1)


def cnn_forward_timing(n, steps, warmup):
    """The network's forward pass alone on an n^3 grid (trained weights; a
    seeded random input), timed with HIP events on the library's stream,
    priced against the dense BF16 matrix-core peak."""
    import paper_2103_10329_amd as mg
    ctx = mg.Context(0)
    print(json.dumps({"cnn_forward": time_cnn_forward(ctx, n, steps, warmup)}), flush=True)
    ctx.close()


def time_cnn_forward(ctx, n, steps, warmup):
    import torch

    from paper_2103_10329_amd import learned as lrn
    ctx.cnn_set_weights(lrn.load_weights())
    gen = torch.Generator(device="cuda").manual_seed(3)
    u = torch.randn((n, n, n), device="cuda", generator=gen) * 1e-3
    out = torch.empty_like(u)
    for _ in range(max(warmup, 1)):
        ctx.cnn_forward(u, out=out)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        ctx.cnn_forward(u, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    tflops = CNN_FLOPS_PER_VOXEL * n ** 3 / (ms * 1e-3) / 1e12
    del u, out
    torch.cuda.empty_cache()
    return {"n": n, "ms": ms, "steps": steps, "tflops": tflops, "frac_bf16_dense_peak": tflops / 2500.0,
            "flops_per_voxel": CNN_FLOPS_PER_VOXEL}


def copy_calibration(size_mib=1024, reps=5):
    """A plain device copy of known size (for scaling the HBM byte counters)."""
    import torch
    x = torch.ones(size_mib << 18, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": size_mib << 20, "reps": reps}), flush=True)


def oracle_solves():
    """Whole solves of the FP64 oracle, as it stands, on all host threads,
    beside the library's on the same data (the library's step sizes for
    both): 20 SIRT iterations (eq. 2) on the 32^3 workload, and 2 iterations
    of Algorithm 1 (3 grids, radial filter, no regularisers) on the 128^3 one.
    Reports both wall times and the relative L2 difference of the results."""
    import torch

    import oracle
    import paper_2103_10329_amd as mg
    import synth
    out = {"cores": oracle.num_threads(), "cpu_model": _cpu_model()}
    for wl, kind in (("c0", "sirt"), ("c1", "pmg")):
        cfg = synth.CONFIGS[wl]
        n = cfg.n
        d = synth.make_dataset(wl, truth=False)
        ctx = mg.Context(0)
        ctx.set_geometry(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, d["views"])
        g = oracle.Geom(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, np.ascontiguousarray(d["views"]))
        b64 = np.asarray(d["b"], dtype=np.float64)
        b = torch.from_numpy(b64.astype(np.float32)).cuda()
        v = torch.zeros((n, n, n), device="cuda")
        if kind == "sirt":
            iters = 20
            alpha = ctx.estimate_step(None, level=0, iters=30, seed=0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(iters):
                ctx.landweber_step(v, b, alpha, None, want_norm=False)
            torch.cuda.synchronize()
            t_gpu = time.perf_counter() - t0
            x = np.zeros((n, n, n))
            t0 = time.perf_counter()
            for _ in range(iters):
                x, _ = oracle.landweber_step(g, x, b64, alpha, None)
            t_cpu = time.perf_counter() - t0
            what = "%d SIRT iterations" % iters
        else:
            levels = cfg.levels
            table = np.maximum(np.linspace(0, np.sqrt(3), 4097), 2.0 / n)
            filt = mg.filter_radial(table, np.sqrt(3))
            alphas = [ctx.estimate_step(filt, level=k, iters=30, seed=0) for k in range(levels - 1)]
            ctx.multigrid_solve(v, b, levels, 2, filt, alphas=alphas, want_hist=False)  # warm-up
            v.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.multigrid_solve(v, b, levels, 2, filt, alphas=alphas, want_hist=False)
            torch.cuda.synchronize()
            t_gpu = time.perf_counter() - t0
            t0 = time.perf_counter()
            x, _ = oracle.multigrid(g, np.zeros((n, n, n)), b64, levels, 2, oracle.filter_radial(table, np.sqrt(3)),
                                    alphas)
            t_cpu = time.perf_counter() - t0
            what = "2 iterations of Algorithm 1 on %d grids" % levels
        vh = v.double().cpu().numpy()
        out[wl] = {"solve": what, "oracle_s": t_cpu, "library_s": t_gpu, "ratio": t_cpu / t_gpu,
                   "rel_l2_difference": float(np.linalg.norm(vh - x) / np.linalg.norm(x))}
        ctx.close()
    print(json.dumps({"oracle_solves": out}), flush=True)


def cpu_baseline(cfg, views, n_sub=8):
    """The FP64 oracle, as it stands, on the host cores: one A and one A^T of
    the same workload's geometry restricted to n_sub of its views (evenly
    spaced), on a seeded random volume; the rate counts voxel*views of that
    sample.  A full solve at this size is impractical on the host."""
    import oracle
    n = cfg.n
    sub = np.ascontiguousarray(views[:: max(1, len(views) // n_sub)][:n_sub])
    g = oracle.Geom(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, sub)
    x = np.random.default_rng(0).random(g.vol_shape)
    t0 = time.perf_counter()
    p = oracle.project(g, x)
    t1 = time.perf_counter()
    oracle.backproject(g, p)
    t2 = time.perf_counter()
    t = t2 - t0
    # the same on one host thread, one view
    cores = oracle.num_threads()
    g1 = oracle.Geom(n, n, n, cfg.h, (0, 0, 0), cfg.nu, cfg.nv, np.ascontiguousarray(sub[:1]))
    oracle.set_num_threads(1)
    t3 = time.perf_counter()
    p1 = oracle.project(g1, x)
    oracle.backproject(g1, p1)
    t4 = time.perf_counter()
    oracle.set_num_threads(cores)
    one = {"value": n ** 3 / (t4 - t3) / 1e9, "seconds": t4 - t3, "threads": 1,
           "sample": "one A and one A^T of the FP64 oracle on 1 view (the first of the sample)"}
    return {"value": n ** 3 * len(sub) / t / 1e9, "unit": "Gvoxel·views/s", "cores": cores, "one_thread": one,
            "kind": "oracle", "seconds": t, "A_s": t1 - t0, "At_s": t2 - t1,
            "sample": "one A and one A^T of the FP64 oracle on %d of the %d views (evenly spaced) of the %d^3, "
                      "%dx%d-detector geometry, seeded random volume" % (len(sub), len(views), n, cfg.nv, cfg.nu),
            "nproc": os.cpu_count(), "cpu_model": _cpu_model()}


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


if __name__ == "__main__":
    main()
