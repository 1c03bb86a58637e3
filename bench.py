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
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sirt", action="store_true")
    ap.add_argument("--sirt-cap", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (scales the HBM byte counters)")
    ap.add_argument("--paper-shaped", action="store_true",
                    help="only run the 640x640x2304 / 3600 x 760^2 workload (prints its own JSON line)")
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

    import torch

    import paper_2103_10329_amd as mg
    import synth

    cfg = synth.CONFIGS[WORKLOAD]
    n, V, nu, nv = cfg.n, cfg.n_views, cfg.nu, cfg.nv
    t0 = time.time()
    d = synth.make_dataset(WORKLOAD, truth=not args.no_sirt)
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
    # inside the timed region only the fine grid's A and A^T launches are
    # bracketed by events (each event is a command on the stream)
    ctx.kernel_timing(True, ops=(mg.MGCT_OP_PROJECT, mg.MGCT_OP_BACKPROJECT), levels=(0,))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(vol)
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
    # every instrumented kernel on every grid, from two further steps after
    # the timed region; the fine grid's A and A^T keep their timed-region figures
    ctx.kernel_timing(True)
    for _ in range(2):
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
    t_dom = kt[dom]["ms_avg"] * 1e-3
    achieved = bytes_per_launch / t_dom / 1e9
    kname = "k_backproject_pl" if dom.startswith("back") else "k_project_sep"
    counters = measured_counters(kname)
    roofline = {"kernel": kname, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS,
                "traffic": counters["bytes_per_launch"] if counters else None,
                "valu_issue": counters["valu_issue"] if counters else None,
                "l2_hit": counters["l2_hit"] if counters else None,
                "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": kt[dom]["ms_avg"]}
    a_at = n ** 3 * V / ((tA + tB) * 1e-3) / 1e9
    # combined A + A^T rate on every grid (grid g: (n / 2^g)^3 voxels, same views)
    a_at_grid = {}
    for g in range(levels):
        ka, kb = kt.get("project@%d" % g), kt.get("backproject@%d" % g)
        if ka and kb:
            a_at_grid[str(g)] = (n >> g) ** 3 * V / ((ka["ms_avg"] + kb["ms_avg"]) * 1e-3) / 1e9

    out = {
        "metric": "A+A\u1d40 Gvoxel\u00b7views/s (% HBM roofline); time-to-residual vs plain SIRT",
        "value": value, "unit": "Gvoxel\u00b7views/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "pmg-128^3-360x192^2-L3-radial", "volume": [n, n, n], "views": V,
                   "detector": [nv, nu], "levels": levels, "filter": "radial ramp max(rho,2/N)",
                   "soft_threshold": lam, "bilateral": list(bil), "coarse": "OS-EMTR M=8 x2"},
        "roofline": roofline,
        "a_plus_at_kernels_gvox_views_s": a_at,
        "a_plus_at_hbm_frac": 2 * bytes_per_launch / ((tA + tB) * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "kernels_ms": kt,
        "a_plus_at_gvox_views_s_by_grid": a_at_grid,
        "step_size_estimate_s": t_alpha,
    }

    if not args.no_sirt:
        out.update(quality(ctx, mg, b, d, step, levels, filt, alphas, lam, bil, args))

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(d, views, alphas, lam, bil)
    print(json.dumps(out), flush=True)
    ctx.close()


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
    cfg = synth.CONFIGS[WORKLOAD]
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
    while k < args.sirt_cap:
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
    cap_os = min(args.sirt_cap, 200)
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
           "sirt_iterations": k if k < args.sirt_cap else None, "sirt_cap": args.sirt_cap,
           "sirt_s": t_sirt, "sirt_alpha": a_sirt,
           "speedup_vs_sirt": (t_sirt / t_pmg) if k < args.sirt_cap else None,
           "osemtr_iterations": reached[0] if reached else None, "osemtr_s": reached[1] if reached else None,
           "osemtr_cap": cap_os}
    log("time-to-residual", ttr)
    log("masked image error", errors)
    return {"time_to_residual": ttr, "image_error_masked": errors}


# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# passes, scaled by the same counters on a plain copy of known size, per
# launch, with its VALU issue fraction (SQ_INSTS_VALU per CU cycle) and L2 hit
# rate from the counter pass; valid only for the kernel source it was
# measured on.
TRAFFIC = {
    # profiles/backproject_project_128cube_360x192_counters.md
    "k_backproject_pl": {"source_sha256": "f23a0e9827bc880d5623e26b67b0ee4243ea940c2f3dfa25edbb20a1941cb161",
                          "bytes_per_launch": 407438624, "valu_issue": 0.86, "l2_hit": 0.958},
    "k_project_sep": {"source_sha256": "f23a0e9827bc880d5623e26b67b0ee4243ea940c2f3dfa25edbb20a1941cb161",
                       "bytes_per_launch": 7172105892, "valu_issue": 0.71, "l2_hit": 0.495},
}


def measured_counters(kernel):
    """The committed counter figures for `kernel`, or None when the source has
    changed since they were taken."""
    import hashlib
    t = TRAFFIC.get(kernel)
    if not t:
        return None
    src = os.path.join(ROOT, "paper_2103_10329_amd", "csrc", "joseph.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != t["source_sha256"]:
            return None
    return t


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
    out = {"workload": "paper-shaped 640x640x2304, 3600 views of 760^2, FP32", "voxel_views": nx * nx * nz * V}
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
    n4 = nx * nx * nz * V
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


def copy_calibration(size_mib=1024, reps=5):
    """A plain device copy of known size (for scaling the HBM byte counters)."""
    import torch
    x = torch.ones(size_mib << 18, device="cuda")
    y = torch.empty_like(x)
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_each_way": size_mib << 20, "reps": reps}), flush=True)


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
    out = {"value": n ** 3 * cfg.n_views / t / 1e9, "unit": "Gvoxel·views/s", "cores": oracle.num_threads(),
           "kind": "oracle", "seconds": t,
           "sample": "one full iteration of Algorithm 1 (3 grids, same 128^3 x 360-view data) by the FP64 oracle",
           "nproc": os.cpu_count(), "cpu_model": _cpu_model()}
    out["one_thread"] = _oracle_one_thread(views[::8], n, cfg.h, cfg.nu, cfg.nv)
    return out


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


# One A and one A^T of the FP64 oracle on a view subset, on one thread (the
# oracle reads its thread count at start-up, so this runs in a child process).
_ONE_THREAD = """
import sys, time
import numpy as np
import oracle
views = np.load(sys.argv[1])
n, h, nu, nv = int(sys.argv[2]), float(sys.argv[3]), int(sys.argv[4]), int(sys.argv[5])
g = oracle.Geom(n, n, n, h, (0, 0, 0), nu, nv, views)
x = np.random.default_rng(0).random(g.vol_shape)
t = time.perf_counter()
oracle.backproject(g, oracle.project(g, x))
print(oracle.num_threads(), time.perf_counter() - t)
"""


def _oracle_one_thread(views, n, h, nu, nv):
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        vf = os.path.join(tmp, "views.npy")
        np.save(vf, np.ascontiguousarray(views))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        try:
            r = subprocess.run([sys.executable, "-c", _ONE_THREAD, vf, str(n), str(h), str(nu), str(nv)],
                               env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
            threads, t = r.stdout.split()
        except (subprocess.SubprocessError, ValueError) as e:
            return {"error": str(e)[:200]}
    t = float(t)
    return {"value": n ** 3 * len(views) / t / 1e9, "unit": "Gvoxel·views/s", "threads": int(threads),
            "seconds": t, "sample": "one A and one A^T on %d of the %d views (every 8th), FP64 oracle" % (
                len(views), 8 * len(views))}


if __name__ == "__main__":
    main()
