"""Benchmark of the reconstruction hot path on one MI355X.

Headline workload: the largest single solve, 320 x 320 x 128 voxels,
3 species, 40 pulses, 512 samples per A-scan, 51 x 51 footprint, 50 inner
TV iterations, 300 outer iterations.  A step is one outer iteration of the
proximal-gradient solver, i.e. the whole per-iteration hot path: switching S,
acoustic contraction H with the residual, its adjoint with S^T, the gradient
step, the TV dual iteration, l1 + nonnegativity and the momentum update.
Each step applies A once and A^T once, so steps/s is the A + A^T apply rate
inside the solver.  Inputs are resident in HBM before the timed region
starts.  FISTA s-to-tol is the wall time of the whole 300-iteration solve,
power iteration from the seeded Gaussian start included.

Beside the headline: the other precisions on the same workload, the
128 x 128 x 64 workload (every precision, the separable, factorised and
two-step forms), isolated applies at 256 x 256 x 96, the 16 uneven problems
of the batched family, and the CPU leg (the FP64 oracle's time on a crop,
and every accuracy figure: sampled A-scans, and c_K against the oracle's
stored c_K on lateral crops of both geometries).

Prints one JSON line.  --gpus must be 1 (the path runs on one GPU).
"""
from __future__ import annotations

import argparse
import importlib.util
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A+Aᵀ applies/s & FISTA s-to-tol, BF16-MFMA vs FP32, at rel err ≤1e-3"
PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "bf16_split": 2500.0, "fp16_split": 2500.0,
               "bf16_refined": 2500.0, "fp32": 157.3}
ALL_PRECS = ("bf16", "bf16_refined", "fp16", "bf16_split", "fp16_split", "fp32")
# golden c_K crops of the oracle (tests/golden), per workload
GOLDEN_CASE = {"C5": "C5_crop16_k2_50", "C2": "C2_crop24_k2_20"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="C5", choices=["C5", "C2"],
                    help="headline workload: C5 = 320x320x128 (default), C2 = 128x128x64")
    ap.add_argument("--prec", default="bf16")
    ap.add_argument("--compare", default="fp16,bf16_split,fp32",
                    help="other precisions timed on the headline workload ('' = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="headline plan with the built-in launch-shape rules instead of the autotuner")
    ap.add_argument("--no-c1-oracle", action="store_true",
                    help="skip the FP64 oracle solve at 32x32x16 used for each precision's c error")
    ap.add_argument("--cpu-crop", type=int, default=0,
                    help="lateral crop side of the oracle timing sample (0: 12 at the largest "
                         "workload, 20 at 128x128x64)")
    ap.add_argument("--kernel-reps", type=int, default=0, help="0: by workload")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the 128x128x64 block (with the separable, factorised and "
                         "two-step forms)")
    ap.add_argument("--no-scales", action="store_true",
                    help="skip the 256x256x96 applies and the 16-problem batch")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline plan and precision: every band-kernel launch of a "
                         "profiled run then belongs to it")
    return ap.parse_args(argv)


def time_events(torch, fn, reps):
    """Average ms of fn() over reps launches, HIP events on the current stream
    (the stream the library's kernels are launched on)."""
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(reps):
        fn()
    e1.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tv_bandwidth(torch, pk, plan, cfg, z_host):
    """The TV prox's dual step (HBM-bound): per-step time from two prox_tv
    calls of K2 and K2/5 dual steps on the same input (the difference holds
    only dual steps, not the prox's set-up and final kernels), its
    algorithmic bytes (40 per species-voxel: u_j, u_{j-1}, z in, u_{j+1} out)
    per second, against a plain 1 GiB device copy timed in the same process
    and against the 8 TB/s HBM figure."""
    z = torch.from_numpy(z_host).cuda()
    x = torch.empty_like(z)
    nws = int(pk.load().psoam_prox_tv_ws_bytes(plan.handle)) // 4 + 64
    ws = torch.empty(nws, dtype=torch.float32, device="cuda")
    k_hi, k_lo = cfg.k2, max(1, cfg.k2 // 5)
    t_hi = time_events(torch, lambda: plan.prox_tv(z, 0.01, k_hi, x=x, ws=ws), 3)
    t_lo = time_events(torch, lambda: plan.prox_tv(z, 0.01, k_lo, x=x, ws=ws), 3)
    step_ms = (t_hi - t_lo) / (k_hi - k_lo)
    del z, x, ws
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    copy_ms = time_events(torch, lambda: b.copy_(a), 5)
    del a, b
    torch.cuda.empty_cache()
    alg = 40.0 * cfg.n_species * cfg.nx * cfg.ny * cfg.nz
    gbps = alg / (step_ms * 1e-3) / 1e9
    copy_gbps = 2.0 * 4 * n / (copy_ms * 1e-3) / 1e9
    return {"dual_step_ms": step_ms, "alg_bytes_per_step": alg, "achieved_GBps": gbps,
            "copy_GBps_measured": copy_gbps, "frac_of_copy": gbps / copy_gbps,
            "frac_of_8TBps": gbps / 8000.0,
            "method": f"(t(prox_tv, K2={k_hi}) - t(prox_tv, K2={k_lo})) / {k_hi - k_lo}, "
                      "HIP events; copy: 1 GiB torch copy_, read + write bytes"}


def alg_flops(cfg, t0, taps):
    """Algorithmic flops of one H (or H^T) apply: 2 K times the number of
    (scan, voxel, sample) triples with a nonzero band entry whose voxel lies in
    the grid and whose sample lies in the A-scan, i.e. for each lateral offset
    its band nonzeros times the scans whose voxel at that offset exists."""
    nz, f, _ = t0.shape
    r = (f - 1) // 2
    t = t0[..., None].astype(np.int64) + np.arange(taps.shape[-1])
    nnz = ((taps != 0) & (t >= 0) & (t < cfg.nt)).sum(axis=(0, 3)).astype(np.float64)   # [F][F]
    d = np.arange(-r, r + 1)
    ry = np.maximum(cfg.ny - np.abs(d), 0).astype(np.float64)
    rx = np.maximum(cfg.nx - np.abs(d), 0).astype(np.float64)
    return 2.0 * cfg.n_pulses * float((nnz * ry[:, None] * rx[None, :]).sum())


def golden_module():
    """The committed script that wrote the oracle's c_K crops (its
    measurements() rebuilds the crop's p with the oracle)."""
    path = os.path.join(ROOT, "tests", "golden", "make_cK_golden.py")
    spec = importlib.util.spec_from_file_location("make_cK_golden", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def headline_inputs(torch, pk, cfg, synth):
    """Seeded synthetic inputs of the workload, resident in HBM: the tube
    phantom, measurements p = A c_true (FP32 path) plus 20 dB Gaussian noise
    drawn on the device from a seeded generator (timing input only; accuracy
    is checked on the oracle's own crops), and the power-iteration start."""
    g_ph, _, _, g_pow = synth.streams(cfg.seed)
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species, cfg.gamma)
    c_true = synth.phantom(cfg, g_ph)
    v0 = synth.power_start(int(np.prod(cfg.c_shape)), g_pow).reshape(cfg.c_shape)
    ref = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec="fp32")
    y_clean = ref.apply_A(torch.from_numpy(c_true).cuda())
    rms = float(torch.sqrt((y_clean.double() ** 2).mean()))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(cfg.seed + 1)
    p_t = y_clean.add_(torch.randn(cfg.y_shape, generator=gen, device="cuda", dtype=torch.float32),
                       alpha=synth.noise_sigma(rms)).contiguous()
    aty_inf = float(ref.apply_AT(p_t).abs().max())
    ref.close()
    torch.cuda.empty_cache()
    return t0, taps, phi, sp, c_true, v0, p_t, aty_inf


def run_prec(torch, pk, cfg, t0, taps, phi, sp, c_true, p_t, alpha1, lam_tv, lam_l1, prec,
             steps, warmup, reps, separable=False, full_solve=False, v0=None, tvs=False,
             tune=False, paper_stop=False):
    """Times one precision on one workload: optionally the full K1-iteration
    solve with its power iteration (first; alpha1 <= 0 takes the step from it),
    isolated applies, the band kernels alone (HIP events), `steps` solver
    steps after `warmup`, optionally the steps with the TV(S c) term.  tune:
    the plan's launch shapes chosen by the autotuner (its report kept).
    paper_stop: the full solve again with the stopping thresholds of the
    paper's experiments (eps1 1e-8, eps2 1e-4, K1 as the cap), tested on the
    device."""
    t_plan = time.perf_counter()
    plan = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=prec, separable=separable, tune=tune)
    info = plan.stats()
    out = dict(plan=plan, info=info)
    if tune:
        out["autotune"] = dict(plan.tune_report, seconds=time.perf_counter() - t_plan)
    c_full = None
    if full_solve:
        c_full = torch.zeros(cfg.c_shape, dtype=torch.float32, device="cuda")
        v0_t = torch.from_numpy(v0).cuda() if v0 is not None else None
        # an untimed solve of two iterations warms the kernels
        plan.solve(p_t, c=c_full, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=2, k2=cfg.k2,
                   alpha1=0.0, n_power=2, v0=v0_t)
        c_full.zero_()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, st_full = plan.solve(p_t, c=c_full, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=cfg.k1,
                                k2=cfg.k2, alpha1=0.0, n_power=30, v0=v0_t)
        torch.cuda.synchronize()
        out["solve_s"] = time.perf_counter() - t1
        out["lambda_max"] = st_full["lambda_max"]
        if paper_stop:
            c_tol = torch.zeros(cfg.c_shape, dtype=torch.float32, device="cuda")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            _, st_tol = plan.solve(p_t, c=c_tol, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=cfg.k1,
                                   k2=cfg.k2, alpha1=0.0, n_power=30, v0=v0_t, eps1=1e-8,
                                   eps2=1e-4, device_stop=True)
            torch.cuda.synchronize()
            out["solve_tol"] = {"eps1": 1e-8, "eps2": 1e-4, "k1_cap": cfg.k1,
                                "iterations": st_tol["iterations"],
                                "seconds": time.perf_counter() - t1,
                                "stopping_tests": "on the device (device_stop)"}
            del c_tol
        if alpha1 <= 0.0:
            alpha1 = st_full["alpha1"]
    out["alpha1"] = alpha1
    out["c_full"] = c_full
    c_in = torch.from_numpy(c_true).cuda()
    y = torch.empty(cfg.y_shape, dtype=torch.float32, device="cuda")
    g = torch.empty(cfg.c_shape, dtype=torch.float32, device="cuda")
    out["y"] = y
    out["t_A"] = time_events(torch, lambda: plan.apply_A(c_in, y), reps)
    out["t_AT"] = time_events(torch, lambda: plan.apply_AT(y, g), reps)
    # band kernels alone (operands left by the applies above)
    plan.apply_A(c_in, y)
    out["t_H"] = time_events(torch, lambda: plan.band_only(0, y), reps)
    plan.apply_AT(y, g)
    out["t_HT"] = time_events(torch, lambda: plan.band_only(1, g), reps)
    del g, c_in
    # solver steps: warmup, then exactly `steps` timed outer iterations
    c = torch.zeros(cfg.c_shape, dtype=torch.float32, device="cuda")
    if warmup > 0:
        plan.solve(p_t, c=c, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=warmup, k2=cfg.k2,
                   alpha1=alpha1)
        c.zero_()
    torch.cuda.synchronize()
    t0_ = time.perf_counter()
    _, st = plan.solve(p_t, c=c, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=steps, k2=cfg.k2,
                       alpha1=alpha1)
    torch.cuda.synchronize()
    out["step_s"] = (time.perf_counter() - t0_) / steps
    assert st["iterations"] == steps
    if tvs:
        # the same steps with the full regulariser's TV(S c) term (stacked dual prox)
        c.zero_()
        n = max(2, steps // 4)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        plan.solve(p_t, c=c, lambda_tv=lam_tv, lambda_l1=lam_l1, lambda_tvs=0.4 * lam_tv,
                   k1=n, k2=cfg.k2, alpha1=alpha1)
        torch.cuda.synchronize()
        out["step_tvs_s"] = (time.perf_counter() - t2) / n
    del c
    return out


def factorised_run(torch, pk, cfg, phi, sp, c_true, p_t, lam_tv, lam_l1, prec, steps, warmup,
                   reps, scans):
    """The paper's factorised acoustic operator on the same workload: shell
    sums Lambda on the matrix cores (a narrow band), then the impulse-response
    pass over the A-scans.  Times the isolated applies, the shell-sum kernels
    alone and solver steps (step size from its own power iteration), and
    keeps sampled A-scans for the CPU leg's comparison with the oracle."""
    import synth
    dr, z_focus, t_focus = synth.shell_geometry(cfg.nz, cfg.nt)
    eir, origin = synth.eir_taps()
    spr = synth.spr_table(cfg.nz, cfg.f)
    plan = pk.Plan.factorised(cfg.nx, cfg.ny, cfg.nz, cfg.n_pulses, cfg.nt, cfg.f, phi, sp, spr,
                              eir, origin, dr, z_focus, t_focus, prec=prec)
    info = plan.stats()
    c_in = torch.from_numpy(c_true).cuda()
    y = torch.empty(cfg.y_shape, dtype=torch.float32, device="cuda")
    g = torch.empty(cfg.c_shape, dtype=torch.float32, device="cuda")
    t_A = time_events(torch, lambda: plan.apply_A(c_in, y), reps)
    t_AT = time_events(torch, lambda: plan.apply_AT(y, g), reps)
    plan.apply_A(c_in, y)
    t_L = time_events(torch, lambda: plan.band_only(0, y), reps)
    plan.apply_AT(y, g)
    t_LT = time_events(torch, lambda: plan.band_only(1, g), reps)
    c = torch.zeros(cfg.c_shape, dtype=torch.float32, device="cuda")
    _, st = plan.solve(p_t, c=c, k1=0, n_power=30)
    alpha1 = st["alpha1"]
    plan.solve(p_t, c=c, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=warmup, k2=cfg.k2, alpha1=alpha1)
    c.zero_()
    torch.cuda.synchronize()
    t0_ = time.perf_counter()
    plan.solve(p_t, c=c, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=steps, k2=cfg.k2, alpha1=alpha1)
    torch.cuda.synchronize()
    step = (time.perf_counter() - t0_) / steps
    plan.apply_A(c_in, y)
    y_g = np.stack([y[:, iy, ix, :].cpu().numpy() for (iy, ix) in scans])
    alg_macs = int(info["useful_macs"][0]) + len(eir) * cfg.nt   # per A-scan of one pulse: shells + EIR
    out = {"dtype": prec, "ms_per_step": step * 1e3, "applies_per_s_in_solver": 1.0 / step,
           "apply_A_ms": t_A, "apply_AT_ms": t_AT, "isolated_applies_per_s": 1e3 / (t_A + t_AT),
           "shell_kernel_ms": t_L, "shell_adjoint_kernel_ms": t_LT,
           "shell_nonzeros_per_ascan": info["useful_macs"][0],
           "chunks": info["chunks"], "band_fill": info["useful_macs"][0] / max(1, info["executed_macs"][0]),
           "alg_macs_per_ascan": alg_macs,
           "rel_err_A_vs_oracle_sampled": None,
           "note": "a different discretisation of the acoustic model (unit-weight shells "
                   "then the 1D pulse convolution), not the banded impulse response: its "
                   "timings are a comparison point, not the headline"}
    plan.close()
    sample = dict(y=y_g, spr=spr, eir=eir, origin=origin, dr=dr, z_focus=z_focus, t_focus=t_focus)
    return out, sample


def profiled_traffic(name):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary profiles/<name>, valid only while the kernel and plan sources hash
    to what was profiled."""
    import hashlib
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None, "no counter summary"
    want = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            want[k.strip()] = v.strip().strip("`")
    h = hashlib.sha1()
    for f in ("psoam_kernels.hip", "psoam_plan.cpp", "psoam_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2510_23739_amd", "csrc", f), "rb").read())
    if want.get("source_sha1") != h.hexdigest():
        return None, "kernel sources changed since the counters were taken"
    try:
        return float(want["hbm_bytes_per_launch"]), os.path.relpath(path, ROOT)
    except (KeyError, ValueError):
        return None, "summary without hbm_bytes_per_launch"


def scale_runs(torch, pk):
    """Isolated A / A^T applies at 256x256x96 (BF16, FP16, BF16 split, FP32),
    and the 16 uneven problems of the batched family (BF16, 100 outer
    iterations each) solved as one batch vs one after another.  Timing inputs
    are seeded uniform values (operator cost does not depend on values;
    parity at these sizes is in the GPU tests)."""
    import synth
    out = {}
    cfg = synth.C3
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species)
    c = torch.from_numpy(np.random.default_rng(cfg.seed).random(cfg.c_shape, dtype=np.float32)).cuda()
    y = torch.empty(cfg.y_shape, dtype=torch.float32, device="cuda")
    g = torch.empty(cfg.c_shape, dtype=torch.float32, device="cuda")
    rows = {}
    flops = alg_flops(cfg, t0, taps)
    for prec in ("bf16", "fp16", "bf16_split", "fp32"):
        log(f"[bench] {cfg.name} {prec}")
        plan = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=prec)
        info = plan.stats()
        reps = 2 if prec == "fp32" else 5
        t_A = time_events(torch, lambda: plan.apply_A(c, y), reps)
        t_AT = time_events(torch, lambda: plan.apply_AT(y, g), reps)
        plan.apply_A(c, y)
        t_H = time_events(torch, lambda: plan.band_only(0, y), reps)
        rows[prec] = {"apply_A_ms": t_A, "apply_AT_ms": t_AT,
                      "isolated_applies_per_s": 1e3 / (t_A + t_AT), "H_kernel_ms": t_H,
                      "H_alg_frac_of_peak": flops / (t_H * 1e-3) / 1e12 / PEAK_TFLOPS[prec],
                      "staged_rows": info["lds_rows"]}
        plan.close()
        torch.cuda.empty_cache()
    out[f"{cfg.nx}x{cfg.ny}x{cfg.nz} S{cfg.n_species} K{cfg.n_pulses} Nt{cfg.nt} F{cfg.f}"] = rows
    del c, y, g
    torch.cuda.empty_cache()
    # batched family: 16 instances, BF16, 100 outer iterations each (K2 20),
    # step from a 10-step power iteration, batch vs one-by-one; every plan's
    # launch shapes chosen by the autotuner (before the timed region)
    log("[bench] batched family")
    plans, ps, opts, choices = [], [], [], []
    t_tune = time.perf_counter()
    for i in range(16):
        cfg = synth.c4_instance(i)
        t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
        plan = pk.Plan.from_config(cfg, synth.phi_depth(cfg.nz), synth.species(cfg.n_species), t0,
                                   taps, prec="bf16", tune=True)
        r = plan.tune_report
        choices.append([r["h_rows"], r["ht_rows"], r["ht_shift"], r["h_loaders"],
                        "x".join(str(v) for v in r["tv_tile"])])
        rng = np.random.default_rng(cfg.seed)
        ps.append(torch.from_numpy(rng.standard_normal(cfg.y_shape, dtype=np.float32)).cuda())
        plans.append(plan)
        opts.append(dict(lambda_tv=1e-3, lambda_l1=1e-3, k1=cfg.k1, k2=20, n_power=10))
    t_tune = time.perf_counter() - t_tune
    cs = [torch.zeros(pl.c_shape, dtype=torch.float32, device="cuda") for pl in plans]
    pk.solve_batch(plans, ps, cs, [dict(o, k1=2) for o in opts])   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    pk.solve_batch(plans, ps, cs, opts)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t
    t = time.perf_counter()
    for pl, p_, c_, o in zip(plans, ps, cs, opts):
        c_.zero_()
        pl.solve(p_, c=c_, lambda_tv=o["lambda_tv"], lambda_l1=o["lambda_l1"], k1=o["k1"], k2=o["k2"],
                 n_power=o["n_power"])
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t
    out[f"batched_16_uneven_bf16_k1_{opts[0]['k1']}"] = {
        "batch_s": t_batch, "one_by_one_s": t_seq, "speedup": t_seq / t_batch,
        "autotuned_plans": {"seconds": t_tune,
                            "choice_per_instance": "H rows, H^T rows, H^T shift, H loaders, TV tile",
                            "choices": choices}}
    for pl in plans:
        pl.close()
    return out


def cpu_baseline(cfg, t0, taps, phi, sp, crop):
    """The oracle, as it stands, timed on the host for one solver step (A,
    A^T, TV prox with K2 inner steps, l1, momentum) on a crop x crop lateral
    sample of the workload's geometry, scaled by the number of (scan, offset)
    pairs evaluated, which is what the oracle's time follows."""
    import oracle
    import synth
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    sub = cfg.crop(crop, crop)
    c = synth.phantom(sub).astype(np.float64)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, cfg.n_pulses)
    p = np.random.default_rng(0).standard_normal(sub.y_shape)
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    t = time.perf_counter()
    oracle.fista(p, A, AT, 1e-3, 1e-3, 1e-3, 1, cfg.k2, c_init=c)
    dt = time.perf_counter() - t

    def pairs(n):
        # (scan, offset) pairs with the voxel inside an n-wide grid, per axis
        return sum(max(0, n - abs(d)) for d in range(-cfg.r, cfg.r + 1))
    scale = (pairs(cfg.nx) * pairs(cfg.ny)) / float(pairs(crop) ** 2)
    step_s = dt * scale
    return {"value": 1.0 / step_s, "unit": "A+AT applies/s", "cores": int(cores), "kind": "oracle",
            "sample": (f"one FP64 oracle solver step (A, A^T, TV prox K2={cfg.k2}, l1, momentum) on "
                       f"a {crop}x{crop}-scan lateral crop (full Nz {cfg.nz}, K {cfg.n_pulses}, "
                       f"Nt {cfg.nt}, F {cfg.f}), {dt:.1f} s, scaled x{scale:.0f} by the number "
                       f"of (scan, offset) pairs to {cfg.nx}x{cfg.ny} scans (extrapolated)")}


def golden_errors(torch, pk, case, precs):
    """c_K of each precision's GPU solve on the oracle's stored crop (same
    measurements, rebuilt by the oracle; the stored alpha1 and weights)
    against the oracle's c_K: (normwise rel err, max-abs rel err) per precision."""
    import oracle
    mk = golden_module()
    meta = json.load(open(mk.JSON))[case]
    cfg, _, _ = mk.case_config(case)
    p, S, t0, taps, phi, sp, v0, c_true = mk.measurements(cfg)
    ref = np.load(os.path.join(ROOT, "tests", "golden", f"cK_{case}.npy"))
    out = {}
    for q in precs:
        plan = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=q)
        c, st = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=meta["lambda_tv"],
                           lambda_l1=meta["lambda_l1"], k1=meta["k1"], k2=meta["k2"],
                           alpha1=meta["alpha1"])
        got = c.cpu().numpy()
        out[q] = (oracle.rel_err(got, ref), float(np.abs(got - ref).max() / np.abs(ref).max()))
        plan.close()
    return out, meta


def c1_errors(torch, pk, precs):
    """Each precision's GPU solve of the 32x32x16 problem against the oracle's
    FISTA, on measurements and a step that the oracle itself produced."""
    import oracle
    import synth
    c1 = synth.C1
    c1_true, t01, taps1, phi1, sp1, n0, v0 = synth.inputs(c1)
    S1 = oracle.switching_matrix(np.asarray(phi1, np.float64), sp1.a, sp1.b, sp1.tau,
                                 sp1.gamma, c1.n_pulses)
    A1 = lambda v: oracle.apply_A(v, S1, t01, taps1, c1.nt)
    AT1 = lambda w: oracle.apply_AT(w, S1, t01, taps1, c1.nz)
    y1 = A1(c1_true.astype(np.float64))
    p1 = (y1 + synth.noise_sigma(float(np.sqrt(np.mean(y1 ** 2)))) * n0).astype(np.float32)
    aty = float(np.abs(AT1(p1.astype(np.float64))).max())
    lam_tv, lam_l1 = 5e-3 * aty, 1e-2 * aty
    alpha1 = 1.0 / (1.01 * oracle.power_iteration(A1, AT1, v0, 30))
    c_ref, _ = oracle.fista(p1.astype(np.float64), A1, AT1, alpha1, lam_tv, lam_l1, c1.k1,
                            c1.k2, shape_c=c1.c_shape)
    out = {}
    for q in precs:
        plan = pk.Plan.from_config(c1, phi1, sp1, t01, taps1, prec=q)
        cg, _ = plan.solve(torch.from_numpy(p1).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1,
                           k1=c1.k1, k2=c1.k2, alpha1=alpha1)
        out[q] = oracle.rel_err(cg.cpu().numpy(), c_ref)
        plan.close()
    return out


def sampled_A_errors(cfg, t0, taps, phi, sp, c_true, samples, scans):
    """A-scans the GPU legs kept, against the oracle's at the same positions."""
    import oracle
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, cfg.n_pulses)
    y_s = oracle.apply_A_scans(c_true, S, t0, taps, cfg.nt, scans)
    return {q: oracle.rel_err(y_g, y_s) for q, y_g in samples.items()}, S


def per_prec_rows(runs, flops, cfg):
    """The JSON rows of the precisions timed on one workload."""
    fp32 = runs.get("fp32")
    rows = {}
    for q, r in runs.items():
        t_pow = 30 * (r["t_A"] + r["t_AT"]) * 1e-3
        rows[q] = {
            "ms_per_step": r["step_s"] * 1e3, "applies_per_s_in_solver": 1.0 / r["step_s"],
            "apply_A_ms": r["t_A"], "apply_AT_ms": r["t_AT"],
            "isolated_applies_per_s": 1e3 / (r["t_A"] + r["t_AT"]),
            "H_kernel_ms": r["t_H"], "HT_kernel_ms": r["t_HT"],
            "H_alg_frac_of_peak": flops / (r["t_H"] * 1e-3) / 1e12 / PEAK_TFLOPS[q],
            "HT_alg_frac_of_peak": flops / (r["t_HT"] * 1e-3) / 1e12 / PEAK_TFLOPS[q],
            "fista_iterations": cfg.k1,
        }
        if "solve_s" in r:
            rows[q]["fista_s_to_tol"] = r["solve_s"]
        else:
            # 30 power steps at the isolated apply rate, then K1 solver steps
            rows[q]["fista_s_to_tol_extrapolated"] = t_pow + cfg.k1 * r["step_s"]
        if "step_tvs_s" in r:
            rows[q]["ms_per_step_with_tv_of_Sc"] = r["step_tvs_s"] * 1e3
        if fp32 is not None and r is not fp32 and r.get("c_full") is not None \
                and fp32.get("c_full") is not None:
            rows[q]["rel_err_c_vs_fp32"] = float((r["c_full"] - fp32["c_full"]).double().norm()
                                                 / fp32["c_full"].double().norm())
    return rows


def secondary_block(torch, pk, synth, args, prec):
    """The 128 x 128 x 64 workload (S 3, K 32, Nt 256, F 31, K2 20, K1 100):
    every precision's solver step, the full solve for the headline precision
    and FP32, the TV(S c) term, the autotuner, and the separable, two-step and
    factorised forms.  Returns (block dict, what the CPU leg compares)."""
    cfg = synth.C2
    log(f"[bench] secondary workload {cfg.name}")
    t0, taps, phi, sp, c_true, v0, p_t, aty_inf = headline_inputs(torch, pk, cfg, synth)
    lam_tv, lam_l1 = 5e-3 * aty_inf, 1e-2 * aty_inf
    reps = 10
    runs = {prec: run_prec(torch, pk, cfg, t0, taps, phi, sp, c_true, p_t, 0.0, lam_tv, lam_l1,
                           prec, args.steps, args.warmup, reps, full_solve=True, v0=v0, tvs=True)}
    alpha1 = runs[prec]["alpha1"]
    for q in ALL_PRECS:
        if q == prec:
            continue
        log(f"[bench] {cfg.name} {q}")
        slow = q == "fp32"
        runs[q] = run_prec(torch, pk, cfg, t0, taps, phi, sp, c_true, p_t, alpha1, lam_tv, lam_l1,
                           q, max(2, args.steps // 4) if slow else args.steps,
                           1 if slow else args.warmup, 3 if slow else reps, full_solve=slow, v0=v0)
    flops = alg_flops(cfg, t0, taps)
    scans = [(5, 7), (64, 64), (127, 0), (90, 33)]
    c_in = torch.from_numpy(c_true).cuda()
    samples = {}
    for q, r in runs.items():
        r["plan"].apply_A(c_in, r["y"])
        samples[q] = np.stack([r["y"][:, iy, ix, :].cpu().numpy() for (iy, ix) in scans])
    block = {"workload": "128x128x64 voxels, 3 species, 32 pulses, Nt 256, footprint 31x31, K2 20, "
                         "K1 100",
             "alg_gflop_per_H": flops / 1e9,
             "band_fill": runs[prec]["info"]["useful_macs"][0]
             / max(1, runs[prec]["info"]["executed_macs"][0]),
             "precisions": per_prec_rows(runs, flops, cfg)}
    # the separable fast form (valid only for the fluence-independent rate,
    # gamma = 0), reported apart from the general path
    if sp.gamma == 0.0:
        log(f"[bench] separable form {prec}")
        rs = run_prec(torch, pk, cfg, t0, taps, phi, sp, c_true, p_t, alpha1, lam_tv, lam_l1,
                      prec, args.steps, args.warmup, reps, separable=True, full_solve=True, v0=v0)
        rs["plan"].apply_A(c_in, rs["y"])
        samples["separable"] = np.stack([rs["y"][:, iy, ix, :].cpu().numpy() for (iy, ix) in scans])
        ref = runs["fp32"]["c_full"]
        block["separable_form"] = {
            "dtype": prec, "ms_per_step": rs["step_s"] * 1e3,
            "applies_per_s_in_solver": 1.0 / rs["step_s"],
            "apply_A_ms": rs["t_A"], "apply_AT_ms": rs["t_AT"],
            "isolated_applies_per_s": 1e3 / (rs["t_A"] + rs["t_AT"]),
            "contraction_H_ms": rs["t_H"], "contraction_HT_ms": rs["t_HT"],
            "fista_s_to_tol": rs["solve_s"],
            "rel_err_A_vs_oracle_sampled": None,
            "rel_err_c_vs_fp32_general": float((rs["c_full"] - ref).double().norm()
                                               / ref.double().norm()),
            "note": "S_v[k][s] = phi_v T[k][s] (gamma = 0): the contraction runs over the "
                    "S species (one 16-column block) and the pulses are expanded after; "
                    "not valid for the fluence-dependent rate"}
        rs["plan"].close()
    # the launch-shape autotuner on this workload (its choice and the kernel
    # times it measured)
    log(f"[bench] autotune {prec}")
    t_tune = time.perf_counter()
    tp = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=prec, tune=True)
    block["autotune"] = dict(tp.tune_report, seconds=time.perf_counter() - t_tune)
    tp.close()
    # the two-step method (the paper's comparison): acoustic inversion of the
    # K pulse volumes with TV, then per-voxel unmixing with l1 + TV
    log("[bench] two-step method")
    ac = pk.Plan.acoustic(cfg.nx, cfg.ny, cfg.nz, cfg.n_pulses, cfg.nt, cfg.f, t0, taps, prec=prec)
    b = torch.zeros(ac.c_shape, dtype=torch.float32, device="cuda")
    _, st_a = ac.solve(p_t, c=b, k1=0, n_power=30)          # step from H's power iteration
    n_ts = max(2, args.steps // 4)
    ac.solve(p_t, c=b, lambda_tv=lam_tv, k1=1, k2=cfg.k2, alpha1=st_a["alpha1"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    ac.solve(p_t, c=b, lambda_tv=lam_tv, k1=n_ts, k2=cfg.k2, alpha1=st_a["alpha1"])
    torch.cuda.synchronize()
    t_ac = (time.perf_counter() - t) / n_ts
    sp_plan = runs[prec]["plan"]
    c_u = torch.zeros(cfg.c_shape, dtype=torch.float32, device="cuda")
    _, st_u = sp_plan.unmix(b, c=c_u, k1=0, n_power=30)     # step from S's power iteration
    sp_plan.unmix(b, c=c_u, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=1, k2=cfg.k2,
                  alpha1=st_u["alpha1"])
    torch.cuda.synchronize()
    t = time.perf_counter()
    sp_plan.unmix(b, c=c_u, lambda_tv=lam_tv, lambda_l1=lam_l1, k1=n_ts, k2=cfg.k2,
                  alpha1=st_u["alpha1"])
    torch.cuda.synchronize()
    t_un = (time.perf_counter() - t) / n_ts
    block["two_step"] = {"dtype": prec, "acoustic_ms_per_iteration": t_ac * 1e3,
                         "unmix_ms_per_iteration": t_un * 1e3,
                         "note": f"per outer iteration (K2 {cfg.k2}); the acoustic step carries "
                                 f"TV on all {cfg.n_pulses} pulse volumes"}
    ac.close()
    del b, c_u
    log("[bench] factorised acoustic operator")
    block["factorised"], fact = factorised_run(torch, pk, cfg, phi, sp, c_true, p_t, lam_tv,
                                               lam_l1, prec, args.steps, args.warmup, reps, scans)
    for r in runs.values():
        r["plan"].close()
    del runs, p_t
    torch.cuda.empty_cache()
    return block, dict(cfg=cfg, t0=t0, taps=taps, phi=phi, sp=sp, c_true=c_true,
                       samples=samples, scans=scans, fact=fact)


def secondary_accuracy(torch, pk, blk, s, with_c1):
    """The CPU leg's accuracy figures of the 128 x 128 x 64 block."""
    import oracle
    gen = {q: v for q, v in s["samples"].items() if q != "separable"}
    errs, S2 = sampled_A_errors(s["cfg"], s["t0"], s["taps"], s["phi"], s["sp"], s["c_true"], gen,
                                s["scans"])
    for q, e in errs.items():
        blk["precisions"][q]["rel_err_A_vs_oracle_sampled"] = e
    if "separable" in s["samples"] and "separable_form" in blk:
        y_s = oracle.apply_A_scans(s["c_true"], S2, s["t0"], s["taps"], s["cfg"].nt, s["scans"])
        blk["separable_form"]["rel_err_A_vs_oracle_sampled"] = oracle.rel_err(
            s["samples"]["separable"], y_s)
    f = s["fact"]
    mask = oracle.shell_mask(s["cfg"].nz, s["cfg"].f, s["cfg"].nt, f["dr"], f["z_focus"],
                             f["t_focus"])
    y_f = oracle.apply_A_fact_scans(s["c_true"], S2, f["spr"], mask, f["eir"], f["origin"],
                                    s["scans"])
    blk["factorised"]["rel_err_A_vs_oracle_sampled"] = oracle.rel_err(f["y"], y_f)
    gerr, _ = golden_errors(torch, pk, GOLDEN_CASE["C2"], list(blk["precisions"]))
    for q, (e, em) in gerr.items():
        blk["precisions"][q]["rel_err_c_vs_oracle_crop"] = e
        blk["precisions"][q]["max_abs_err_c_vs_oracle_crop"] = em
    if with_c1:
        for q, e in c1_errors(torch, pk, list(blk["precisions"])).items():
            blk["precisions"][q]["rel_err_c_vs_oracle_32x32x16"] = e


def main(argv=None):
    args = parse(argv)
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; --gpus must be 1 "
                          "(sharding the path across GPUs is not built)"}))
        sys.exit(2)
    import torch

    import paper_2510_23739_amd as pk
    import synth

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    pk.load()
    cfg = synth.CONFIGS[args.workload]
    big = args.workload == "C5"
    reps = args.kernel_reps or (5 if big else 10)
    log(f"[bench] inputs for {cfg.name}")
    t0, taps, phi, sp, c_true, v0, p_t, aty_inf = headline_inputs(torch, pk, cfg, synth)
    lam_tv, lam_l1 = 5e-3 * aty_inf, 1e-2 * aty_inf
    log(f"[bench] {cfg.name} {args.prec}: full solve, applies, kernels, steps")
    res = run_prec(torch, pk, cfg, t0, taps, phi, sp, c_true, p_t, 0.0, lam_tv, lam_l1, args.prec,
                   args.steps, args.warmup, reps, full_solve=True, v0=v0, tvs=not big,
                   tune=not args.no_tune, paper_stop=True)
    alpha1 = res["alpha1"]
    tvb = tv_bandwidth(torch, pk, res["plan"], cfg, c_true)
    runs = {args.prec: res}
    others = [] if args.headline_only else [q for q in args.compare.split(",") if q and q != args.prec]
    for q in others:
        log(f"[bench] {cfg.name} {q}")
        slow = q == "fp32"
        split = "split" in q
        n = 2 if slow else (max(2, args.steps // 4) if split else args.steps)
        runs[q] = run_prec(torch, pk, cfg, t0, taps, phi, sp, c_true, p_t, alpha1, lam_tv, lam_l1,
                           q, n, 1 if (slow or split) else args.warmup,
                           2 if slow else (3 if split else reps))
    flops = alg_flops(cfg, t0, taps)
    scans = [(5, 7), (cfg.ny // 2, cfg.nx // 2), (cfg.ny - 1, 0), (cfg.ny * 7 // 10, cfg.nx // 4)]
    c_in = torch.from_numpy(c_true).cuda()
    samples = {}
    for q, r in runs.items():
        r["plan"].apply_A(c_in, r["y"])
        samples[q] = np.stack([r["y"][:, iy, ix, :].cpu().numpy() for (iy, ix) in scans])
    del c_in
    # the dominant kernel of the step: the longer of the two band contractions
    dom = "HT" if res["t_HT"] >= res["t_H"] else "H"
    t_dom = res["t_" + dom]
    achieved = flops / (t_dom * 1e-3) / 1e12
    peak = PEAK_TFLOPS[args.prec]
    kname = {"H": "band16_lds (H, y = H b)", "HT": "band16_lds_adj (S^T H^T)"}[dom]
    traffic, traffic_src = profiled_traffic(f"{'band16_lds_adj' if dom == 'HT' else 'band16_lds_H'}"
                                            f"_{cfg.name}_{args.prec}_hbm.md")
    info = res["info"]
    out = {
        "metric": METRIC,
        "value": 1.0 / res["step_s"],
        "unit": "A+AT applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["step_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp16" if args.prec.startswith("fp16") else ("fp32" if args.prec == "fp32" else "bf16"),
        "precision_mode": args.prec,
        "data": "synthetic: seeded tube phantom, synthesized focused-transducer impulse response, "
                "20 dB noise",
        "config": {"workload": f"{cfg.nx}x{cfg.ny}x{cfg.nz} voxels, {cfg.n_species} species, "
                               f"{cfg.n_pulses} pulses, Nt {cfg.nt}, footprint {cfg.f}x{cfg.f}, "
                               f"K2 {cfg.k2}, K1 {cfg.k1}; step = one solver iteration (A, A^T, "
                               f"TV prox, l1, momentum)",
                   "nx": cfg.nx, "ny": cfg.ny, "nz": cfg.nz, "species": cfg.n_species,
                   "pulses": cfg.n_pulses, "nt": cfg.nt, "footprint": cfg.f, "k1": cfg.k1,
                   "k2": cfg.k2},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"{kname}, {args.prec}: algorithmic flops 2*K*sum over offsets of "
                               f"band nonzeros x in-grid scans = {flops / 1e9:.1f} GFLOP per launch",
                     "avg_ms": t_dom, "other_band_kernel_ms": res["t_H" if dom == "HT" else "t_HT"],
                     "traffic_source": traffic_src},
        "cpu_baseline": None,
        "fista_s_to_tol": res["solve_s"], "fista_iterations": cfg.k1,
        "fista_paper_stopping": res.get("solve_tol"),
        "power_iteration": {"steps": 30, "start": "seeded Gaussian",
                            "lambda_max": res["lambda_max"], "alpha1": alpha1},
        "band_fill": info["useful_macs"][0] / max(1, info["executed_macs"][0]),
        "tv_prox_dual_step": tvb,
        "autotune": res.get("autotune"),
        "precisions": per_prec_rows(runs, flops, cfg),
    }
    headline_precs = list(runs)
    for r in runs.values():
        r["plan"].close()
    del runs, res, p_t
    torch.cuda.empty_cache()
    sec = None
    if not (args.headline_only or args.no_secondary):
        out["workload_128x128x64"], sec = secondary_block(torch, pk, synth, args, args.prec)
    if not (args.headline_only or args.no_scales):
        out["scales"] = scale_runs(torch, pk)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline and accuracy (oracle)")
        out["cpu_baseline"] = cpu_baseline(cfg, t0, taps, phi, sp,
                                           args.cpu_crop or (12 if big else 20))
        errs, _ = sampled_A_errors(cfg, t0, taps, phi, sp, c_true, samples, scans)
        for q, e in errs.items():
            out["precisions"][q]["rel_err_A_vs_oracle_sampled"] = e
        case = GOLDEN_CASE[cfg.name]
        gerr, meta = golden_errors(torch, pk, case, headline_precs)
        for q, (e, em) in gerr.items():
            out["precisions"][q]["rel_err_c_vs_oracle_crop"] = e
            out["precisions"][q]["max_abs_err_c_vs_oracle_crop"] = em
        out["c_parity"] = {"case": case, "crop": f"{meta['side']}x{meta['side']} scans, full Nz, "
                                                  f"K, Nt, F", "k1": meta["k1"], "k2": meta["k2"],
                           "reference": "FP64 oracle c_K (tests/golden)"}
        if sec is not None:
            secondary_accuracy(torch, pk, out["workload_128x128x64"], sec, not args.no_c1_oracle)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
