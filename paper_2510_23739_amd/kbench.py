"""Kernel micro-benchmark: repeated launches of the band contractions (and the
TV dual step) on one synthetic workload, for profiling under rocprofv3.

    python -m paper_2510_23739_amd.kbench --config C2 --prec bf16 --reps 5

Prints one JSON line with the average time of each launch kind (HIP events on
the stream the kernels run on).
"""
from __future__ import annotations

import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="C2")
    ap.add_argument("--crop", type=int, default=0, help="lateral crop (0 = full grid)")
    ap.add_argument("--pulses", type=int, default=0, help="pulse count (0 = the workload's)")
    ap.add_argument("--prec", default="bf16")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--what", default="fwd,adj,tv")
    ap.add_argument("--tune", action="store_true",
                    help="launch shapes chosen by the autotuner (plain and batched plans)")
    ap.add_argument("--fact", action="store_true",
                    help="factorised acoustic operator (shell sums + impulse-response pass)")
    args = ap.parse_args()
    import numpy as np
    import torch

    import paper_2510_23739_amd as pk
    import synth

    cfg = synth.CONFIGS[args.config]
    if args.crop:
        cfg = cfg.crop(args.crop, args.crop)
    if args.pulses:
        import dataclasses
        cfg = dataclasses.replace(cfg, n_pulses=args.pulses)
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species)
    rng = np.random.default_rng(0)
    c = torch.from_numpy(rng.random(cfg.c_shape, dtype=np.float32)).cuda()
    if args.fact:
        dr, z_focus, t_focus = synth.shell_geometry(cfg.nz, cfg.nt)
        eir, origin = synth.eir_taps()
        plan = pk.Plan.factorised(cfg.nx, cfg.ny, cfg.nz, cfg.n_pulses, cfg.nt, cfg.f, phi, sp,
                                  synth.spr_table(cfg.nz, cfg.f), eir, origin, dr, z_focus,
                                  t_focus, prec=args.prec)
    else:
        plan = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=args.prec, tune=args.tune)
    y = torch.empty(cfg.y_shape, dtype=torch.float32, device="cuda")
    g = torch.empty(cfg.c_shape, dtype=torch.float32, device="cuda")
    st = torch.cuda.current_stream()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(args.reps):
            fn()
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.reps

    out = {"config": cfg.name, "prec": args.prec, "factorised": args.fact, "tuned": args.tune,
           "stats": plan.stats()}
    what = args.what.split(",")
    if "mfma" in what:
        # dense BF16 matrix-core rate of this device: a loop of
        # v_mfma_f32_16x16x32_bf16 on independent accumulators, 8 blocks per CU
        import ctypes as C
        lib = C.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpsoam_calib.so"))
        lib.psoam_calib_mfma_bf16.restype = C.c_int
        lib.psoam_calib_mfma_bf16.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_void_p]
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        blocks, iters = 8 * cus, 512
        buf = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")

        def mfma_loop():
            rc = lib.psoam_calib_mfma_bf16(C.c_void_p(buf.data_ptr()), blocks, iters,
                                           C.c_void_p(st.cuda_stream))
            if rc:
                raise RuntimeError(f"psoam_calib_mfma_bf16 returned {rc}")

        ms = timed(mfma_loop)
        flops = blocks * 4 * iters * 8 * 16 * 16 * 32 * 2
        out["mfma_bf16_cus"] = cus
        out["mfma_bf16_ms"] = ms
        out["mfma_bf16_tflops"] = flops / (ms * 1e-3) / 1e12
    if "copy" in what:
        # plain device copy of a known size: calibrates the HBM byte counters
        n = 1 << 28  # 1 GiB of float32
        xa = torch.ones(n, dtype=torch.float32, device="cuda")
        xb = torch.empty_like(xa)
        out["copy_bytes"] = 4 * n
        out["copy_ms"] = timed(lambda: xb.copy_(xa))
        del xa, xb
    if "fwd" in what:
        plan.apply_A(c, y)
        out["H_ms"] = timed(lambda: plan.band_only(0, y))
    if "adj" in what:
        plan.apply_A(c, y)
        plan.apply_AT(y, g)
        out["HT_ms"] = timed(lambda: plan.band_only(1, g))
    if "apply" in what:
        out["apply_A_ms"] = timed(lambda: plan.apply_A(c, y))
        out["apply_AT_ms"] = timed(lambda: plan.apply_AT(y, g))
    if "tune" in what and not args.fact:
        # the launch-shape autotuner on this workload: wall time and choice
        import time
        t_0 = time.perf_counter()
        tp = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=args.prec, tune=True)
        out["tune_s"] = time.perf_counter() - t_0
        out["tune_report"] = tp.tune_report
        tp.close()
    if "solve" in what:
        # solver iterations at a fixed step; A c stands in for the measurements
        plan.apply_A(c, y)
        x = torch.zeros_like(c)
        out["solve_step_ms"] = timed(lambda: plan.solve(y, c=x, lambda_tv=1e-3, lambda_l1=1e-3,
                                                        k1=5, k2=cfg.k2, alpha1=1e-3)) / 5
    if "tv" in what:
        out["prox_tv_k20_ms"] = timed(lambda: plan.prox_tv(c, 0.01, 20, x=g))
    if "batch" in what:
        # the batched uneven family (16 instances, 100 outer iterations, K2 20,
        # 10-step power iteration): one solve_batch call, then one by one
        import time
        plans, ps, opts = [], [], []
        for i in range(16):
            ci = synth.c4_instance(i)
            a0, a1 = synth.sir_table(ci.nz, ci.f, ci.nt)
            plans.append(pk.Plan.from_config(ci, synth.phi_depth(ci.nz), synth.species(ci.n_species),
                                             a0, a1, prec=args.prec, tune=args.tune))
            rng = np.random.default_rng(ci.seed)
            ps.append(torch.from_numpy(rng.standard_normal(ci.y_shape, dtype=np.float32)).cuda())
            opts.append(dict(lambda_tv=1e-3, lambda_l1=1e-3, k1=ci.k1, k2=20, n_power=10))
        cs = [torch.zeros(pl.c_shape, dtype=torch.float32, device="cuda") for pl in plans]
        pk.solve_batch(plans, ps, cs, [dict(o, k1=2) for o in opts])
        torch.cuda.synchronize()
        t_0 = time.perf_counter()
        pk.solve_batch(plans, ps, cs, opts)
        torch.cuda.synchronize()
        out["batch_s"] = time.perf_counter() - t_0
        t_0 = time.perf_counter()
        for pl, p_, c_, o in zip(plans, ps, cs, opts):
            c_.zero_()
            pl.solve(p_, c=c_, **o)
        torch.cuda.synchronize()
        out["one_by_one_s"] = time.perf_counter() - t_0
        for pl in plans:
            pl.close()
    if "r3" in what:
        out["prox_r3_k20_ms"] = timed(lambda: plan.prox_r3(c, 0.01, 0.005, 0.01, 20, x=g))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
