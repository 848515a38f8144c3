"""Shared helpers of the GPU tests: building plans and oracle references from
the same seeded synthetic inputs."""
from __future__ import annotations

import numpy as np

import oracle
import synth


# Normwise relative error bounds of one operator apply (A or A^T) against the
# FP64 oracle.  A 16-bit product carries up to 2^-8 (BF16) or 2^-11 (FP16)
# relative error and the errors of the ~5k terms of one output are nearly
# independent, so the normwise error is of that order; the split forms keep
# ~16 bits.  The bounds sit about twice above the largest errors measured on
# the test workloads (BF16 A^T 2.9e-3, FP16 2.9e-4, BF16 split 4.9e-6, FP32
# 2.7e-6 at 320 x 320 x 128), so a regression that doubles an error fails.
TOL_OP = {"fp32": 6e-6, "bf16": 6e-3, "fp16": 6e-4, "bf16_split": 1e-5, "fp16_split": 1e-5,
          "bf16_refined": 4e-3}
# max-abs error bounds, relative to max |ref| over the compared outputs
TOL_MAX = {"fp32": 1e-5, "bf16": 8e-3, "fp16": 1e-3, "bf16_split": 1.5e-5, "fp16_split": 1.5e-5,
           "bf16_refined": 5e-3}


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def lib_plan(cfg, t0, taps, phi, sp, prec):
    import paper_2510_23739_amd as pk
    return pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=prec)


def oracle_S(cfg, phi, sp):
    return oracle.switching_matrix(np.asarray(phi, np.float64), sp.a, sp.b, sp.tau, sp.gamma,
                                   cfg.n_pulses)


def lam_weights(aty_inf: float):
    """Regularisation weights proportional to |A^T p|_inf (untuned, fixed ratios)."""
    return 5e-3 * aty_inf, 1e-2 * aty_inf


def nan_buf(shape):
    """Output buffer poisoned with NaN, so a call that writes nothing fails."""
    import torch
    return torch.full(tuple(shape), float("nan"), dtype=torch.float32, device="cuda")


def say(msg: str) -> None:
    print(msg, flush=True)


def ragged_cfg(seed=0):
    """Small geometry with every size off the tile grid: Nx not a multiple of
    8, Nt not of 16, Nz not of 8, K not of 16, and an asymmetric random band
    that runs off both ends of the A-scan."""
    cfg = synth.Config("ragged", nx=13, ny=7, nz=11, n_species=3, n_pulses=19, nt=45, f=5,
                       k1=8, k2=6, seed=seed)
    rng = np.random.default_rng(seed)
    t0, taps = synth.random_table(cfg.nz, cfg.f, cfg.nt, 7, rng, t0_lo=-5, t0_hi=cfg.nt + 2)
    phi = rng.uniform(0.2, 1.0, size=(cfg.ny, cfg.nx, cfg.nz)).astype(np.float32)
    sp = synth.species(3, gamma=1.0)
    return cfg, t0, taps, phi, sp
