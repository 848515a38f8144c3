"""Shared helpers of the GPU tests: building plans and oracle references from
the same seeded synthetic inputs."""
from __future__ import annotations

import numpy as np

import oracle
import synth


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
