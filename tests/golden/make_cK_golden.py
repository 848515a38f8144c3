"""Write the reference concentrations c_K of the FP64 oracle's solver
(Alg. alg:prox-outer with the dual TV prox of Alg. alg:prox-inner) for
lateral crops of the larger workloads' geometry: full depth, pulses, samples
and footprint, a smaller scan grid, so that the oracle finishes in minutes.

    python tests/golden/make_cK_golden.py [name ...]

Uses only the oracle and the seeded generators.  For each case it draws the
crop's phantom, impulse-response table, fluence, noise and power-iteration
start from the workload's seed, forms the measurements p = A c_true + noise
at 20 dB SNR with the oracle, estimates eig_max(A^T A) by 30 power
iterations, sets alpha1 = 1/(1.01 eig), lambda_TV = 5e-3 |A^T p|_inf,
lambda_1 = 1e-2 |A^T p|_inf, runs K1 FISTA iterations with K2 dual steps from
c = 0, and writes c_K (float32, [S][Ny][Nx][Nz]) to cK_<name>.npy plus the
scalars to cK_golden.json.  The GPU tests rebuild p the same way (the oracle's
apply_A on the same generator output) and pass the stored alpha1 and weights.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

# name: (base workload, crop side, K1, K2); "C4_<i>" is instance i of the
# batched uneven family
CASES = {
    "C2_crop24_k2_20": ("C2", 24, 20, 20),
    "C2_crop24_k2_50": ("C2", 24, 20, 50),
    "C5_crop16_k2_50": ("C5", 16, 20, 50),
    "C3_crop16_k2_20": ("C3", 16, 20, 20),
    "C4_3_crop12": ("C4_3", 12, 20, 20),
    "C4_4_crop12": ("C4_4", 12, 20, 20),
    "C4_13_crop12": ("C4_13", 12, 20, 20),
}
N_POWER = 30
JSON = os.path.join(HERE, "cK_golden.json")


def case_config(name: str):
    base, side, k1, k2 = CASES[name]
    full = synth.c4_instance(int(base[3:])) if base.startswith("C4_") else synth.CONFIGS[base]
    cfg = full.crop(side, side, name=name)
    return cfg, k1, k2


def measurements(cfg):
    """(p float32, S, t0, taps, phi, species, v0): the oracle's A c_true plus
    the seeded noise at the generators' SNR."""
    c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, cfg.n_pulses)
    y_clean = oracle.apply_A(c_true.astype(np.float64), S, t0, taps, cfg.nt)
    sig = synth.noise_sigma(float(np.sqrt(np.mean(y_clean ** 2))))
    p = (y_clean + sig * n0).astype(np.float32)
    return p, S, t0, taps, phi, sp, v0, c_true


_SHARED = {}   # (base, side) -> measurements, weights and step (cases differ in K2 only)


def make(name: str) -> dict:
    cfg, k1, k2 = case_config(name)
    t_start = time.time()
    key = CASES[name][:2]
    if key not in _SHARED:
        p, S, t0, taps, phi, sp, v0, c_true = measurements(cfg)
        AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
        A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
        aty = float(np.abs(AT(p.astype(np.float64))).max())
        lam = oracle.power_iteration(A, AT, v0, N_POWER)
        _SHARED[key] = (p, S, t0, taps, c_true, aty, lam)
        print(f"{name}: power iteration done ({time.time() - t_start:.0f} s), eig {lam:.6e}",
              flush=True)
    p, S, t0, taps, c_true, aty, lam = _SHARED[key]
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    p64 = p.astype(np.float64)
    lam_tv, lam_l1 = 5e-3 * aty, 1e-2 * aty
    alpha1 = 1.0 / (1.01 * lam)
    c, it = oracle.fista(p64, A, AT, alpha1, lam_tv, lam_l1, k1, k2, shape_c=cfg.c_shape)
    np.save(os.path.join(HERE, f"cK_{name}.npy"), c.astype(np.float32))
    meta = dict(base=CASES[name][0], side=cfg.nx, nz=cfg.nz, n_species=cfg.n_species,
                n_pulses=cfg.n_pulses, nt=cfg.nt, f=cfg.f, seed=cfg.seed, k1=k1, k2=k2,
                n_power=N_POWER, eig_max=lam, alpha1=alpha1, lambda_tv=lam_tv,
                lambda_l1=lam_l1, iterations=it, norm_cK=float(np.linalg.norm(c)),
                rel_err_vs_phantom=oracle.rel_err(c, c_true),
                oracle_seconds=round(time.time() - t_start, 1))
    print(f"{name}: {meta}", flush=True)
    return meta


def main(names):
    table = json.load(open(JSON)) if os.path.exists(JSON) else {}
    table["_source"] = ("FP64 oracle (oracle/core.py: power_iteration, fista with prox_w) on "
                        "synth.inputs of each crop; written by tests/golden/make_cK_golden.py")
    for name in names:
        table[name] = make(name)
        with open(JSON, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
