"""Reconstructed concentrations against the FP64 oracle's c_K on lateral crops
of the larger workloads' geometry (full depth, pulses, samples, footprint):
128 x 128 x 64-geometry crops of 24 x 24 scans with K2 = 20 and 50 dual steps,
a 320 x 320 x 128-geometry crop (40 pulses, Nt 512, footprint 51 x 51) of
16 x 16 scans with K2 = 50, a 256 x 256 x 96-geometry crop (footprint 41 x 41,
Nt 384) of 16 x 16 scans with K2 = 20, and 12 x 12-scan crops of three instances of the
batched uneven family (solved together by psoam_solve_batch), each after
K1 = 20 solver iterations (Alg. alg:prox-outer, TV + l1 + nonnegativity).

The reference c_K, the step alpha1 (the oracle's power iteration) and the
weights were written by tests/golden/make_cK_golden.py from the oracle alone;
the measurements are rebuilt here the same way (the oracle's A on the seeded
phantom plus the seeded noise), so no input comes from the GPU.  Bounds:
1e-3 relative for the one-part 16-bit forms (the target of the mixed
precision path), 1e-4 for FP32 and the split forms.
"""
import importlib.util
import json
import os

import numpy as np
import pytest

import oracle
from gpu_common import lib_plan, say, torch_cuda

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")
_spec = importlib.util.spec_from_file_location("make_cK_golden",
                                               os.path.join(GOLDEN, "make_cK_golden.py"))
mk = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(mk)

TABLE = json.load(open(mk.JSON)) if os.path.exists(mk.JSON) else {}
CASES = sorted(k for k in TABLE if not k.startswith("_"))
TOL_C = {"bf16": 1e-3, "fp16": 1e-3, "bf16_refined": 1e-3, "fp32": 1e-4, "bf16_split": 1e-4,
         "fp16_split": 1e-4}
PRECS = {"C2_crop24_k2_20": ["bf16", "fp16", "bf16_refined", "fp32", "bf16_split", "fp16_split"],
         "C2_crop24_k2_50": ["bf16", "fp32"],
         "C5_crop16_k2_50": ["bf16", "fp16", "fp32", "bf16_split"],
         "C3_crop16_k2_20": ["bf16", "fp16", "fp32", "bf16_split", "fp16_split"]}

_MEAS = {}


def _case(name):
    if name not in _MEAS:
        cfg, k1, k2 = mk.case_config(name)
        say(f"[golden] {name}: rebuilding measurements with the oracle")
        p, S, t0, taps, phi, sp, v0, c_true = mk.measurements(cfg)
        ref = np.load(os.path.join(GOLDEN, f"cK_{name}.npy"))
        _MEAS[name] = (cfg, p, t0, taps, phi, sp, ref)
    return _MEAS[name]


@pytest.mark.parametrize("name,prec", [(n, p) for n in CASES for p in PRECS.get(n, ["bf16"])])
def test_concentrations_match_oracle(name, prec):
    torch = torch_cuda()
    meta = TABLE[name]
    cfg, p, t0, taps, phi, sp, ref = _case(name)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    c, st = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=meta["lambda_tv"],
                       lambda_l1=meta["lambda_l1"], k1=meta["k1"], k2=meta["k2"],
                       alpha1=meta["alpha1"])
    got = c.cpu().numpy()
    e = oracle.rel_err(got, ref)
    em = float(np.abs(got - ref).max()) / float(np.abs(ref).max())
    say(f"[golden] {name} {prec}: c_K rel err {e:.3e}, max-abs {em:.3e} "
        f"(K1 {meta['k1']}, K2 {meta['k2']})")
    assert st["iterations"] == meta["k1"]
    assert e <= TOL_C[prec]
    plan.close()


BATCH = ["C4_3_crop12", "C4_4_crop12", "C4_13_crop12"]


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_batched_family_crops_match_oracle(prec):
    """Crops of three uneven instances (depths 77, 59, 89; 21, 48, 29 pulses;
    2, 2, 3 species; Nt 384, 352, 320) solved in one psoam_solve_batch call
    (per-problem streams, captured iteration pairs), twice, each c_K against
    its stored oracle c_K."""
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    plans, ps, opts, refs = [], [], [], []
    for name in BATCH:
        meta = TABLE[name]
        cfg, p, t0, taps, phi, sp, ref = _case(name)
        plans.append(lib_plan(cfg, t0, taps, phi, sp, prec))
        ps.append(torch.from_numpy(p).cuda())
        opts.append(dict(lambda_tv=meta["lambda_tv"], lambda_l1=meta["lambda_l1"], k1=meta["k1"],
                         k2=meta["k2"], alpha1=meta["alpha1"]))
        refs.append(ref)
    for call in range(2):
        cs = [torch.zeros(pl.c_shape, dtype=torch.float32, device="cuda") for pl in plans]
        stats = pk.solve_batch(plans, ps, cs, opts)
        torch.cuda.synchronize()
        for name, c, st, ref, o in zip(BATCH, cs, stats, refs, opts):
            e = oracle.rel_err(c.cpu().numpy(), ref)
            say(f"[golden] batch call {call} {name} {prec}: c_K rel err {e:.3e}")
            assert st["iterations"] == o["k1"]
            assert e <= TOL_C[prec]
    for pl in plans:
        pl.close()


def test_golden_cases_present():
    assert {"C2_crop24_k2_20", "C2_crop24_k2_50", "C5_crop16_k2_50",
            "C3_crop16_k2_20"} | set(BATCH) <= set(CASES)
