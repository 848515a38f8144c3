"""Batched uneven solves (psoam_solve_batch): the captured, concurrent path
gives each problem the same concentrations as solving it alone, over graphs
replayed several times, with odd iteration counts (an uncaptured last
iteration), different iteration counts per problem (several capture phases),
mixed precisions, and eager work and synchronisation between two calls."""
from __future__ import annotations

import numpy as np
import pytest

import synth
from gpu_common import lib_plan, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu


def _problems():
    probs = []
    cfg = synth.C1
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    probs.append((cfg, t0, taps, synth.phi_depth(cfg.nz), synth.species(cfg.n_species), "bf16", 7))
    cfg, t0, taps, phi, sp = ragged_cfg(3)
    probs.append((cfg, t0, taps, phi, sp, "fp32", 8))
    cfg = synth.Config("u3", 40, 24, 20, 3, 12, 96, 9, k1=6, k2=5, seed=77)
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    probs.append((cfg, t0, taps, synth.phi_depth(cfg.nz), synth.species(3), "fp16", 5))
    cfg = synth.Config("u4", 17, 33, 14, 2, 20, 64, 7, k1=4, k2=3, seed=78)
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    probs.append((cfg, t0, taps, synth.phi_depth(cfg.nz), synth.species(2, gamma=1.0),
                  "bf16_split", 4))
    return probs


def test_solve_batch_matches_one_by_one():
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    probs = _problems()
    plans, ps, opts, ref = [], [], [], []
    for i, (cfg, t0, taps, phi, sp, prec, k1) in enumerate(probs):
        plan = lib_plan(cfg, t0, taps, phi, sp, prec)
        rng = np.random.default_rng(100 + i)
        p = torch.from_numpy(rng.standard_normal(cfg.y_shape).astype(np.float32)).cuda()
        aty = float(plan.apply_AT(p).abs().max())
        o = dict(lambda_tv=5e-3 * aty, lambda_l1=1e-2 * aty, k1=k1, k2=cfg.k2, n_power=12)
        c, st = plan.solve(p, lambda_tv=o["lambda_tv"], lambda_l1=o["lambda_l1"], k1=k1,
                           k2=cfg.k2, n_power=12)
        assert st["iterations"] == k1
        # even problems estimate the step in the batch (concurrent power
        # iterations), odd ones are given the step the lone solve found
        o["alpha1"] = 0.0 if i % 2 == 0 else st["alpha1"]
        plans.append(plan)
        ps.append(p)
        opts.append(o)
        ref.append(c.clone())
    for call in range(2):
        cs = [torch.zeros(pl.c_shape, dtype=torch.float32, device="cuda") for pl in plans]
        stats = pk.solve_batch(plans, ps, cs, opts)
        torch.cuda.synchronize()
        for i, (c, r, s) in enumerate(zip(cs, ref, stats)):
            assert s["iterations"] == opts[i]["k1"]
            assert s["status"] == 0
            d = float((c - r).abs().max() / r.abs().max().clamp_min(1e-30))
            say(f"[batch] call {call} problem {i} ({probs[i][5]}, k1 {opts[i]['k1']}): "
                f"max diff vs one-by-one {d:.3e}")
            assert d <= 1e-6
        # eager work and a synchronisation between the two calls
        plans[0].apply_A(cs[0])
        torch.cuda.synchronize()
    for pl in plans:
        pl.close()


def test_solve_batch_falls_back_for_stopping_tests_and_repeated_plans():
    """eps2 > 0 needs host decisions inside the loop, and a plan given twice
    shares its buffers: both are solved one after another, with the same
    results as one-by-one solves."""
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg = synth.C1
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    plan = lib_plan(cfg, t0, taps, synth.phi_depth(cfg.nz), synth.species(2), "fp32")
    rng = np.random.default_rng(5)
    p = torch.from_numpy(rng.standard_normal(cfg.y_shape).astype(np.float32)).cuda()
    o1 = dict(lambda_tv=0.0, lambda_l1=0.0, k1=30, k2=1, alpha1=1e-3, eps2=1e-2)
    o2 = dict(lambda_tv=0.0, lambda_l1=0.0, k1=5, k2=1, alpha1=1e-3)
    r1, s1 = plan.solve(p, k1=30, k2=1, alpha1=1e-3, eps2=1e-2)
    r2, s2 = plan.solve(p, k1=5, k2=1, alpha1=1e-3)
    cs = [torch.zeros(plan.c_shape, dtype=torch.float32, device="cuda") for _ in range(2)]
    stats = pk.solve_batch([plan, plan], [p, p], cs, [o1, o2])
    assert stats[0]["iterations"] == s1["iterations"] <= 30
    assert stats[1]["iterations"] == 5
    assert torch.equal(cs[0], r1) and torch.equal(cs[1], r2)
    plan.close()
