"""FP16 operands in any units: the library scales every FP16 operand by a
power of two chosen per call from the data (see include/psoam.h), so inputs
a thousand or ten thousand times larger or smaller than the synthetic
workload's give the same relative error as the workload itself.  Checked
against the FP64 oracle with c, y and p scaled by 1e4 and 1e-4 (A is linear
and the regulariser positively homogeneous, so the scaled solve's c_K is the
unscaled one times the factor when the weights are scaled alike): the banded
operator's A, A^T and FISTA, the factorised operator's A and A^T (its own
operand paths) and the separable form's A and A^T."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_OP, lib_plan, nan_buf, oracle_S, say, torch_cuda

pytestmark = pytest.mark.gpu

SCALES = (1e4, 1e-4)


@pytest.fixture(scope="module")
def c1():
    cfg = synth.C1
    c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    return cfg, c_true, t0, taps, phi, sp, n0, v0, oracle_S(cfg, phi, sp)


@pytest.mark.parametrize("prec", ["fp16", "fp16_split"])
@pytest.mark.parametrize("f", SCALES)
def test_banded_operator_any_units(c1, prec, f):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    c = (c_true * f).astype(np.float32)
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(cfg.y_shape)).cpu().numpy()
    ea = oracle.rel_err(y, oracle.apply_A(c, S, t0, taps, cfg.nt))
    yr = (np.random.default_rng(3).standard_normal(cfg.y_shape) * f).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape)).cpu().numpy()
    eat = oracle.rel_err(g, oracle.apply_AT(yr, S, t0, taps, cfg.nz))
    say(f"[fp16-range] banded {prec} x{f:g}: A {ea:.3e}, A^T {eat:.3e}")
    assert np.isfinite(y).all() and np.isfinite(g).all()
    assert ea <= TOL_OP[prec] and eat <= TOL_OP[prec]
    plan.close()


@pytest.mark.parametrize("prec", ["fp16", "fp16_split"])
@pytest.mark.parametrize("f", SCALES)
def test_solve_any_units(c1, prec, f):
    """20 FISTA iterations with TV + l1 on measurements scaled by f (weights
    scaled alike, the oracle's step): c_K / f against the oracle's unscaled c_K."""
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    y_clean = A(c_true.astype(np.float64))
    p = (y_clean + synth.noise_sigma(float(np.sqrt(np.mean(y_clean ** 2)))) * n0).astype(np.float32)
    aty = float(np.abs(AT(p.astype(np.float64))).max())
    lam_tv, lam_l1 = 5e-3 * aty, 1e-2 * aty
    alpha1 = 1.0 / (1.01 * oracle.power_iteration(A, AT, v0, 30))
    c_ref, _ = oracle.fista(p.astype(np.float64), A, AT, alpha1, lam_tv, lam_l1, cfg.k1, cfg.k2,
                            shape_c=cfg.c_shape)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    ps = torch.from_numpy((p * f).astype(np.float32)).cuda()
    c, st = plan.solve(ps, lambda_tv=lam_tv * f, lambda_l1=lam_l1 * f, k1=cfg.k1, k2=cfg.k2,
                       alpha1=alpha1)
    e = oracle.rel_err(c.cpu().numpy() / f, c_ref)
    say(f"[fp16-range] FISTA {prec} x{f:g}: c_K rel err {e:.3e}")
    assert st["iterations"] == cfg.k1
    assert e <= (1e-3 if prec == "fp16" else 1e-4)
    plan.close()


@pytest.mark.parametrize("f", SCALES)
def test_factorised_operator_any_units(f):
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg = synth.C1
    dr, z_focus, t_focus = synth.shell_geometry(cfg.nz, cfg.nt)
    eir, origin = synth.eir_taps()
    spr = synth.spr_table(cfg.nz, cfg.f)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species)
    S = oracle_S(cfg, phi, sp)
    mask = oracle.shell_mask(cfg.nz, cfg.f, cfg.nt, dr, z_focus, t_focus)
    plan = pk.Plan.factorised(cfg.nx, cfg.ny, cfg.nz, cfg.n_pulses, cfg.nt, cfg.f, phi, sp, spr,
                              eir, origin, dr, z_focus, t_focus, prec="fp16")
    rng = np.random.default_rng(5)
    c = (rng.random(cfg.c_shape) * f).astype(np.float32)
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(cfg.y_shape)).cpu().numpy()
    ea = oracle.rel_err(y, oracle.apply_A_fact(c, S, spr, mask, eir, origin))
    yr = (rng.standard_normal(cfg.y_shape) * f).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape)).cpu().numpy()
    eat = oracle.rel_err(g, oracle.apply_AT_fact(yr, S, spr, mask, eir, origin))
    say(f"[fp16-range] factorised fp16 x{f:g}: A {ea:.3e}, A^T {eat:.3e}")
    assert np.isfinite(y).all() and np.isfinite(g).all()
    assert ea <= TOL_OP["fp16"] and eat <= TOL_OP["fp16"]
    plan.close()


@pytest.mark.parametrize("f", SCALES)
def test_separable_form_any_units(c1, f):
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    plan = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec="fp16", separable=True)
    c = (c_true * f).astype(np.float32)
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(cfg.y_shape)).cpu().numpy()
    ea = oracle.rel_err(y, oracle.apply_A(c, S, t0, taps, cfg.nt))
    yr = (np.random.default_rng(4).standard_normal(cfg.y_shape) * f).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape)).cpu().numpy()
    eat = oracle.rel_err(g, oracle.apply_AT(yr, S, t0, taps, cfg.nz))
    say(f"[fp16-range] separable fp16 x{f:g}: A {ea:.3e}, A^T {eat:.3e}")
    assert ea <= TOL_OP["fp16"] and eat <= TOL_OP["fp16"]
    plan.close()
