"""The two-step method (the paper's comparison): the acoustic-only plan (H on
the K pulse volumes, identity switching) against the oracle's H and H^T, its
solve (TV on every pulse image, nonnegativity) against the oracle's FISTA
with A = H, the unmixing step against the oracle's FISTA with A = S, and the
two steps end to end."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, nan_buf, oracle_S, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 8e-3, "fp16": 1.5e-3}


def _acoustic(cfg, t0, taps, prec):
    import paper_2510_23739_amd as pk
    return pk.Plan.acoustic(cfg.nx, cfg.ny, cfg.nz, cfg.n_pulses, cfg.nt, cfg.f, t0, taps, prec=prec)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_acoustic_plan_matches_oracle_H(prec, which):
    torch = torch_cuda()
    if which == "c1":
        cfg = synth.C1
        t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    else:
        cfg, t0, taps, _, _ = ragged_cfg(6)
    rng = np.random.default_rng(41)
    b = rng.uniform(0, 1, (cfg.n_pulses, cfg.ny, cfg.nx, cfg.nz)).astype(np.float32)
    y = rng.standard_normal(cfg.y_shape).astype(np.float32)
    plan = _acoustic(cfg, t0, taps, prec)
    ya = nan_buf(cfg.y_shape)
    plan.apply_A(torch.from_numpy(b).cuda(), ya)
    ba = nan_buf(b.shape)
    plan.apply_AT(torch.from_numpy(y).cuda(), ba)
    e_a = oracle.rel_err(ya.cpu().numpy(), oracle.apply_H(b, t0, taps, cfg.nt))
    e_t = oracle.rel_err(ba.cpu().numpy(), oracle.apply_HT(y, t0, taps, cfg.nz))
    say(f"[two-step] acoustic {which} {prec}: H {e_a:.3e}  H^T {e_t:.3e}")
    assert e_a <= TOL[prec] and e_t <= TOL[prec]
    plan.close()


def _c1_data():
    cfg = synth.C1
    c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    S = oracle_S(cfg, phi, sp)
    y = oracle.apply_A(c_true.astype(np.float64), S, t0, taps, cfg.nt)
    p = (y + synth.noise_sigma(float(np.sqrt(np.mean(y ** 2)))) * n0).astype(np.float32)
    return cfg, c_true, t0, taps, phi, sp, S, p


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2)])
def test_two_step_matches_oracle(prec, tol):
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, c_true, t0, taps, phi, sp, S, p = _c1_data()
    H = lambda b: oracle.apply_H(b, t0, taps, cfg.nt)
    HT = lambda w: oracle.apply_HT(w, t0, taps, cfg.nz)
    bshape = (cfg.n_pulses, cfg.ny, cfg.nx, cfg.nz)
    nu1 = 5e-3 * float(np.abs(HT(p.astype(np.float64))).max())
    # step sizes given to both sides: H by the oracle's power iteration, S exactly
    v0 = np.random.default_rng(3).standard_normal(bshape)
    a_h = 1.0 / (1.01 * oracle.power_iteration(H, HT, v0, 30))
    a_s = 1.0 / oracle.switching_norm2(S)
    b_ref, _ = oracle.fista(p.astype(np.float64), H, HT, a_h, nu1, 0.0, 15, 10, shape_c=bshape)
    Sop = lambda c: oracle.apply_S(c, S)
    STop = lambda r: oracle.apply_ST(r, S)
    nu2 = 1e-2 * float(np.abs(STop(b_ref)).max())
    nu3 = 5e-3 * float(np.abs(STop(b_ref)).max())
    c_ref, _ = oracle.fista(b_ref, Sop, STop, a_s, nu3, nu2, 15, 10, shape_c=cfg.c_shape)
    assert np.linalg.norm(b_ref) > 0 and np.linalg.norm(c_ref) > 0
    ac = _acoustic(cfg, t0, taps, prec)
    sp_plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    b, c, (st1, st2) = pk.two_step(ac, sp_plan, torch.from_numpy(p).cuda(), nu1, nu2, nu3,
                                   k1_acoustic=15, k1_unmix=15, k2=10, alpha_acoustic=a_h,
                                   alpha_unmix=a_s)
    e_b = oracle.rel_err(b.cpu().numpy(), b_ref)
    # the unmixing step alone, from the oracle's b (isolates its own error)
    c_only, _ = sp_plan.unmix(torch.from_numpy(b_ref.astype(np.float32)).cuda(), lambda_tv=nu3,
                              lambda_l1=nu2, k1=15, k2=10, alpha1=a_s)
    e_u = oracle.rel_err(c_only.cpu().numpy(), c_ref)
    e_c = oracle.rel_err(c.cpu().numpy(), c_ref)
    say(f"[two-step] C1 {prec}: b {e_b:.3e}  unmix alone {e_u:.3e}  c end to end {e_c:.3e}")
    assert st1["iterations"] == 15 and st2["iterations"] == 15
    assert e_b <= tol and e_c <= 3 * tol
    assert e_u <= 1e-5
    ac.close()
    sp_plan.close()


def test_unmix_per_voxel_switching_matches_oracle():
    """Per-voxel fluence and the fluence-dependent rate (gamma = 1)."""
    torch = torch_cuda()
    cfg, t0, taps, phi, sp = ragged_cfg(7)
    S = oracle_S(cfg, phi, sp)
    rng = np.random.default_rng(9)
    b = (rng.uniform(0, 1, (cfg.n_pulses, cfg.ny, cfg.nx, cfg.nz)) * 1e-2).astype(np.float32)
    a_s = 1.0 / oracle.switching_norm2(S)
    c_ref, _ = oracle.fista(b.astype(np.float64), lambda c: oracle.apply_S(c, S),
                            lambda r: oracle.apply_ST(r, S), a_s, 1e-5, 2e-5, 12, 8,
                            shape_c=cfg.c_shape)
    assert np.linalg.norm(c_ref) > 0 and (c_ref == 0).mean() < 0.9  # not shrunk away
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    c, st = plan.unmix(torch.from_numpy(b).cuda(), lambda_tv=1e-5, lambda_l1=2e-5, k1=12, k2=8,
                       alpha1=a_s)
    e = oracle.rel_err(c.cpu().numpy(), c_ref)
    say(f"[two-step] unmix ragged per-voxel: rel err {e:.3e}")
    assert e <= 1e-5
    plan.close()
