"""GPU parity of the full one-step regulariser with its TV(S c) term: the
stacked dual prox (psoam_prox_r3) against the oracle's prox_r3, the solver
with lambda_tvs > 0 against the oracle's FISTA (same step), its objective
trace, and the batched solve with that prox against one-by-one solves."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, nan_buf, oracle_S, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu


def _c1():
    cfg = synth.C1
    c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    S = oracle_S(cfg, phi, sp)
    return cfg, c_true, t0, taps, phi, sp, n0, v0, S


@pytest.mark.parametrize("which", ["ragged_per_voxel", "c1_depth_table"])
@pytest.mark.parametrize("th", [(0.2, 0.05, 0.1), (0.0, 0.1, 0.0), (0.3, 0.0, 0.05)])
def test_prox_r3_matches_oracle(which, th):
    torch = torch_cuda()
    if which == "ragged_per_voxel":
        cfg, t0, taps, phi, sp = ragged_cfg(2)
    else:
        cfg = synth.C1
        t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
        phi, sp = synth.phi_depth(cfg.nz), synth.species(cfg.n_species, gamma=1.0)
    S = oracle_S(cfg, phi, sp)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    z = (np.random.default_rng(21).standard_normal(cfg.c_shape) * 0.5 + 0.2).astype(np.float32)
    x = nan_buf(cfg.c_shape)
    plan.prox_r3(torch.from_numpy(z).cuda(), *th, 12, x=x)
    ref = oracle.prox_r3(z, S, *th, 12)
    e = oracle.rel_err(x.cpu().numpy(), ref)
    say(f"[r3] prox {which} th={th}: rel err {e:.3e}")
    assert e <= 1e-5
    plan.close()


@pytest.mark.parametrize("which", ["c2_crop_depth_table", "k40_per_voxel"])
def test_prox_r3_many_pulses_matches_oracle(which):
    """The dual step's switching coefficients come from exp at the first
    pulse of each group of four and a per-pulse ratio inside it: checked
    against the oracle's table at 32 pulses (a 24 x 24 crop of the
    128 x 128 x 64 geometry: full depth, 3 species, depth-only fluence, the
    default rate) and at 40 pulses with a per-voxel fluence and the
    fluence-dependent rate (a ragged grid; the last group of four is full,
    the depth not a multiple of the tile), 20 dual steps, with max-abs
    figures beside the normwise error."""
    torch = torch_cuda()
    if which == "c2_crop_depth_table":
        cfg = synth.C2.crop(24, 24)
        phi, sp = synth.phi_depth(cfg.nz), synth.species(cfg.n_species)
        t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    else:
        cfg = synth.Config("k40", nx=10, ny=9, nz=21, n_species=3, n_pulses=40, nt=48, f=5,
                           k1=4, k2=20, seed=31)
        rng = np.random.default_rng(31)
        t0, taps = synth.random_table(cfg.nz, cfg.f, cfg.nt, 7, rng, t0_lo=-3, t0_hi=cfg.nt)
        phi = rng.uniform(0.2, 1.0, size=(cfg.ny, cfg.nx, cfg.nz)).astype(np.float32)
        sp = synth.species(3, gamma=1.0)
    S = oracle_S(cfg, phi, sp)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    z = (np.random.default_rng(22).standard_normal(cfg.c_shape) * 0.5 + 0.2).astype(np.float32)
    zt = torch.from_numpy(z).cuda()
    th, th0 = (0.05, 0.1, 0.02), (0.05, 0.0, 0.02)
    out = []
    for t in (th, th0):
        x = nan_buf(cfg.c_shape)
        plan.prox_r3(zt, *t, 20, x=x)
        out.append(x.cpu().numpy().astype(np.float64))
    ref, ref0 = oracle.prox_r3(z, S, *th, 20), oracle.prox_r3(z, S, *th0, 20)
    e = oracle.rel_err(out[0], ref)
    em = float(np.max(np.abs(out[0] - ref)))
    # the TV(S c) term's own contribution (about 1% of x here), against the oracle's
    ed = oracle.rel_err(out[0] - out[1], ref - ref0)
    say(f"[r3] prox {which} K={cfg.n_pulses}: rel err {e:.3e}, max-abs {em:.3e}; "
        f"TV(S c) contribution {oracle.rel_err(ref, ref0):.2e} of x, its rel err {ed:.3e}")
    assert e <= 1e-5 and em <= 1e-5 * max(1.0, float(np.max(np.abs(ref))))
    assert ed <= 1e-3
    plan.close()


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16", 1e-2)])
def test_fista_with_tvs_matches_oracle(prec, tol):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = _c1()
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    y = A(c_true.astype(np.float64))
    p = (y + synth.noise_sigma(float(np.sqrt(np.mean(y ** 2)))) * n0).astype(np.float32)
    aty = float(np.abs(AT(p.astype(np.float64))).max())
    lam_tv, lam_l1, lam_tvs = 5e-3 * aty, 1e-2 * aty, 2e-3 * aty
    alpha1 = 1.0 / (1.01 * oracle.power_iteration(A, AT, v0, 30))
    k1, k2 = 8, 10
    tr_ref = []
    c_ref, _ = oracle.fista(p.astype(np.float64), A, AT, alpha1, lam_tv, lam_l1, k1, k2,
                            shape_c=cfg.c_shape, lam_tvs=lam_tvs, S=S, trace=tr_ref)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    c, st, tr = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1,
                           lambda_tvs=lam_tvs, k1=k1, k2=k2, alpha1=alpha1, trace=True)
    e = oracle.rel_err(c.cpu().numpy(), c_ref)
    say(f"[r3] FISTA C1 {prec} with TV(Sc): rel err c {e:.3e}; F {tr[-1]:.6e} vs {tr_ref[-1]:.6e}")
    assert st["iterations"] == k1
    assert e <= tol
    # the objective includes the TV(S c) term
    np.testing.assert_allclose(tr, tr_ref, rtol=10 * tol)
    plan.close()


def test_batch_with_tvs_matches_one_by_one():
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = _c1()
    cfg2, t02, taps2, phi2, sp2 = ragged_cfg(4)
    plans = [lib_plan(cfg, t0, taps, phi, sp, "bf16"), lib_plan(cfg2, t02, taps2, phi2, sp2, "fp32")]
    ps, opts, ref = [], [], []
    for i, pl in enumerate(plans):
        p = torch.from_numpy(np.random.default_rng(60 + i).standard_normal(pl.y_shape)
                             .astype(np.float32)).cuda()
        o = dict(lambda_tv=0.05, lambda_l1=0.02, lambda_tvs=0.03, k1=5, k2=6, alpha1=1e-3)
        c, _ = pl.solve(p, **{k: o[k] for k in o})
        ps.append(p)
        opts.append(o)
        ref.append(c.clone())
    cs = [torch.zeros(pl.c_shape, dtype=torch.float32, device="cuda") for pl in plans]
    pk.solve_batch(plans, ps, cs, opts)
    torch.cuda.synchronize()
    for c, r in zip(cs, ref):
        assert torch.equal(c, r)
    for pl in plans:
        pl.close()
