"""Parity at the full sizes, in the launch configuration the benchmark times.

128 x 128 x 64 voxels, 3 species, 32 pulses, Nt 256, footprint 31 x 31 (the
benchmark workload), 256 x 256 x 96, 32 pulses, Nt 384, footprint 41 x 41,
320 x 320 x 128, 40 pulses, Nt 512, footprint 51 x 51, and two instances of
the batched family:
A and A^T through the library, compared with the FP64 oracle on outputs the
oracle evaluates one by one (A-scans at chosen scan positions, A^T at chosen
voxel columns, including the grid corners where the footprint is cut), every
output written (the buffers start as NaN), the adjoint identity over the whole
grid, and the first solver iteration (l1 + nonnegativity, which acts voxel by
voxel) on sampled columns.  Inputs are the seeded generators'; nothing the
oracle reads comes from the GPU.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, nan_buf, oracle_S, say, torch_cuda

pytestmark = pytest.mark.gpu

# normwise relative error bounds of one operator apply (see the operator tests)
TOL = {"fp32": 1e-5, "bf16": 8e-3, "fp16": 1.5e-3, "bf16_split": 2e-5, "fp16_split": 2e-5,
       "bf16_refined": 8e-3}


def _problem(cfg):
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species)
    c = synth.phantom(cfg).astype(np.float32)
    S = oracle_S(cfg, phi, sp)
    Hs = oracle.band_stack(t0, taps, cfg.nt)
    y = np.random.default_rng(cfg.seed + 17).standard_normal(cfg.y_shape).astype(np.float32)
    return t0, taps, phi, sp, c, S, Hs, y


def _corners(n):
    return [(0, 0), (0, n - 1), (n - 1, n - 1), (n - 1, 0)]


@pytest.fixture(scope="module")
def c2():
    cfg = synth.C2
    return (cfg,) + _problem(cfg)


@pytest.fixture(scope="module")
def c3():
    cfg = synth.C3
    return (cfg,) + _problem(cfg)


def _check_A(torch, data, prec, scans):
    cfg, t0, taps, phi, sp, c, S, Hs, _ = data
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    y = nan_buf(cfg.y_shape)
    plan.apply_A(torch.from_numpy(c).cuda(), y)
    assert bool(torch.isfinite(y).all()), "A left outputs unwritten"
    got = np.stack([y[:, iy, ix, :].cpu().numpy() for (iy, ix) in scans])
    ref = oracle.apply_A_scans(c, S, t0, taps, cfg.nt, scans, Hs=Hs)
    e = oracle.rel_err(got, ref)
    say(f"[full] {cfg.name} A {prec}: {len(scans)} A-scans rel err {e:.3e}")
    plan.close()
    return e


def _check_AT(torch, data, prec, cols):
    cfg, t0, taps, phi, sp, _, S, Hs, y = data
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    g = nan_buf(cfg.c_shape)
    plan.apply_AT(torch.from_numpy(y).cuda(), g)
    assert bool(torch.isfinite(g).all()), "A^T left outputs unwritten"
    got = np.stack([g[:, jy, jx, :].cpu().numpy() for (jy, jx) in cols])
    ref = oracle.apply_AT_columns(y, S, t0, taps, cfg.nz, cols, Hs=Hs)
    e = oracle.rel_err(got, ref)
    say(f"[full] {cfg.name} A^T {prec}: {len(cols)} columns rel err {e:.3e}")
    plan.close()
    return e


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16_split", "fp16_split", "fp32", "bf16_refined"])
def test_c2_apply_A_sampled(c2, prec):
    torch = torch_cuda()
    scans = _corners(128) + [(64, 64), (5, 120), (90, 33), (15, 16)]
    assert _check_A(torch, c2, prec, scans) <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16_split", "fp16_split", "fp32", "bf16_refined"])
def test_c2_apply_AT_sampled(c2, prec):
    torch = torch_cuda()
    cols = _corners(128) + [(64, 64), (17, 111), (100, 3), (15, 16)]
    assert _check_AT(torch, c2, prec, cols) <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_c3_apply_A_and_AT_sampled(c3, prec):
    torch = torch_cuda()
    pts = _corners(256) + [(128, 128), (20, 230), (200, 61)]
    assert _check_A(torch, c3, prec, pts) <= TOL[prec]
    assert _check_AT(torch, c3, prec, pts) <= TOL[prec]


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-6), ("bf16", 5e-3), ("fp16", 1e-3),
                                      ("bf16_refined", 5e-3)])
def test_c2_adjoint_identity(c2, prec, tol):
    """<A x, y> = <x, A^T y> over the whole grid (FP64 sums of the outputs)."""
    torch = torch_cuda()
    cfg, t0, taps, phi, sp, c, S, Hs, y = c2
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    xt = torch.from_numpy(c).cuda()
    yt = torch.from_numpy(y).cuda()
    lhs = float((plan.apply_A(xt).double() * yt.double()).sum())
    rhs = float((xt.double() * plan.apply_AT(yt).double()).sum())
    scale = float(plan.apply_A(xt).double().norm() * yt.double().norm())
    say(f"[full] C2 adjoint identity {prec}: <Ax,y> {lhs:.6e} <x,A^T y> {rhs:.6e}")
    assert abs(lhs - rhs) <= tol * scale
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_c2_first_iteration_sampled(c2, prec):
    """From c = 0 the first iteration is c1 = max(alpha1 A^T p - alpha1 lambda_1, 0)
    when lambda_TV = 0 (gradient at xi = 0 is -A^T p; the l1 + nonnegativity
    prox acts per voxel), so sampled columns of the solver's output follow from
    the oracle's A^T columns.  Runs the solver's own launches (fused residual
    H, H^T with S^T, the combined prox, momentum)."""
    torch = torch_cuda()
    cfg, t0, taps, phi, sp, _, S, Hs, y = c2
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    cols = _corners(128) + [(64, 64), (40, 77)]
    ref_g = oracle.apply_AT_columns(y, S, t0, taps, cfg.nz, cols, Hs=Hs)
    alpha1 = 0.5 / float(np.abs(ref_g).max())
    lam1 = 0.3 * float(np.abs(ref_g).max())
    ref = np.maximum(alpha1 * ref_g - alpha1 * lam1, 0.0)
    c, st = plan.solve(torch.from_numpy(y).cuda(), lambda_tv=0.0, lambda_l1=lam1, k1=1, k2=1,
                       alpha1=alpha1)
    assert st["iterations"] == 1
    got = np.stack([c[:, jy, jx, :].cpu().numpy() for (jy, jx) in cols])
    e = oracle.rel_err(got, ref)
    say(f"[full] C2 first solver iteration {prec}: rel err {e:.3e}")
    assert e <= 3 * TOL[prec]
    plan.close()


# ---------------------------------------------------------------------------
# the largest single solve (320 x 320 x 128, 3 species, 40 pulses, Nt 512,
# footprint 51 x 51) and two instances of the batched family, in the
# precision and launch configuration the benchmark times (BF16).  Inputs are
# seeded uniform values (the tube phantom takes longer to draw at this size
# than the check itself); outputs start as NaN, so a tile left unwritten
# fails the finiteness check.
# ---------------------------------------------------------------------------
def _uniform_problem(cfg):
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species)
    rng = np.random.default_rng(cfg.seed + 5)
    c = rng.random(cfg.c_shape, dtype=np.float32)
    y = rng.random(cfg.y_shape, dtype=np.float32)
    y -= 0.5
    S = oracle_S(cfg, phi, sp)
    Hs = oracle.band_stack(t0, taps, cfg.nt)
    return t0, taps, phi, sp, c, S, Hs, y


@pytest.fixture(scope="module")
def c5():
    cfg = synth.C5
    return (cfg,) + _uniform_problem(cfg)


def test_c5_apply_A_sampled(c5):
    torch = torch_cuda()
    n = c5[0].nx
    assert _check_A(torch, c5, "bf16", [(0, 0), (n - 1, n // 3), (n // 2, n // 2)]) <= TOL["bf16"]


def test_c5_apply_AT_sampled(c5):
    torch = torch_cuda()
    n = c5[0].nx
    assert _check_AT(torch, c5, "bf16", [(n - 1, 0), (n // 2, n // 2 + 7)]) <= TOL["bf16"]


@pytest.mark.parametrize("inst", [8, 4])
def test_batched_family_instance_sampled(inst):
    """Instance 8 (191 x 191 x 51, 22 pulses, Nt 320) and 4 (89 x 89 x 59,
    48 pulses, Nt 352): neither lateral size is a multiple of the position
    block, and 48 pulses fill three 16-pulse blocks."""
    torch = torch_cuda()
    cfg = synth.c4_instance(inst)
    data = (cfg,) + _uniform_problem(cfg)
    n = cfg.nx
    pts = [(0, n - 1), (n - 1, n - 1), (n // 2, 3), (n - 2, n // 2)]
    assert _check_A(torch, data, "bf16", pts) <= TOL["bf16"]
    assert _check_AT(torch, data, "bf16", pts) <= TOL["bf16"]
