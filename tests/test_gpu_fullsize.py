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
from gpu_common import TOL_MAX, TOL_OP, lib_plan, nan_buf, oracle_S, say, torch_cuda

pytestmark = pytest.mark.gpu

TOL = TOL_OP   # operator bounds shared with the small-size parity tests


def _max_abs(got, ref, rows):
    """Max-abs error relative to max |ref|, over everything and over the
    listed rows of the last axis (tile and octet edges)."""
    scale = float(np.abs(ref).max())
    rows = [r for r in rows if r < ref.shape[-1]]
    return (float(np.abs(got - ref).max()) / scale,
            float(np.abs(got[..., rows] - ref[..., rows]).max()) / scale)


def _edges(n, tile):
    """Rows on either side of every tile boundary, and the last row."""
    return sorted({r for b in range(tile, n, tile) for r in (b - 1, b)} | {n - 1})


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
    # samples at the 16-row output tile edges and the last (ragged) tile
    em, eb = _max_abs(got, ref, _edges(cfg.nt, 16) + list(range(max(0, cfg.nt - 16), cfg.nt)))
    say(f"[full] {cfg.name} A {prec}: {len(scans)} A-scans rel err {e:.3e}, max-abs {em:.3e}, "
        f"max-abs at tile edges {eb:.3e}")
    plan.close()
    assert em <= TOL_MAX[prec] and eb <= TOL_MAX[prec]
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
    # depths at the 8-deep octet edges and the 16-deep output tile edges
    em, eb = _max_abs(got, ref, _edges(cfg.nz, 8))
    say(f"[full] {cfg.name} A^T {prec}: {len(cols)} columns rel err {e:.3e}, max-abs {em:.3e}, "
        f"max-abs at octet edges {eb:.3e}")
    plan.close()
    assert em <= TOL_MAX[prec] and eb <= TOL_MAX[prec]
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


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16_split", "fp32"])
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


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_c2_first_iteration_with_tv(c2, prec):
    """First solver iteration with TV + l1 + nonnegativity on the whole
    128 x 128 x 64 grid (K2 = 20 dual steps across the depth tiles).  The
    measurements are nonzero on a 3 x 3 block of scan positions only, so
    A^T p vanishes outside the block of voxel columns within the footprint
    of those scans; the oracle evaluates A^T p on that block (a cropped grid
    holds every term there) and c1 = prox(alpha1 A^T p) on the whole volume."""
    torch = torch_cuda()
    cfg, t0, taps, phi, sp, _, S, Hs, _ = c2
    R = cfg.r
    iy0, ix0 = 60, 70
    p = np.zeros(cfg.y_shape, np.float32)
    p[:, iy0:iy0 + 3, ix0:ix0 + 3, :] = np.random.default_rng(2024).standard_normal(
        (cfg.n_pulses, 3, 3, cfg.nt)).astype(np.float32)
    ya, yb, xa, xb = iy0 - R, iy0 + 3 + R, ix0 - R, ix0 + 3 + R
    g = np.zeros(cfg.c_shape)
    g[:, ya:yb, xa:xb, :] = oracle.apply_AT(p[:, ya:yb, xa:xb, :], S, t0, taps, cfg.nz)
    gmax = float(np.abs(g).max())
    alpha1, lam_tv, lam_l1 = 0.5 / gmax, 0.05 * gmax, 0.02 * gmax
    ref = oracle.prox_w(alpha1 * g, alpha1 * lam_tv, alpha1 * lam_l1, 20)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    c, st = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1, k1=1,
                       k2=20, alpha1=alpha1)
    assert st["iterations"] == 1
    got = c.cpu().numpy()
    e = oracle.rel_err(got, ref)
    em = float(np.abs(got - ref).max()) / float(np.abs(ref).max())
    say(f"[full] C2 first solver iteration with TV {prec}: rel err {e:.3e}, max-abs {em:.3e}, "
        f"nonzero voxels {np.count_nonzero(ref)} of {ref.size}")
    assert np.count_nonzero(ref) > 1000
    assert e <= 3 * TOL[prec] and em <= 3 * TOL_MAX[prec]
    plan.close()


def test_c2_finite_difference_gradient(c2):
    """The autograd gradient of 1/2 |A c - p|^2 (backward = the library's A^T)
    against central differences, FP32, on the whole 128 x 128 x 64 grid (the
    objective is quadratic, so only rounding separates the two).  Directions:
    the gradient itself (the largest directional derivative, so the
    difference of the two FP32 objective values is well above their rounding)
    and a seeded random direction mixed into it."""
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, t0, taps, phi, sp, c0, S, Hs, y = c2
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    c = torch.from_numpy(0.5 * c0).cuda().requires_grad_(True)
    pt = torch.from_numpy(y).cuda()
    loss = 0.5 * ((pk.A(c, plan) - pt) ** 2).sum()
    loss.backward()
    gr = c.grad.detach().double().cpu().numpy()
    rng = np.random.default_rng(2025)
    rnd = rng.standard_normal(cfg.c_shape)
    h = 1e-1 * float(np.linalg.norm(0.5 * c0))

    def f(cc):
        r = plan.apply_A(cc.contiguous()).double() - pt.double()
        return 0.5 * float((r * r).sum())
    for label, d in (("gradient", gr), ("gradient + random", gr / np.linalg.norm(gr)
                                         + 0.5 * rnd / np.linalg.norm(rnd))):
        d = d / np.linalg.norm(d)
        dt = torch.from_numpy(d).float().cuda()
        with torch.no_grad():
            fd = (f(c + h * dt) - f(c - h * dt)) / (2 * h)
        an = float((c.grad.double() * dt.double()).sum())
        say(f"[full] C2 finite difference ({label}) {fd:.8e} analytic {an:.8e} "
            f"rel {abs(fd - an) / abs(an):.2e}")
        assert fd == pytest.approx(an, rel=1e-5)
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


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16_split", "fp32"])
def test_c5_apply_A_sampled(c5, prec):
    torch = torch_cuda()
    n = c5[0].nx
    pts = [(0, 0), (n - 1, n // 3), (n // 2, n // 2), (15, 16)]
    assert _check_A(torch, c5, prec, pts) <= TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16", "bf16_split", "fp32"])
def test_c5_apply_AT_sampled(c5, prec):
    torch = torch_cuda()
    n = c5[0].nx
    pts = [(n - 1, 0), (n // 2, n // 2 + 7), (16, 15)]
    assert _check_AT(torch, c5, prec, pts) <= TOL[prec]


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
