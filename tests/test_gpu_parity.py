"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Tolerances are normwise relative errors (the paper's NRMSE), the operator
bounds of gpu_common.TOL_OP, with the max-abs error beside them.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_MAX, TOL_OP, lib_plan, nan_buf, oracle_S, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu


def _max_abs(got, ref):
    return float(np.abs(got - ref).max()) / float(np.abs(ref).max())


@pytest.fixture(scope="module")
def c1():
    cfg = synth.C1
    c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    S = oracle_S(cfg, phi, sp)
    return cfg, c_true, t0, taps, phi, sp, n0, v0, S


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16", "bf16_split", "fp16_split", "bf16_refined"])
def test_apply_A_and_AT_C1(c1, prec):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    say(f"[parity] C1 apply_A/AT prec={prec}")
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    c = torch.from_numpy(c_true).cuda()
    y = plan.apply_A(c, nan_buf(cfg.y_shape))
    y_ref = oracle.apply_A(c_true, S, t0, taps, cfg.nt)
    e, em = oracle.rel_err(y.cpu().numpy(), y_ref), _max_abs(y.cpu().numpy(), y_ref)
    say(f"   rel err A = {e:.3e}, max-abs {em:.3e}")
    assert e <= TOL_OP[prec] and em <= TOL_MAX[prec]
    yr = np.random.default_rng(1).standard_normal(cfg.y_shape).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape))
    g_ref = oracle.apply_AT(yr, S, t0, taps, cfg.nz)
    e, em = oracle.rel_err(g.cpu().numpy(), g_ref), _max_abs(g.cpu().numpy(), g_ref)
    say(f"   rel err AT = {e:.3e}, max-abs {em:.3e}")
    assert e <= TOL_OP[prec] and em <= TOL_MAX[prec]


@pytest.mark.parametrize("prec,kernel", [("fp32", "global"), ("bf16", "lds"), ("bf16_split", "lds"),
                                         ("fp16", "lds"), ("bf16", "global"),
                                         ("bf16_split", "global"), ("bf16", "lds8"),
                                         ("fp16_split", "lds8"), ("bf16_refined", "lds"),
                                         ("bf16_refined", "global"), ("bf16_refined", "lds8"),
                                         ("bf16", "lds8load"), ("fp16", "lds8load"),
                                         ("bf16_refined", "lds8load"), ("bf16", "lds12"),
                                         ("fp16", "lds12"), ("bf16_refined", "lds12")])
def test_ragged_random_table(prec, kernel, monkeypatch):
    """Sizes off every tile boundary, per-voxel fluence with the fluence-
    dependent rate, asymmetric random band running off both ends; both the
    LDS-staged and the global-operand band kernels."""
    torch = torch_cuda()
    monkeypatch.setenv("PSOAM_BAND_GLOBAL", "1" if kernel == "global" else "0")
    monkeypatch.setenv("PSOAM_LDS_ROWS", "8" if kernel.startswith("lds8") else
                       "12" if kernel == "lds12" else "4")
    monkeypatch.setenv("PSOAM_LDS_LOADW", "1" if kernel == "lds8load" else "0")
    cfg, t0, taps, phi, sp = ragged_cfg(3)
    say(f"[parity] ragged prec={prec}")
    S = oracle_S(cfg, phi, sp)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    if kernel == "lds12":
        assert plan.stats()["lds_rows"] == [12, 12]
    rng = np.random.default_rng(4)
    c = rng.standard_normal(cfg.c_shape).astype(np.float32)
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(cfg.y_shape)).cpu().numpy()
    y_ref = oracle.apply_A(c, S, t0, taps, cfg.nt)
    e, em = oracle.rel_err(y, y_ref), _max_abs(y, y_ref)
    say(f"   rel err A = {e:.3e}, max-abs {em:.3e}")
    assert e <= TOL_OP[prec] and em <= TOL_MAX[prec]
    yr = rng.standard_normal(cfg.y_shape).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape)).cpu().numpy()
    g_ref = oracle.apply_AT(yr, S, t0, taps, cfg.nz)
    e, em = oracle.rel_err(g, g_ref), _max_abs(g, g_ref)
    say(f"   rel err AT = {e:.3e}, max-abs {em:.3e}")
    assert e <= TOL_OP[prec] and em <= TOL_MAX[prec]


@pytest.mark.parametrize("shift", ["0", "4"])
@pytest.mark.parametrize("prec", ["bf16", "fp16_split"])
def test_adjoint_operand_shift(c1, prec, shift, monkeypatch):
    """The 16-bit H^T operand with its samples stored at offset 0 or 4: the
    external adjoint (packed from y), and the solver (residual written by
    H's epilogue), both on the 32x32x16 problem and a ragged one."""
    torch = torch_cuda()
    monkeypatch.setenv("PSOAM_ADJ_SHIFT", shift)
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    yr = np.random.default_rng(12).standard_normal(cfg.y_shape).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape)).cpu().numpy()
    e = oracle.rel_err(g, oracle.apply_AT(yr, S, t0, taps, cfg.nz))
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    alpha1 = 1.0 / (1.01 * oracle.power_iteration(A, AT, v0, 30))
    c_ref, _ = oracle.fista(p.astype(np.float64), A, AT, alpha1, lam_tv, lam_l1, 6, cfg.k2,
                            shape_c=cfg.c_shape)
    c, _ = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1, k1=6,
                      k2=cfg.k2, alpha1=alpha1)
    ec = oracle.rel_err(c.cpu().numpy(), c_ref)
    cfg2, t02, taps2, phi2, sp2 = ragged_cfg(6)
    S2 = oracle_S(cfg2, phi2, sp2)
    plan2 = lib_plan(cfg2, t02, taps2, phi2, sp2, prec)
    y2 = np.random.default_rng(13).standard_normal(cfg2.y_shape).astype(np.float32)
    g2 = plan2.apply_AT(torch.from_numpy(y2).cuda(), nan_buf(cfg2.c_shape)).cpu().numpy()
    e2 = oracle.rel_err(g2, oracle.apply_AT(y2, S2, t02, taps2, cfg2.nz))
    say(f"[parity] adjoint shift {shift} {prec}: A^T {e:.3e}, ragged A^T {e2:.3e}, FISTA(6) c {ec:.3e}")
    assert e <= TOL_OP[prec] and e2 <= TOL_OP[prec]
    assert ec <= (1e-3 if prec == "bf16" else 1e-4)
    plan.close()
    plan2.close()


def test_point_source_fp32(c1):
    """A unit voxel gives the synthesised impulse response times the switching
    curve at every scan of its footprint (checked against the oracle's
    element-wise definition)."""
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    c = np.zeros(cfg.c_shape, np.float32)
    c[1, 3, 30, 9] = 1.0   # near a lateral border
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(cfg.y_shape)).cpu().numpy()
    y_ref = oracle.apply_A(c, S, t0, taps, cfg.nt)
    assert oracle.rel_err(y, y_ref) <= 1e-6
    assert np.count_nonzero(y[:, 10:, :20]) == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_dot_product_identity(c1, prec):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    rng = np.random.default_rng(7)
    x = torch.from_numpy(rng.standard_normal(cfg.c_shape).astype(np.float32)).cuda()
    yv = torch.from_numpy(rng.standard_normal(cfg.y_shape).astype(np.float32)).cuda()
    lhs = float((plan.apply_A(x, nan_buf(cfg.y_shape)).double() * yv.double()).sum())
    rhs = float((x.double() * plan.apply_AT(yv, nan_buf(cfg.c_shape)).double()).sum())
    scale = float(plan.apply_A(x).double().norm() * yv.double().norm())
    say(f"[parity] dot test {prec}: |lhs-rhs|/scale = {abs(lhs - rhs) / scale:.3e}")
    assert abs(lhs - rhs) <= (1e-6 if prec == "fp32" else 2e-3) * scale


def test_prox_l1_matches_closed_form():
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    z = np.random.default_rng(2).standard_normal(100003).astype(np.float32)
    z[:5] = [0.25, -0.25, 0.0, 0.2500001, -0.2499999]
    th = np.float32(0.25)
    zt = torch.from_numpy(z).cuda()
    x1 = pk.prox_l1(zt, float(th), nonneg=True, x=nan_buf(zt.shape)).cpu().numpy()
    np.testing.assert_array_equal(x1, np.maximum(z - th, np.float32(0)))
    x2 = pk.prox_l1(zt, float(th), nonneg=False, x=nan_buf(zt.shape)).cpu().numpy()
    ref = np.sign(z) * np.maximum(np.abs(z) - th, np.float32(0))
    np.testing.assert_array_equal(x2, ref.astype(np.float32))
    # in place
    pk.prox_l1(zt, float(th), nonneg=True, x=zt)
    np.testing.assert_array_equal(zt.cpu().numpy(), x1)


@pytest.mark.parametrize("n_inner,theta,nonneg", [(20, 0.05, False), (50, 0.3, True), (0, 0.1, True), (7, 0.0, False)])
def test_prox_tv_matches_oracle(c1, n_inner, theta, nonneg):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    z = (c_true + 0.2 * np.random.default_rng(5).standard_normal(cfg.c_shape)).astype(np.float32)
    x = plan.prox_tv(torch.from_numpy(z).cuda(), theta, n_inner, nonneg=nonneg,
                     x=nan_buf(cfg.c_shape)).cpu().numpy()
    ref = oracle.prox_tv(z, theta, n_inner, nonneg=nonneg)
    e = oracle.rel_err(x, ref)
    say(f"[parity] prox_tv K2={n_inner} theta={theta}: rel err {e:.3e}")
    assert e <= 1e-5


def test_prox_tv_ragged_inplace():
    torch = torch_cuda()
    cfg, t0, taps, phi, sp = ragged_cfg(1)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    z = np.random.default_rng(8).standard_normal(cfg.c_shape).astype(np.float32)
    zt = torch.from_numpy(z).cuda()
    plan.prox_tv(zt, 0.2, 25, nonneg=False, x=zt)
    e = oracle.rel_err(zt.cpu().numpy(), oracle.prox_tv(z, 0.2, 25))
    assert e <= 1e-5


def _c1_problem(c1):
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    y_clean = oracle.apply_A(c_true.astype(np.float64), S, t0, taps, cfg.nt)
    sig = synth.noise_sigma(float(np.sqrt(np.mean(y_clean ** 2))))
    p = (y_clean + sig * n0).astype(np.float32)
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    aty = np.abs(AT(p.astype(np.float64))).max()
    lam_tv, lam_l1 = 5e-3 * aty, 1e-2 * aty
    return p, A, AT, lam_tv, lam_l1


def test_power_iteration_matches_oracle(c1):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    lam_ref = oracle.power_iteration(A, AT, v0, 30)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    _, st = plan.solve(torch.from_numpy(p).cuda(), k1=0, n_power=30,
                       v0=torch.from_numpy(v0).cuda())
    say(f"[parity] power iteration: gpu {st['lambda_max']:.8e} oracle {lam_ref:.8e}")
    assert st["lambda_max"] == pytest.approx(lam_ref, rel=1e-5)
    assert st["alpha1"] == pytest.approx(1.0 / (1.01 * lam_ref), rel=1e-5)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-4), ("bf16_split", 1e-4), ("bf16", 1e-3),
                                      ("fp16", 1e-3), ("bf16_refined", 1e-3)])
def test_fista_C1_matches_oracle(c1, prec, tol):
    """C1 end to end: 20 FISTA iterations, 20 dual TV iterations, TV + l1 +
    nonnegativity, the oracle's step passed in; concentrations compared."""
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    lam = oracle.power_iteration(A, AT, v0, 30)
    alpha1 = 1.0 / (1.01 * lam)
    c_ref, it = oracle.fista(p.astype(np.float64), A, AT, alpha1, lam_tv, lam_l1, cfg.k1, cfg.k2,
                             shape_c=cfg.c_shape)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    c, st = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1,
                       k1=cfg.k1, k2=cfg.k2, alpha1=alpha1)
    e = oracle.rel_err(c.cpu().numpy(), c_ref)
    say(f"[parity] FISTA C1 {prec}: iterations {st['iterations']} rel err c = {e:.3e}")
    assert st["iterations"] == cfg.k1
    assert e <= tol
    # the reconstruction moved toward the phantom
    assert oracle.rel_err(c.cpu().numpy(), c_true) < 1.0


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_solve_with_unaligned_measurements(c1, prec):
    """Measurements at an address that is not 16-byte aligned (a view one
    float into a buffer): the residual epilogue takes its per-sample loads
    and the iterates equal those of the aligned call bit for bit."""
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    pa = torch.from_numpy(p).cuda()
    buf = torch.zeros(p.size + 1, dtype=torch.float32, device="cuda")
    pu = buf[1:].view(p.shape)
    pu.copy_(pa)
    assert pu.data_ptr() % 16 != 0
    o = dict(lambda_tv=lam_tv, lambda_l1=lam_l1, k1=5, k2=5, alpha1=1e-3)
    ca, sa = plan.solve(pa, **o)
    cu, su = plan.solve(pu, **o)
    say(f"[parity] unaligned measurements {prec}: max |dc| {float((ca - cu).abs().max()):.3e}")
    assert torch.equal(ca, cu)
    plan.close()


def test_fista_trace_and_stopping(c1):
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    lam = oracle.power_iteration(A, AT, v0, 30)
    alpha1 = 1.0 / (1.01 * lam)
    tr_ref = []
    oracle.fista(p.astype(np.float64), A, AT, alpha1, lam_tv, lam_l1, 6, 10, trace=tr_ref,
                 shape_c=cfg.c_shape)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    _, st, tr = plan.solve(torch.from_numpy(p).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1, k1=6,
                           k2=10, alpha1=alpha1, trace=True)
    np.testing.assert_allclose(tr, tr_ref, rtol=1e-5)
    _, it_ref = oracle.fista(p.astype(np.float64), A, AT, alpha1, 0.0, 0.0, 400, 1, eps2=1e-3,
                             shape_c=cfg.c_shape)
    _, st2 = plan.solve(torch.from_numpy(p).cuda(), k1=400, k2=1, alpha1=alpha1, eps2=1e-3)
    say(f"[parity] eps2 stop: gpu {st2['iterations']} oracle {it_ref}")
    assert abs(st2["iterations"] - it_ref) <= 1


def test_autograd_backward_is_adjoint(c1):
    """torch.autograd through A: the gradient of 1/2|A c - p|^2 equals
    A^T (A c - p) of the oracle; central differences agree (the objective is
    quadratic, so only rounding remains)."""
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    c0 = (0.5 * c_true).astype(np.float32)
    c = torch.from_numpy(c0).cuda().requires_grad_(True)
    pt = torch.from_numpy(p).cuda()
    loss = 0.5 * ((pk.A(c, plan) - pt) ** 2).sum()
    loss.backward()
    g_ref = AT(A(c0.astype(np.float64)) - p)
    e = oracle.rel_err(c.grad.cpu().numpy(), g_ref)
    say(f"[parity] autograd gradient rel err {e:.3e}")
    assert e <= 1e-5
    # central differences along the gradient direction, in float64 on the loss
    d = torch.from_numpy(g_ref / np.linalg.norm(g_ref)).float().cuda()
    h = 1e-2 * float(np.linalg.norm(c0))

    def f(cc):
        r = plan.apply_A(cc.contiguous()).double() - pt.double()
        return 0.5 * float((r * r).sum())
    with torch.no_grad():
        fd = (f(c + h * d) - f(c - h * d)) / (2 * h)
    an = float((c.grad.double() * d.double()).sum())
    say(f"[parity] finite difference {fd:.8e} analytic {an:.8e}")
    assert fd == pytest.approx(an, rel=1e-5)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_loader_waves_change_nothing(c1, prec, monkeypatch):
    """The staged H kernel with four loader waves (the next row loaded during
    the current row's contractions) against the same kernel staging its rows
    itself, 8-row workgroups on the 32x32x16 grid and a ragged one: the same
    LDS tiles and the same products in the same order, so A is equal bit for
    bit, and so are the solve's iterates; A^T (the same kernel either way)
    and the iterates also meet the oracle's."""
    torch = torch_cuda()
    cfg, c_true, t0, taps, phi, sp, n0, v0, S = c1
    p, A, AT, lam_tv, lam_l1 = _c1_problem(c1)
    c_ref, _ = oracle.fista(p.astype(np.float64), A, AT, 1e-3, lam_tv, lam_l1, 4, 5,
                            shape_c=cfg.c_shape)
    cfg2, t02, taps2, phi2, sp2 = ragged_cfg(9)
    S2 = oracle_S(cfg2, phi2, sp2)
    c2 = np.random.default_rng(5).standard_normal(cfg2.c_shape).astype(np.float32)
    y2 = np.random.default_rng(6).standard_normal(cfg2.y_shape).astype(np.float32)
    g_ref = oracle.apply_AT(y2, S2, t02, taps2, cfg2.nz)
    monkeypatch.setenv("PSOAM_LDS_ROWS", "8")
    out = {}
    for lw in ("0", "1"):
        monkeypatch.setenv("PSOAM_LDS_LOADW", lw)
        plan = lib_plan(cfg, t0, taps, phi, sp, prec)
        plan2 = lib_plan(cfg2, t02, taps2, phi2, sp2, prec)
        out[lw] = (plan.apply_A(torch.from_numpy(c_true).cuda()),
                   plan2.apply_A(torch.from_numpy(c2).cuda()),
                   plan2.apply_AT(torch.from_numpy(y2).cuda()).cpu().numpy(),
                   plan.solve(torch.from_numpy(p).cuda(), lambda_tv=lam_tv, lambda_l1=lam_l1,
                              k1=4, k2=5, alpha1=1e-3)[0].cpu().numpy())
        plan.close()
        plan2.close()
    assert torch.equal(out["0"][0], out["1"][0]) and torch.equal(out["0"][1], out["1"][1])
    d_at = oracle.rel_err(out["1"][2], out["0"][2])
    e_at = [oracle.rel_err(out[lw][2], g_ref) for lw in ("0", "1")]
    e_c = [oracle.rel_err(out[lw][3], c_ref) for lw in ("0", "1")]
    say(f"[parity] loader waves {prec}: A bitwise equal; A^T differs by {d_at:.2e} "
        f"(oracle {e_at[0]:.2e} / {e_at[1]:.2e}); FISTA(4) c {e_c[0]:.2e} / {e_c[1]:.2e}")
    assert d_at == 0.0
    np.testing.assert_array_equal(out["0"][3], out["1"][3])
    assert max(e_at) <= TOL_OP[prec] and max(e_c) <= 1e-3


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_row_counts_change_nothing(prec, monkeypatch):
    """Workgroups of 4, 8 and 12 output rows: every output row still takes
    the staged rows, runs and pulse blocks in the same order, so A, A^T and
    the solve's iterates are equal bit for bit; the C1 grid and a ragged one.
    The objective trace sums the residual form's FP64 partials (one per
    workgroup row, zero for the blocks past the last position when the
    position blocks do not divide among the 8 XCDs) in an order that follows
    the row count, so it agrees to FP64 rounding."""
    torch = torch_cuda()
    cases = [ragged_cfg(13)]
    cfg1 = synth.C1
    t01, taps1 = synth.sir_table(cfg1.nz, cfg1.f, cfg1.nt)
    cases.append((cfg1, t01, taps1, synth.phi_depth(cfg1.nz), synth.species(cfg1.n_species)))
    monkeypatch.setenv("PSOAM_LDS_LOADW", "0")
    for (cfg, t0, taps, phi, sp) in cases:
        S = oracle_S(cfg, phi, sp)
        rng = np.random.default_rng(23)
        c = rng.standard_normal(cfg.c_shape).astype(np.float32)
        y = rng.standard_normal(cfg.y_shape).astype(np.float32)
        out = {}
        for rows in ("4", "8", "12"):
            monkeypatch.setenv("PSOAM_LDS_ROWS", rows)
            plan = lib_plan(cfg, t0, taps, phi, sp, prec)
            assert plan.stats()["lds_rows"] == [int(rows)] * 2
            c_s, _, tr = plan.solve(torch.from_numpy(y).cuda(), lambda_tv=0.05, lambda_l1=0.02,
                                    k1=4, k2=5, alpha1=1e-3, trace=True)
            out[rows] = (plan.apply_A(torch.from_numpy(c).cuda()).cpu().numpy(),
                         plan.apply_AT(torch.from_numpy(y).cuda()).cpu().numpy(),
                         c_s.cpu().numpy(), np.asarray(tr))
            plan.close()
        for rows in ("8", "12"):
            for a, b in zip(out["4"][:3], out[rows][:3]):
                np.testing.assert_array_equal(a, b)
            np.testing.assert_allclose(out[rows][3], out["4"][3], rtol=1e-13, atol=0.0)
        e = oracle.rel_err(out["12"][0], oracle.apply_A(c, S, t0, taps, cfg.nt))
        say(f"[parity] rows 4/8/12 {prec} {cfg.name}: bitwise equal; A vs oracle {e:.2e}")
        assert e <= TOL_OP[prec]


@pytest.mark.parametrize("prec,rows,loadw", [("bf16", "4", "0"), ("bf16", "8", "1"), ("fp16", "8", "0"),
                                             ("bf16_split", "4", "0"), ("fp16_split", "8", "0"),
                                             ("bf16_refined", "8", "1"), ("bf16", "12", "0"),
                                             ("fp16", "12", "0")])
def test_half_last_block_changes_nothing(prec, rows, loadw, monkeypatch):
    """The last 16-pulse block run in half form (K mod 16 in 1..8: 8 pulses
    per staged column, two positions per matrix-core block) against the same
    block padded to 16 pulses: every output element is the same dot product
    over the same chunks in the same order, and the S^T sum over pulses pairs
    the lanes the same way (the padded form only adds zeros), so A, A^T and
    the solve's iterates are equal bit for bit; both meet the oracle.  The
    ragged grid (K = 19) and a 40-pulse grid with 8-row workgroups."""
    torch = torch_cuda()
    monkeypatch.setenv("PSOAM_LDS_ROWS", rows)
    monkeypatch.setenv("PSOAM_LDS_LOADW", loadw)
    cases = [ragged_cfg(11)]
    cfg5 = synth.Config("k40", nx=21, ny=10, nz=24, n_species=3, n_pulses=40, nt=70, f=9,
                        k1=4, k2=5, seed=12)
    t05, taps5 = synth.sir_table(cfg5.nz, cfg5.f, cfg5.nt)
    cases.append((cfg5, t05, taps5, synth.phi_depth(cfg5.nz), synth.species(3)))
    for (cfg, t0, taps, phi, sp) in cases:
        S = oracle_S(cfg, phi, sp)
        rng = np.random.default_rng(21)
        c = rng.standard_normal(cfg.c_shape).astype(np.float32)
        y = rng.standard_normal(cfg.y_shape).astype(np.float32)
        out = {}
        for hb in ("0", "1"):
            monkeypatch.setenv("PSOAM_HALF_BLOCK", hb)
            plan = lib_plan(cfg, t0, taps, phi, sp, prec)
            out[hb] = (plan.apply_A(torch.from_numpy(c).cuda()).cpu().numpy(),
                       plan.apply_AT(torch.from_numpy(y).cuda()).cpu().numpy(),
                       plan.solve(torch.from_numpy(y).cuda(), lambda_tv=1e-2, lambda_l1=1e-2,
                                  k1=3, k2=4, alpha1=1e-3)[0].cpu().numpy())
            plan.close()
        ea = oracle.rel_err(out["1"][0], oracle.apply_A(c, S, t0, taps, cfg.nt))
        eat = oracle.rel_err(out["1"][1], oracle.apply_AT(y, S, t0, taps, cfg.nz))
        say(f"[parity] half last block {cfg.name} {prec} rows {rows} loaders {loadw}: "
            f"A {ea:.2e}, A^T {eat:.2e}; equal to the padded block: "
            f"{[bool(np.array_equal(a, b)) for a, b in zip(out['0'], out['1'])]}")
        for a, b in zip(out["0"], out["1"]):
            np.testing.assert_array_equal(a, b)
        assert ea <= TOL_OP[prec] and eat <= TOL_OP[prec]
