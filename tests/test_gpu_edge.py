"""GPU edge cases: the degenerate geometries of the operator, against closed
forms and the oracle.

- A = I: one species, one pulse, a one-column footprint, an impulse response
  that is a unit impulse at the voxel's own depth (Nt = Nz), unit fluence and
  a switching model without decay (a = 1, b = 0), so S and H are identities.
  A c and A^T y equal their input up to one rounding of the operand (none in
  FP32); the power iteration finds lambda = 1; FISTA on min 1/2 |c - p|^2 +
  lambda_1 |c|_1 with c >= 0 reaches the closed form max(p - lambda_1, 0)
  (Sec. 2.3, eq. one-step and the prox of the l1 term), and with the TV term
  it matches the oracle's iterates.
- The smallest grid (one voxel, one sample, footprint 1) and a footprint
  wider than the grid (every neighbour outside the grid is zero, Sec. 2.2).
- Empty work: prox_l1 of zero elements, a solve of zero iterations.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import TOL_OP, nan_buf, oracle_S, say, torch_cuda

pytestmark = pytest.mark.gpu

PRECS = ["fp32", "bf16", "fp16", "bf16_split", "fp16_split", "bf16_refined"]
# one rounding of each operand element: the unit roundoff of the format
# (BF16 8 significant bits, FP16 11; the split forms carry a second part of
# the same format, ~16 bits); FP32 multiplies by 1 and adds zeros exactly
UNIT = {"fp32": 1e-7, "bf16": 2.0 ** -8, "fp16": 2.0 ** -11, "bf16_split": 2.0 ** -16,
        "fp16_split": 2.0 ** -16, "bf16_refined": 2.0 ** -8}


def _plan(nx, ny, nz, k, nt, f, phi, sp, t0, taps, prec):
    import paper_2510_23739_amd as pk
    return pk.Plan(nx, ny, nz, k, nt, f, phi, sp, t0, taps, prec=prec)


def _identity(prec, nx=9, ny=5, nz=20):
    t0 = np.arange(nz, dtype=np.int32).reshape(nz, 1, 1)
    taps = np.ones((nz, 1, 1, 1), dtype=np.float32)
    phi = np.ones(nz, dtype=np.float32)
    sp = synth.Species((1.0,), (0.0,), (1.0,), 0.0)
    return _plan(nx, ny, nz, 1, nz, 1, phi, sp, t0, taps, prec), (1, ny, nx, nz)


@pytest.mark.parametrize("prec", PRECS)
def test_identity_operator(prec):
    torch = torch_cuda()
    say(f"[edge] identity operator {prec}")
    plan, shape = _identity(prec)
    rng = np.random.default_rng(21)
    c = rng.standard_normal(shape).astype(np.float32)
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(shape)).cpu().numpy()
    ea = oracle.rel_err(y, c)
    g = plan.apply_AT(torch.from_numpy(c).cuda(), nan_buf(shape)).cpu().numpy()
    eat = oracle.rel_err(g, c)
    _, st = plan.solve(torch.zeros(shape, device="cuda"), k1=0, n_power=30,
                       v0=torch.from_numpy(rng.standard_normal(shape).astype(np.float32)).cuda())
    say(f"   A {ea:.3e}  A^T {eat:.3e}  lambda {st['lambda_max']:.9f}")
    assert ea <= UNIT[prec] and eat <= UNIT[prec]
    # the normalised iterate is stored in FP32, so <v, v> = 1 to ~2^-23
    assert abs(st["lambda_max"] - 1.0) <= max(2 * UNIT[prec], 1e-6)
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16_split"])
def test_identity_solve(prec):
    torch = torch_cuda()
    say(f"[edge] identity solve {prec}")
    plan, shape = _identity(prec)
    p = np.random.default_rng(22).standard_normal(shape).astype(np.float32)
    pg = torch.from_numpy(p).cuda()
    alpha1 = 1.0 / 1.01
    # l1 + nonnegativity only: the closed form
    c, st = plan.solve(pg, lambda_l1=0.3, k1=30, k2=10, alpha1=alpha1)
    e = oracle.rel_err(c.cpu().numpy(), np.maximum(p.astype(np.float64) - 0.3, 0.0))
    # with TV: the oracle's iterates on the same operator
    I = lambda v: v
    c_ref, _ = oracle.fista(p.astype(np.float64), I, I, alpha1, 0.2, 0.1, 12, 15, shape_c=shape)
    c2, _ = plan.solve(pg, lambda_tv=0.2, lambda_l1=0.1, k1=12, k2=15, alpha1=alpha1)
    e2 = oracle.rel_err(c2.cpu().numpy(), c_ref)
    say(f"   l1 closed form {e:.3e}  TV+l1 vs oracle {e2:.3e}")
    tol = max(UNIT[prec], 1e-5)
    assert st["iterations"] == 30
    assert e <= 4 * tol and e2 <= 4 * tol
    plan.close()


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("dims", [(1, 1, 1, 1, 1, 1, 1), (1, 1, 3, 3, 7, 5, 2),
                                  (2, 3, 1, 2, 5, 3, 3)],
                         ids=["one-voxel", "footprint-wider-than-grid", "one-depth"])
def test_tiny_grids_match_oracle(prec, dims):
    """dims = (nx, ny, nz, n_pulses, nt, f, n_species)."""
    torch = torch_cuda()
    nx, ny, nz, k, nt, f, ns = dims
    say(f"[edge] tiny grid {dims} {prec}")
    rng = np.random.default_rng(23)
    t0, taps = synth.random_table(nz, f, nt, 3, rng, t0_lo=-1, t0_hi=nt)
    phi = rng.uniform(0.3, 1.0, size=(ny, nx, nz)).astype(np.float32)
    sp = synth.species(ns, gamma=1.0)
    cfg = synth.Config("tiny", nx=nx, ny=ny, nz=nz, n_species=ns, n_pulses=k, nt=nt, f=f, k1=1)
    S = oracle_S(cfg, phi, sp)
    plan = _plan(nx, ny, nz, k, nt, f, phi, sp, t0, taps, prec)
    c = rng.standard_normal(cfg.c_shape).astype(np.float32)
    y = plan.apply_A(torch.from_numpy(c).cuda(), nan_buf(cfg.y_shape)).cpu().numpy()
    ea = oracle.rel_err(y, oracle.apply_A(c, S, t0, taps, nt))
    yr = rng.standard_normal(cfg.y_shape).astype(np.float32)
    g = plan.apply_AT(torch.from_numpy(yr).cuda(), nan_buf(cfg.c_shape)).cpu().numpy()
    eat = oracle.rel_err(g, oracle.apply_AT(yr, S, t0, taps, nz))
    say(f"   A {ea:.3e}  A^T {eat:.3e}")
    assert ea <= TOL_OP[prec] and eat <= TOL_OP[prec]
    plan.close()


def test_empty_work():
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    say("[edge] empty prox_l1, zero-iteration solve")
    z = torch.empty(0, device="cuda")
    x = pk.prox_l1(z, 0.5)
    assert x.numel() == 0
    plan, shape = _identity("bf16")
    c0 = torch.from_numpy(np.random.default_rng(24).standard_normal(shape).astype(np.float32)).cuda()
    c = c0.clone()
    _, st = plan.solve(torch.zeros(shape, device="cuda"), c=c, k1=0, alpha1=0.5)
    torch.cuda.synchronize()
    assert st["iterations"] == 0
    assert torch.equal(c, c0)
    plan.close()
