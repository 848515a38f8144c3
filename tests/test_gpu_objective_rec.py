"""The solver's objective without a second H apply: F(c_{k+1})'s data term
from A c_{k+1} = (A xi_{k+1} + beta_k A c_k) / (1 + beta_k) (A is linear and
xi_{k+1} = c_{k+1} + beta_k (c_{k+1} - c_k), Alg. alg:prox-outer), formed in
the epilogue of the next iteration's H.  Against the direct evaluation
(PSOAM_OBJ_DIRECT=1: S and H applied to c_{k+1}): the iterates are the same
bit for bit (the objective only feeds the stopping test), the traces agree
to rounding (FP32) or to the 16-bit operand's rounding, and both meet the
oracle's trace; the eps1 stop lands on the same iteration."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, oracle_S, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu


def _problem(which):
    if which == "c1":
        cfg = synth.C1
        c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    else:
        cfg, t0, taps, phi, sp = ragged_cfg(17)
        rng = np.random.default_rng(17)
        c_true = np.abs(rng.standard_normal(cfg.c_shape)).astype(np.float32)
        n0 = rng.standard_normal(cfg.y_shape)
    S = oracle_S(cfg, phi, sp)
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    y = A(c_true.astype(np.float64))
    p = (y + synth.noise_sigma(float(np.sqrt(np.mean(y ** 2)))) * n0).astype(np.float32)
    aty = float(np.abs(AT(p.astype(np.float64))).max())
    v0 = synth.power_start(int(np.prod(cfg.c_shape)), np.random.default_rng(3)).reshape(cfg.c_shape)
    alpha1 = 1.0 / (1.01 * oracle.power_iteration(A, AT, v0, 30))
    return cfg, t0, taps, phi, sp, p, A, AT, 5e-3 * aty, 1e-2 * aty, alpha1


@pytest.mark.parametrize("prec,kernel,rtol", [("fp32", "lds", 1e-6), ("bf16", "lds", 1e-2),
                                              ("fp16", "lds", 1e-2), ("bf16", "global", 1e-2),
                                              ("fp32", "ragged", 1e-6), ("bf16", "ragged", 1e-2)])
def test_recurrence_matches_direct_objective(prec, kernel, rtol, monkeypatch):
    torch = torch_cuda()
    which = "ragged" if kernel == "ragged" else "c1"
    cfg, t0, taps, phi, sp, p, A, AT, lam_tv, lam_l1, alpha1 = _problem(which)
    monkeypatch.setenv("PSOAM_BAND_GLOBAL", "1" if kernel == "global" else "0")
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    pt = torch.from_numpy(p).cuda()
    o = dict(lambda_tv=lam_tv, lambda_l1=lam_l1, k1=12, k2=6, alpha1=alpha1, trace=True)
    out = {}
    for direct in ("1", "0"):
        monkeypatch.setenv("PSOAM_OBJ_DIRECT", direct)
        out[direct] = plan.solve(pt, **o)
    (cd, sd, trd), (cr, sr, trr) = out["1"], out["0"]
    tr_ref = []
    oracle.fista(p.astype(np.float64), A, AT, alpha1, lam_tv, lam_l1, 12, 6, trace=tr_ref,
                 shape_c=cfg.c_shape)
    dtr = float(np.max(np.abs(np.asarray(trr) - np.asarray(trd)) / np.abs(np.asarray(trd))))
    eref = float(np.max(np.abs(np.asarray(trr) - np.asarray(tr_ref)) / np.abs(np.asarray(tr_ref))))
    say(f"[objective] {prec} {kernel}: iterates equal {bool(torch.equal(cd, cr))}; trace "
        f"recurrence vs direct {dtr:.2e}, vs oracle {eref:.2e}")
    assert torch.equal(cd, cr)
    assert sd["iterations"] == sr["iterations"] == 12
    np.testing.assert_allclose(trr, trd, rtol=rtol)
    np.testing.assert_allclose(trr, tr_ref, rtol=1e-5 if prec == "fp32" else 1e-2)
    plan.close()


@pytest.mark.parametrize("device_stop", [False, True])
def test_recurrence_eps1_stop_matches_direct(device_stop, monkeypatch):
    torch = torch_cuda()
    cfg, t0, taps, phi, sp, p, A, AT, lam_tv, lam_l1, alpha1 = _problem("c1")
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    pt = torch.from_numpy(p).cuda()
    o = dict(lambda_tv=lam_tv, lambda_l1=lam_l1, k1=400, k2=6, alpha1=alpha1, eps1=1e-5,
             trace=True, device_stop=device_stop)
    out = {}
    for direct in ("1", "0"):
        monkeypatch.setenv("PSOAM_OBJ_DIRECT", direct)
        out[direct] = plan.solve(pt, **o)
    (cd, sd, trd), (cr, sr, trr) = out["1"], out["0"]
    say(f"[objective] eps1 stop (device {device_stop}): direct {sd['iterations']}, "
        f"recurrence {sr['iterations']}")
    assert 3 <= sd["iterations"] < o["k1"]
    assert sr["iterations"] == sd["iterations"]
    assert torch.equal(cd, cr)
    np.testing.assert_allclose(trr, trd, rtol=1e-6)
    plan.close()
