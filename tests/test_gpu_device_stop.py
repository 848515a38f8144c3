"""Device-side stopping tests (psoam_solve_opts.device_stop): the two tests
of Alg. alg:prox-outer (relative objective change below eps1, relative change
of the momentum iterate below eps2) evaluated by a one-thread kernel after
each iteration, whose flag every later kernel of the solve checks.  Against
the host-side tests: the same iteration count, the same concentrations bit
for bit, the same objective trace; against the oracle's stopping iteration
(within one, as for the host tests); and inside the batched, graph-captured
solves, where each problem stops on its own flag while the others run on."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, oracle_S, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    cfg = synth.C1
    c_true, t0, taps, phi, sp, n0, v0 = synth.inputs(cfg)
    S = oracle_S(cfg, phi, sp)
    A = lambda v: oracle.apply_A(v, S, t0, taps, cfg.nt)
    AT = lambda w: oracle.apply_AT(w, S, t0, taps, cfg.nz)
    y = A(c_true.astype(np.float64))
    p = (y + synth.noise_sigma(float(np.sqrt(np.mean(y ** 2)))) * n0).astype(np.float32)
    alpha1 = 1.0 / (1.01 * oracle.power_iteration(A, AT, v0, 30))
    aty = float(np.abs(AT(p.astype(np.float64))).max())
    return cfg, t0, taps, phi, sp, p, A, AT, alpha1, 5e-3 * aty, 1e-2 * aty


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("which", ["eps2", "eps1_trace"])
def test_device_tests_match_host_tests(c1, prec, which):
    torch = torch_cuda()
    cfg, t0, taps, phi, sp, p, A, AT, alpha1, lam_tv, lam_l1 = c1
    plan = lib_plan(cfg, t0, taps, phi, sp, prec)
    pt = torch.from_numpy(p).cuda()
    o = dict(lambda_tv=lam_tv, lambda_l1=lam_l1, k1=400, k2=6, alpha1=alpha1)
    if which == "eps2":
        o["eps2"] = 2e-3
    else:
        o.update(eps1=1e-5, trace=True)
    out = {}
    for dev in (False, True):
        r = plan.solve(pt, device_stop=dev, **o)
        out[dev] = r
    (ch, sh), (cd, sd) = out[False][:2], out[True][:2]
    say(f"[device-stop] {which} {prec}: host {sh['iterations']} iterations, device "
        f"{sd['iterations']}, c equal {bool(torch.equal(ch, cd))}")
    assert 3 <= sh["iterations"] < o["k1"]
    assert sd["iterations"] == sh["iterations"]
    assert torch.equal(ch, cd)
    if which == "eps1_trace":
        np.testing.assert_array_equal(out[True][2], out[False][2])
        assert sd["objective"] == sh["objective"]
    plan.close()


def test_device_eps2_stop_matches_oracle(c1):
    """The xi-change test fires within one iteration of the oracle's."""
    torch = torch_cuda()
    cfg, t0, taps, phi, sp, p, A, AT, alpha1, lam_tv, lam_l1 = c1
    _, it_ref = oracle.fista(p.astype(np.float64), A, AT, alpha1, 0.0, 0.0, 400, 1, eps2=1e-3,
                             shape_c=cfg.c_shape)
    plan = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    _, st = plan.solve(torch.from_numpy(p).cuda(), k1=400, k2=1, alpha1=alpha1, eps2=1e-3,
                       device_stop=True)
    say(f"[device-stop] eps2 1e-3: device {st['iterations']}, oracle {it_ref}")
    assert abs(st["iterations"] - it_ref) <= 1
    plan.close()


def test_batch_captures_stopping_problems(c1):
    """Problems with stopping tests run captured in the batch under
    device_stop and give the one-by-one host-tested results: iterations and
    concentrations, bitwise; a problem without tests runs its full count
    beside them."""
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, t0, taps, phi, sp, p, A, AT, alpha1, lam_tv, lam_l1 = c1
    probs = [(cfg, t0, taps, phi, sp, "bf16", torch.from_numpy(p).cuda(),
              dict(lambda_tv=lam_tv, lambda_l1=lam_l1, k1=300, k2=5, alpha1=alpha1, eps2=5e-3))]
    cfg2, t02, taps2, phi2, sp2 = ragged_cfg(4)
    rng = np.random.default_rng(41)
    p2 = torch.from_numpy(rng.standard_normal(cfg2.y_shape).astype(np.float32)).cuda()
    probs.append((cfg2, t02, taps2, phi2, sp2, "fp32", p2,
                  dict(lambda_tv=1e-3, lambda_l1=1e-3, k1=250, k2=4, n_power=10, eps1=1e-5)))
    cfg3 = synth.Config("u5", 21, 19, 12, 2, 9, 48, 5, k1=9, k2=3, seed=79)
    t03, taps3 = synth.sir_table(cfg3.nz, cfg3.f, cfg3.nt)
    p3 = torch.from_numpy(rng.standard_normal(cfg3.y_shape).astype(np.float32)).cuda()
    probs.append((cfg3, t03, taps3, synth.phi_depth(cfg3.nz), synth.species(2), "fp16", p3,
                  dict(lambda_tv=1e-3, lambda_l1=1e-3, k1=9, k2=3, alpha1=1e-3)))
    plans, ps, opts, ref = [], [], [], []
    for (cf, a, b, ph, s_, prec, pp, o) in probs:
        plan = lib_plan(cf, a, b, ph, s_, prec)
        c, st = plan.solve(pp, **o)
        ref.append((c.clone(), st["iterations"]))
        plans.append(plan)
        ps.append(pp)
        opts.append(dict(o, device_stop=True))
    assert ref[0][1] < 300 and ref[2][1] == 9
    for call in range(2):
        cs = [torch.zeros(pl.c_shape, dtype=torch.float32, device="cuda") for pl in plans]
        stats = pk.solve_batch(plans, ps, cs, opts)
        torch.cuda.synchronize()
        for i, (c, (r, it), s) in enumerate(zip(cs, ref, stats)):
            say(f"[device-stop] batch call {call} problem {i}: {s['iterations']} iterations "
                f"(alone {it}), equal {bool(torch.equal(c, r))}")
            assert s["iterations"] == it
            assert torch.equal(c, r)
        # eager work on the same plans between the calls
        plans[0].apply_A(torch.zeros(plans[0].c_shape, device="cuda"))
    for pl in plans:
        pl.close()
