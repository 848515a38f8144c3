"""The launch-shape autotuner (psoam_plan_create_tuned): the tuned plan
applies the same operator as the default plan (the shape changes which rows
a workgroup holds and the H^T operand's sample offset, not the products; with
another offset the band's octet grouping and so the summation order can
differ, hence a rounding-level tolerance), its report matches the plan it
returns, and a second creation with the same inputs takes the cached choice
without timing."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, nan_buf, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu


def _inputs(which):
    if which == "c1":
        cfg = synth.C1
        _, t0, taps, phi, sp, _, _ = synth.inputs(cfg)
        return cfg, t0, taps, phi, sp
    return ragged_cfg(8)


@pytest.mark.parametrize("prec", ["bf16", "fp16_split"])
@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_tuned_plan_matches_default(which, prec):
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, t0, taps, phi, sp = _inputs(which)
    say(f"[tune] {which} {prec}")
    base = lib_plan(cfg, t0, taps, phi, sp, prec)
    tuned = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=prec, tune=True)
    rep = tuned.tune_report
    say(f"   report {rep}")
    assert rep["h_rows"] in (4, 8) and rep["ht_rows"] in (4, 8) and rep["ht_shift"] in (0, 4)
    assert tuned.stats()["lds_rows"] == [rep["h_rows"], rep["ht_rows"]]
    if not rep["from_cache"]:
        assert rep["candidates"] >= 2
        assert 0.0 < rep["h_ms"] <= rep["h_ms_default"]
        assert 0.0 < rep["ht_ms"] <= rep["ht_ms_default"]
    rng = np.random.default_rng(9)
    c = torch.from_numpy(rng.standard_normal(cfg.c_shape).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.standard_normal(cfg.y_shape).astype(np.float32)).cuda()
    ya, yb = base.apply_A(c, nan_buf(cfg.y_shape)), tuned.apply_A(c, nan_buf(cfg.y_shape))
    ga, gb = base.apply_AT(y, nan_buf(cfg.c_shape)), tuned.apply_AT(y, nan_buf(cfg.c_shape))
    o = dict(lambda_tv=0.05, lambda_l1=0.02, k1=4, k2=4, alpha1=1e-3)
    ca, _ = base.solve(y, **o)
    cb, _ = tuned.solve(y, **o)
    e = [oracle.rel_err(b.cpu().numpy(), a.cpu().numpy()) for a, b in ((ya, yb), (ga, gb), (ca, cb))]
    say(f"   tuned vs default: A {e[0]:.2e}  A^T {e[1]:.2e}  solve {e[2]:.2e}")
    assert max(e) <= 1e-5
    # the same inputs again: the cached choice, nothing timed
    again = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec=prec, tune=True)
    r2 = again.tune_report
    assert r2["from_cache"] == 1 and r2["candidates"] == 0
    assert (r2["h_rows"], r2["ht_rows"], r2["ht_shift"]) == (rep["h_rows"], rep["ht_rows"],
                                                            rep["ht_shift"])
    for p in (base, tuned, again):
        p.close()


def test_fp32_plan_is_built_untuned():
    torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, t0, taps, phi, sp = _inputs("ragged")
    p = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec="fp32", tune=True)
    assert p.tune_report["candidates"] == 0 and p.tune_report["from_cache"] == 0
    p.close()
