"""The launch-shape autotuner (psoam_plan_create_tuned): the tuned plan
applies the same operator as the default plan (the shape changes which rows
a workgroup holds, H's loader waves, the H^T operand's sample offset and the
TV step's tile, not the products; with another offset the band's octet
grouping and so the summation order can differ, hence a rounding-level
tolerance), its report matches the plan it returns, a second creation with
the same inputs takes the cached choice without timing, and a creation that
does not consult the process's cache (as a new process) reads the choice
from the disk cache."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import lib_plan, nan_buf, ragged_cfg, say, torch_cuda

pytestmark = pytest.mark.gpu

TV_TILES = ([8, 8, 32, 512], [4, 8, 32, 256], [4, 16, 32, 512], [4, 8, 64, 512], [8, 8, 32, 1024])


@pytest.fixture(autouse=True)
def _tune_file(tmp_path_factory, monkeypatch):
    # a disk cache of this module's own, empty at the start of the session
    path = tmp_path_factory.getbasetemp() / "psoam_tune.txt"
    monkeypatch.setenv("PSOAM_TUNE_CACHE", str(path))
    return path


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
    assert rep["h_rows"] in (4, 8, 12) and rep["ht_rows"] in (4, 8, 12) and rep["ht_shift"] in (0, 4)
    assert rep["h_loaders"] in (0, 4) and rep["tv_tile"] in TV_TILES
    assert tuned.stats()["lds_rows"] == [rep["h_rows"], rep["ht_rows"]]
    if not rep["from_cache"]:
        assert rep["candidates"] >= 2 + len(TV_TILES) - 1
        assert 0.0 < rep["h_ms"] <= rep["h_ms_default"]
        assert 0.0 < rep["ht_ms"] <= rep["ht_ms_default"]
        assert 0.0 < rep["tv_ms"] <= rep["tv_ms_default"]
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
    keys = ("h_rows", "ht_rows", "ht_shift", "h_loaders", "tv_tile", "fp32_runs")
    assert [r2[k] for k in keys] == [rep[k] for k in keys]
    for p in (base, tuned, again):
        p.close()


def test_disk_cache_serves_a_later_creation(_tune_file, monkeypatch):
    """A tuned plan writes its choice to the disk cache; a later creation with
    the same inputs that does not consult this process's cache (as a fresh
    process would not) takes it from the file (from_cache 2) without timing,
    and a line for other inputs does not match."""
    torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, t0, taps, phi, sp = _inputs("ragged")
    first = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec="fp16", tune=True)
    rep = first.tune_report
    first.close()
    lines = open(_tune_file).read().splitlines()
    say(f"[tune] disk cache {_tune_file}: {len(lines)} lines, last {lines[-1]!r}")
    assert lines and all("\t" in ln for ln in lines)
    monkeypatch.setenv("PSOAM_TUNE_MEMO", "0")
    again = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec="fp16", tune=True)
    r2 = again.tune_report
    again.close()
    say(f"   from the file: {r2}")
    assert r2["from_cache"] == 2 and r2["candidates"] == 0
    keys = ("h_rows", "ht_rows", "ht_shift", "h_loaders", "tv_tile", "fp32_runs")
    assert [r2[k] for k in keys] == [rep[k] for k in keys]
    # other inputs (another table): not in the file, so tuned afresh
    cfg2, t02, taps2, phi2, sp2 = ragged_cfg(13)
    other = pk.Plan.from_config(cfg2, phi2, sp2, t02, taps2, prec="fp16", tune=True)
    assert other.tune_report["from_cache"] == 0 and other.tune_report["candidates"] >= 2
    other.close()


@pytest.mark.parametrize("which", ["c1", "ragged"])
def test_fp32_plan_tunes_its_kernel(which):
    """FP32 plans: the tuner times the run-packed and the per-tile kernel for
    H and H^T and the TV tiles; the tuned plan applies the same operator as
    the default one up to the summation order of the other kernel."""
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    cfg, t0, taps, phi, sp = _inputs(which)
    base = lib_plan(cfg, t0, taps, phi, sp, "fp32")
    p = pk.Plan.from_config(cfg, phi, sp, t0, taps, prec="fp32", tune=True)
    rep = p.tune_report
    say(f"[tune] fp32 {which}: {rep}")
    assert rep["h_rows"] == 0 and rep["ht_rows"] == 0
    assert all(x in (0, 1) for x in rep["fp32_runs"]) and rep["tv_tile"] in TV_TILES
    if not rep["from_cache"]:
        assert rep["candidates"] >= 2 + len(TV_TILES) - 1
        assert 0.0 < rep["h_ms"] <= rep["h_ms_default"]
        assert 0.0 < rep["ht_ms"] <= rep["ht_ms_default"]
    rng = np.random.default_rng(10)
    c = torch.from_numpy(rng.standard_normal(cfg.c_shape).astype(np.float32)).cuda()
    y = torch.from_numpy(rng.standard_normal(cfg.y_shape).astype(np.float32)).cuda()
    e = [oracle.rel_err(p.apply_A(c).cpu().numpy(), base.apply_A(c).cpu().numpy()),
         oracle.rel_err(p.apply_AT(y).cpu().numpy(), base.apply_AT(y).cpu().numpy())]
    say(f"   tuned vs default: A {e[0]:.2e}  A^T {e[1]:.2e}")
    assert max(e) <= 1e-6
    base.close()
    p.close()
