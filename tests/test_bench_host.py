"""Host logic of bench.py (no GPU): the one-GPU guard, and the gate that
reports the profiled HBM traffic only while the kernel sources hash to the
ones the counters were taken from."""
import hashlib
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = ("psoam_kernels.hip", "psoam_plan.cpp", "psoam_internal.h")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _sources(tmp_path):
    """A copy of the kernel sources under a scratch root."""
    csrc = tmp_path / "paper_2510_23739_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in SOURCES:
        shutil.copy(os.path.join(ROOT, "paper_2510_23739_amd", "csrc", f), csrc / f)
    (tmp_path / "profiles").mkdir()
    return csrc


def _sha(csrc):
    h = hashlib.sha1()
    for f in SOURCES:
        h.update((csrc / f).read_bytes())
    return h.hexdigest()


@pytest.fixture()
def bench(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench as b
    yield b
    sys.path.remove(ROOT)


def test_profiled_traffic_follows_the_source_hash(tmp_path, monkeypatch, bench):
    csrc = _sources(tmp_path)
    name = "band16_lds_adj_C5_bf16_hbm.md"
    (tmp_path / "profiles" / name).write_text(
        f"# counters\n\n- hbm_bytes_per_launch: 5.5e+09\n- source_sha1: `{_sha(csrc)}`\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    val, src = bench.profiled_traffic(name)
    assert val == pytest.approx(5.5e9)
    assert src.endswith(name)
    # any edit of a kernel source voids the figure
    with open(csrc / "psoam_plan.cpp", "a") as fh:
        fh.write("\n")
    val, why = bench.profiled_traffic(name)
    assert val is None and "changed" in why


def test_profiled_traffic_without_a_summary(tmp_path, monkeypatch, bench):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    val, why = bench.profiled_traffic("band16_lds_H_C2_bf16_hbm.md")
    assert val is None and "no counter summary" in why


def test_algorithmic_flops_count_in_grid_pairs(bench):
    """The roofline numerator counts, per lateral offset, the band nonzeros
    times the scans whose voxel at that offset is inside the grid: brute force
    over scans and offsets on a small table."""
    import numpy as np

    import synth
    cfg = synth.Config("t", nx=9, ny=6, nz=5, n_species=2, n_pulses=3, nt=20, f=5, k1=1)
    rng = np.random.default_rng(0)
    t0, taps = synth.random_table(cfg.nz, cfg.f, cfg.nt, 4, rng, t0_lo=-3, t0_hi=cfg.nt)
    taps[0, 1, 2, :] = 0.0
    r = cfg.r
    count = 0
    for iy in range(cfg.ny):
        for ix in range(cfg.nx):
            for jdy in range(cfg.f):
                for jdx in range(cfg.f):
                    if not (0 <= iy + jdy - r < cfg.ny and 0 <= ix + jdx - r < cfg.nx):
                        continue
                    for z in range(cfg.nz):
                        for j in range(taps.shape[-1]):
                            t = t0[z, jdy, jdx] + j
                            count += int(taps[z, jdy, jdx, j] != 0 and 0 <= t < cfg.nt)
    assert bench.alg_flops(cfg, t0, taps) == 2.0 * cfg.n_pulses * count


def test_argument_defaults_name_the_largest_workload(bench):
    a = bench.parse([])
    assert a.workload == "C5" and a.gpus == 1 and a.prec == "bf16"
