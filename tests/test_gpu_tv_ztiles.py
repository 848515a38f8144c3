"""The TV prox (dual iteration of Alg. alg:prox-inner with L = grad) on grids
deeper than one depth tile of the fused dual-step kernel (32 depths): the
backward eta_z plane and the forward w halo cross tile boundaries, and the
XCD-contiguous tile order holds several depth tiles per lateral tile.

Grids: 9 x 13 x 70 (three depth tiles, the last partial, every size off the
8 x 8 lateral tile), 24 x 24 x 128 (the depth of the largest workload), the
full 128 x 128 x 64 volume of the benchmark workload and the full
320 x 320 x 128 volume of the largest one.  Each result is compared with the
oracle's prox_tv normwise and element by element (max-abs error over the
volume, and separately on the depth planes next to each tile boundary).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import nan_buf, say, torch_cuda

pytestmark = pytest.mark.gpu

TOL = 1e-5        # normwise, FP32 dual iteration vs FP64
TOL_MAX = 1e-5    # max-abs, relative to max |x_ref|


def _plan(ny, nx, nz, ns=2):
    import paper_2510_23739_amd as pk
    cfg = synth.Config("tv", nx=nx, ny=ny, nz=nz, n_species=ns, n_pulses=2, nt=16, f=3, k1=1)
    rng = np.random.default_rng(nz)
    t0, taps = synth.random_table(nz, 3, 16, 4, rng, t0_lo=0, t0_hi=12)
    phi = synth.phi_depth(nz)
    return pk.Plan.from_config(cfg, phi, synth.species(ns), t0, taps, prec="fp32"), cfg


def _check(torch, plan, z, theta, k2, nonneg, label, inplace=False):
    zt = torch.from_numpy(z).cuda()
    if inplace:
        plan.prox_tv(zt, theta, k2, nonneg=nonneg, x=zt)
        x = zt.cpu().numpy()
    else:
        x = plan.prox_tv(zt, theta, k2, nonneg=nonneg, x=nan_buf(z.shape)).cpu().numpy()
    ref = oracle.prox_tv(z, theta, k2, nonneg=nonneg)
    e = oracle.rel_err(x, ref)
    scale = float(np.abs(ref).max())
    emax = float(np.abs(x - ref).max()) / scale
    nz = z.shape[-1]
    planes = sorted({p for b in range(32, nz, 32) for p in (b - 1, b) if p < nz} | {nz - 1})
    ebnd = float(np.abs(x[..., planes] - ref[..., planes]).max()) / scale
    say(f"[tv-z] {label} K2={k2} theta={theta} nonneg={nonneg}: rel err {e:.3e}, "
        f"max-abs {emax:.3e}, max-abs at depth-tile planes {planes} {ebnd:.3e}")
    assert np.isfinite(x).all()
    assert e <= TOL and emax <= TOL_MAX and ebnd <= TOL_MAX


@pytest.mark.parametrize("k2,theta,nonneg", [(20, 0.05, False), (50, 0.2, True),
                                             (20, 0.3, True), (50, 0.02, False)])
def test_prox_tv_three_depth_tiles(k2, theta, nonneg):
    torch = torch_cuda()
    plan, cfg = _plan(9, 13, 70)
    rng = np.random.default_rng(k2 + int(1000 * theta))
    z = rng.standard_normal(cfg.c_shape).astype(np.float32)
    # a smooth part too, so the clamp is partly inactive
    z += np.sin(np.arange(cfg.nz) / 9.0).astype(np.float32)
    _check(torch, plan, z, theta, k2, nonneg, "9x13x70")
    plan.close()


def test_prox_tv_three_depth_tiles_in_place():
    torch = torch_cuda()
    plan, cfg = _plan(9, 13, 70)
    z = np.random.default_rng(3).standard_normal(cfg.c_shape).astype(np.float32)
    _check(torch, plan, z, 0.1, 30, True, "9x13x70 in place", inplace=True)
    plan.close()


def test_prox_tv_depth_128():
    torch = torch_cuda()
    plan, cfg = _plan(24, 24, 128, ns=3)
    rng = np.random.default_rng(128)
    z = (rng.standard_normal(cfg.c_shape) * 0.3).astype(np.float32)
    z += synth.phantom(cfg, rng)
    _check(torch, plan, z, 0.05, 50, False, "24x24x128")
    plan.close()


@pytest.mark.parametrize("k2,nonneg", [(20, True), (50, False)])
def test_prox_tv_benchmark_volume(k2, nonneg):
    """The whole 3 x 128 x 128 x 64 volume of the benchmark workload."""
    torch = torch_cuda()
    base = synth.C2
    plan, cfg = _plan(base.ny, base.nx, base.nz, ns=base.n_species)
    rng = np.random.default_rng(2000 + k2)
    z = synth.phantom(base) + (0.2 * rng.standard_normal(base.c_shape)).astype(np.float32)
    _check(torch, plan, z.astype(np.float32), 0.04, k2, nonneg, "128x128x64")
    plan.close()


def test_prox_tv_largest_volume():
    """The whole 3 x 320 x 320 x 128 volume of the largest workload (ten dual
    steps: the oracle's time grows with the volume)."""
    torch = torch_cuda()
    base = synth.C5
    plan, cfg = _plan(base.ny, base.nx, base.nz, ns=base.n_species)
    rng = np.random.default_rng(5000)
    z = (rng.standard_normal(base.c_shape) * 0.3).astype(np.float32)
    z += np.sin(np.arange(base.nz) / 11.0).astype(np.float32)
    _check(torch, plan, z, 0.05, 10, True, "320x320x128")
    plan.close()


@pytest.mark.parametrize("tile", [1, 2, 3, 4])
def test_every_tile_shape_gives_the_default_result(tile, monkeypatch):
    """Each tile shape of the fused dual step (chosen per plan by the
    autotuner) against the default 8 x 8 x 32 tile: every output is the same
    expression of the same inputs, so the prox is equal bit for bit; on the
    ragged 9 x 13 x 70 grid (partial tiles in every direction, and one or
    three depth tiles of 64 or 32) and against the oracle."""
    torch = torch_cuda()
    rng = np.random.default_rng(70 + tile)
    z = rng.standard_normal((2, 9, 13, 70)).astype(np.float32)
    out = {}
    for t in (0, tile):
        monkeypatch.setenv("PSOAM_TV_TILE", str(t))
        plan, cfg = _plan(9, 13, 70)
        zt = torch.from_numpy(z).cuda()
        out[t] = plan.prox_tv(zt, 0.1, 20, nonneg=True, x=nan_buf(z.shape)).cpu().numpy()
        plan.close()
    ref = oracle.prox_tv(z, 0.1, 20, nonneg=True)
    e = oracle.rel_err(out[tile], ref)
    say(f"[tv-z] tile {tile}: rel err {e:.3e}, equal to the default tile "
        f"{bool(np.array_equal(out[0], out[tile]))}")
    np.testing.assert_array_equal(out[0], out[tile])
    assert e <= TOL
