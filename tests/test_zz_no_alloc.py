"""psoam_prox_tv_noalloc, the TV prox for callers that cannot allocate device
memory: through the C ABI, against psoam_prox_tv with a caller workspace (the
same kernels in the same order, so the results must be equal bit for bit), on
two calls in a row, the second on a smaller grid, then the first grid again;
the device's free memory does not change across calls after the first; a
grid beyond the static buffer's limit is rejected with EINVAL."""
import numpy as np
import pytest

import synth
from gpu_common import say, torch_cuda

pytestmark = pytest.mark.gpu


def _plan(nx, ny, nz, ns):
    import paper_2510_23739_amd as pk
    cfg = synth.Config("na", nx=nx, ny=ny, nz=nz, n_species=ns, n_pulses=2, nt=16, f=3, k1=1)
    t0, taps = synth.random_table(nz, 3, 16, 4, np.random.default_rng(nz), t0_lo=0, t0_hi=12)
    return pk.Plan.from_config(cfg, synth.phi_depth(nz), synth.species(ns), t0, taps,
                               prec="fp32"), cfg


def _pair(torch, plan, cfg, seed, theta, k2, nonneg):
    z = torch.from_numpy(np.random.default_rng(seed).standard_normal(cfg.c_shape)
                         .astype(np.float32)).cuda()
    x_ws = plan.prox_tv(z, theta, k2, nonneg=nonneg)
    x_na = torch.full_like(z, float("nan"))
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan.prox_tv_noalloc(z, theta, k2, nonneg=nonneg, x=x_na)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return x_ws, x_na, free0, free1


def test_noalloc_prox_tv_matches_workspace_form():
    torch = torch_cuda()
    big, cfg_big = _plan(32, 32, 40, 2)     # two depth tiles
    small, cfg_small = _plan(13, 7, 11, 3)  # every size off the tile grid
    # first call on this device (looks up the static buffer's address)
    big.prox_tv_noalloc(torch.zeros(cfg_big.c_shape, device="cuda"), 0.1, 2,
                        x=torch.empty(cfg_big.c_shape, device="cuda"))
    for label, plan, cfg, seed, theta, k2, nonneg in (
            ("32x32x40", big, cfg_big, 1, 0.1, 20, True),
            ("13x7x11 (smaller)", small, cfg_small, 2, 0.3, 15, False),
            ("32x32x40 again", big, cfg_big, 3, 0.05, 9, False)):
        x_ws, x_na, free0, free1 = _pair(torch, plan, cfg, seed, theta, k2, nonneg)
        say(f"[no-alloc] {label}: equal {bool(torch.equal(x_ws, x_na))}, "
            f"max |diff| {float((x_ws - x_na).abs().max()):.3e}, free memory change {free1 - free0}")
        assert torch.equal(x_ws, x_na)
        assert free1 == free0
    big.close()
    small.close()


def test_noalloc_rejects_grids_beyond_the_limit():
    torch = torch_cuda()
    import paper_2510_23739_amd as pk
    plan, cfg = _plan(128, 128, 80, 3)      # 3 x 128 x 128 x 80 = 3932160 > 3728256
    z = torch.zeros(cfg.c_shape, device="cuda")
    with pytest.raises(pk.PsoamError) as ei:
        plan.prox_tv_noalloc(z, 0.1, 5, x=torch.empty_like(z))
    say(f"[no-alloc] oversize: {ei.value}")
    assert ei.value.code == 1 and "exceeds" in str(ei.value)
    plan.close()
