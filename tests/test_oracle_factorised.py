"""Pins of the oracle's factorised acoustic operator (Sec. 2.2.3 "Acoustic
Model": unit-weight discrete semicircles, eqs. q-above-final, q-below-final;
the temporal convolution of eq. acoustic-temporal-conv):

- the shell membership rule against spheres sampled densely point by point
  (every voxel a sampled point falls in is a member; every member has a
  sampled point within the sampling gap of its box), on both sides of the
  focal plane, for even and odd depth counts;
- the radius-0 sample (the focal point) against the voxel that holds it;
- the convolution convention against a unit impulse;
- the whole factorised operator against the already pinned band form of its
  composition, whose columns are built here with numpy.convolve, for a
  random asymmetric spatial response, an off-centre asymmetric impulse
  response and per-voxel switching; and its adjoint identity.
"""
import numpy as np
import pytest

import oracle


def _sphere_points(radius, h):
    """Points on a sphere of the given radius with neighbour gaps <= ~h
    (latitude rings, each ring sampled uniformly)."""
    if radius == 0.0:
        return np.zeros((1, 3))
    n_lat = max(2, int(np.ceil(np.pi * radius / h)) + 1)
    pts = []
    for th in np.linspace(0.0, np.pi, n_lat):
        ring = radius * np.sin(th)
        n_lon = max(1, int(np.ceil(2 * np.pi * ring / h)))
        ph = np.arange(n_lon) * (2 * np.pi / n_lon)
        pts.append(np.stack([ring * np.cos(ph), ring * np.sin(ph),
                             np.full(n_lon, radius * np.cos(th))], axis=1))
    return np.concatenate(pts)            # columns: y, x, z offsets from the focus


@pytest.mark.parametrize("nz,z_focus", [(8, 3.5), (7, 3.0)])
def test_shell_mask_matches_sampled_spheres(nz, z_focus):
    f, nt, dr, t_focus = 7, 22, 0.6, 11
    R = (f - 1) // 2
    h = 0.05
    mask = oracle.shell_mask(nz, f, nt, dr, z_focus, t_focus)
    for t in range(nt):
        rho = abs(t - t_focus) * dr
        pts = _sphere_points(rho, h)
        lower = t >= t_focus
        # the half sphere of this sample: voxels on the matching side of the
        # focal plane (by their centre depth)
        vy = np.rint(pts[:, 0]).astype(int)
        vx = np.rint(pts[:, 1]).astype(int)
        vz = np.rint(pts[:, 2] + z_focus).astype(int)
        ok = (np.abs(vy) <= R) & (np.abs(vx) <= R) & (vz >= 0) & (vz < nz)
        side = (vz - z_focus >= 0) if lower else (vz - z_focus < 0)
        ok &= side
        # skip points on a box face (rounding there is a tie)
        frac = np.abs(np.stack([pts[:, 0], pts[:, 1], pts[:, 2] + z_focus], 1) % 1.0 - 0.5)
        ok &= frac.min(axis=1) > 1e-9
        hit = np.zeros((nz, f, f), dtype=bool)
        hit[vz[ok], vy[ok] + R, vx[ok] + R] = True
        assert not (hit & ~mask[t]).any(), f"sample {t}: a crossed voxel is missing"
        # every member is within the sampling gap of the sphere
        mem = np.argwhere(mask[t])                       # (z, jy, jx)
        centres = np.stack([mem[:, 1] - R, mem[:, 2] - R, mem[:, 0] - z_focus], axis=1)
        for k in range(0, len(centres), 16):
            c = centres[k:k + 16]
            d = np.maximum(np.abs(pts[:, None, :] - c[None, :, :]) - 0.5, 0.0)
            dist = np.sqrt((d * d).sum(axis=2)).min(axis=0)
            assert (dist <= h).all(), (t, mem[k:k + 16][dist > h])
        # the sides never mix
        dz = np.arange(nz) - z_focus
        assert not mask[t][(dz < 0) if lower else (dz >= 0)].any()


@pytest.mark.parametrize("nz,z_focus,expect_z", [(8, 3.5, 4), (7, 3.0, 3)])
def test_focal_sample_is_the_voxel_holding_the_focus(nz, z_focus, expect_z):
    """Radius 0 (the focal spot, where the signal is the initial pressure
    there): one member, the voxel whose box holds the focal point on the
    lower side (the sign of 0 taken as +1)."""
    f = 5
    mask = oracle.shell_mask(nz, f, 12, 0.6, z_focus, 6)
    members = list(zip(*np.nonzero(mask[6])))
    assert members == [(expect_z, 2, 2)]


def test_eir_conv_of_an_impulse_is_the_shifted_response():
    v = np.array([0.3, -1.0, 0.7, 0.2])
    q = np.zeros((1, 1, 1, 20))
    q[..., 9] = 1.0
    p = oracle.eir_conv(q, v, 1)
    expect = np.zeros(20)
    expect[9 - 1:9 - 1 + 4] = v                     # p[9 + j - origin] = v[j]
    np.testing.assert_array_equal(p[0, 0, 0], expect)
    # the adjoint pairs with it exactly
    rng = np.random.default_rng(1)
    a, b = rng.standard_normal((2, 3, 2, 2, 20))
    assert np.vdot(oracle.eir_conv(a, v, 1), b) == pytest.approx(np.vdot(a, oracle.eir_corr(b, v, 1)),
                                                                 rel=1e-13)


def _composed_band(spr, mask, v, origin):
    """Band form of V Lambda: column (z, jdy, jdx) is the impulse response
    convolved (numpy.convolve) with eta times the column's shell indicator;
    stored over the whole A-scan (t0 = 0, width Nt)."""
    nt, nz, f = mask.shape[0], mask.shape[1], mask.shape[2]
    taps = np.zeros((nz, f, f, nt))
    for z in range(nz):
        for jy in range(f):
            for jx in range(f):
                lam = mask[:, z, jy, jx] * float(spr[z, jy, jx])
                full = np.convolve(lam, v)              # full[m] = sum_j v[j] lam[m - j]
                taps[z, jy, jx] = full[origin:origin + nt]
    return np.zeros((nz, f, f), dtype=np.int64), taps


@pytest.mark.parametrize("per_voxel", [True, False])
def test_factorised_operator_equals_band_form_of_its_composition(per_voxel):
    rng = np.random.default_rng(31)
    ny, nx, nz, f, nt, K, S_n = 5, 6, 6, 5, 18, 3, 2
    mask = oracle.shell_mask(nz, f, nt, 0.55, 2.5, 8)
    spr = rng.uniform(0.1, 1.0, size=(nz, f, f))           # asymmetric in dy, dx and z
    v = np.array([0.4, -1.0, 0.6, 0.25, -0.1])
    origin = 1
    S = rng.uniform(0.1, 1.0, size=((ny, nx, nz) if per_voxel else (nz,)) + (K, S_n))
    c = rng.standard_normal((S_n, ny, nx, nz))
    y = rng.standard_normal((K, ny, nx, nt))
    t0, taps = _composed_band(spr, mask, v, origin)
    np.testing.assert_allclose(oracle.apply_A_fact(c, S, spr, mask, v, origin),
                               oracle.apply_A(c, S, t0, taps, nt), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.apply_AT_fact(y, S, spr, mask, v, origin),
                               oracle.apply_AT(y, S, t0, taps, nz), rtol=1e-12, atol=1e-12)
    # sampled forms agree with the whole operator
    scans = [(0, 0), (4, 5), (2, 3)]
    full = oracle.apply_A_fact(c, S, spr, mask, v, origin)
    got = oracle.apply_A_fact_scans(c, S, spr, mask, v, origin, scans)
    np.testing.assert_allclose(got, np.stack([full[:, a, b] for a, b in scans]), rtol=1e-12,
                               atol=1e-12)
    fullT = oracle.apply_AT_fact(y, S, spr, mask, v, origin)
    gotT = oracle.apply_AT_fact_columns(y, S, spr, mask, v, origin, scans)
    np.testing.assert_allclose(gotT, np.stack([fullT[:, a, b] for a, b in scans]), rtol=1e-12,
                               atol=1e-12)
    # adjoint identity
    lhs = np.vdot(oracle.apply_A_fact(c, S, spr, mask, v, origin), y)
    rhs = np.vdot(c, oracle.apply_AT_fact(y, S, spr, mask, v, origin))
    assert lhs == pytest.approx(rhs, rel=1e-12)
