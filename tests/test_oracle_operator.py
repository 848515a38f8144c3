"""Pins of the oracle's forward operator A = H S against things other than
the oracle: brute-force matrices built entry by entry, the paper's printed
photo-physics constants, closed forms and invariants."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _tiny(seed=0, ns=2, ny=3, nx=4, nz=3, K=3, nt=10, f=3, width=4, per_voxel=True):
    rng = np.random.default_rng(seed)
    t0, taps = synth.random_table(nz, f, nt, width, rng, t0_lo=-2, t0_hi=nt - 1)
    if per_voxel:
        phi = rng.uniform(0.3, 1.0, size=(ny, nx, nz))
    else:
        phi = rng.uniform(0.3, 1.0, size=nz)
    sp = synth.species(ns, gamma=1.0)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, K)
    c = rng.standard_normal((ns, ny, nx, nz))
    y = rng.standard_normal((K, ny, nx, nt))
    return c, y, S, t0, taps, nt, nz


def test_switching_matrix_matches_photophysics_table():
    """At the first pulse the extinction is eps_ON, and it decays to eps_OFF
    (eq. epsilon); the fluence multiplies the deposited energy (eq. final-H).
    The species constants are the printed Table tab:photophysics values."""
    tab = json.load(open(os.path.join(GOLDEN, "photophysics_table.json")))
    sp = synth.species(2, gamma=0.0)
    for s, name in enumerate(("A", "B")):
        assert sp.a[s] == pytest.approx(tab["species"][name]["eps_off"], rel=1e-12)
        assert sp.a[s] + sp.b[s] == pytest.approx(tab["species"][name]["eps_on"], rel=1e-12)
    phi = np.array([1.0, 0.5, 0.2])
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, 0.0, 400)
    for s, name in enumerate(("A", "B")):
        on, off = tab["species"][name]["eps_on"], tab["species"][name]["eps_off"]
        np.testing.assert_allclose(S[:, 0, s], phi * on, rtol=1e-12)
        np.testing.assert_allclose(S[:, -1, s], phi * off, rtol=1e-9)
        # strictly decreasing from ON toward OFF over the first pulses
        assert np.all(np.diff(S[:, :40, s], axis=1) < 0)


def test_switching_matrix_special_cases():
    phi = np.array([1.0, 0.7, 0.3])
    # b_s = 0: no switching, S = Phi * a for every pulse (the non-switching background)
    S = oracle.switching_matrix(phi, [2.0e-3], [0.0], [3.0], 1.0, 6)
    np.testing.assert_allclose(S[..., 0], np.outer(phi, np.ones(6)) * 2.0e-3, rtol=1e-15)
    # gamma = 0 and gamma = 1 coincide where Phi = 1, differ elsewhere
    sp = synth.species(3)
    S0 = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, 0.0, 8)
    S1 = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, 1.0, 8)
    np.testing.assert_allclose(S0[0], S1[0], rtol=1e-15)
    assert np.abs(S0[2] - S1[2]).max() > 1e-5
    # explicit value: Phi*(a + b*exp(-k*Phi^gamma/tau))
    k, s, z = 5, 1, 2
    expect = phi[z] * (sp.a[s] + sp.b[s] * np.exp(-k * phi[z] / sp.tau[s]))
    assert S1[z, k, s] == pytest.approx(expect, rel=1e-14)


@pytest.mark.parametrize("per_voxel", [True, False])
def test_A_matches_bruteforce_dense_matrix(per_voxel):
    """Random asymmetric band table, taps running off both ends of the A-scan,
    per-voxel or per-depth fluence: A and A^T equal the entry-by-entry matrix."""
    c, y, S, t0, taps, nt, nz = _tiny(per_voxel=per_voxel)
    K = y.shape[0]
    M = oracle.dense_A(c.shape, K, nt, S, t0, taps)
    np.testing.assert_allclose(oracle.apply_A(c, S, t0, taps, nt).ravel(), M @ c.ravel(),
                               rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.apply_AT(y, S, t0, taps, nz).ravel(), M.T @ y.ravel(),
                               rtol=1e-12, atol=1e-12)


def test_adjoint_identity():
    c, y, S, t0, taps, nt, nz = _tiny(seed=3, ny=5, nx=6, nz=4, nt=16, f=5, width=5)
    lhs = np.vdot(oracle.apply_A(c, S, t0, taps, nt), y)
    rhs = np.vdot(c, oracle.apply_AT(y, S, t0, taps, nz))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_point_source_equals_impulse_response():
    """A unit concentration at one voxel produces, at every scan within the
    footprint, the synthesised impulse response of that offset times the
    switching curve, and nothing elsewhere."""
    cfg = synth.C1
    t0, taps = synth.sir_table(cfg.nz, cfg.f, cfg.nt)
    phi = synth.phi_depth(cfg.nz)
    sp = synth.species(cfg.n_species)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, cfg.n_pulses)
    s0, y0, x0, z0 = 1, 10, 13, 5
    c = np.zeros(cfg.c_shape)
    c[s0, y0, x0, z0] = 1.0
    y = oracle.apply_A(c, S, t0, taps, cfg.nt)
    R = cfg.r
    expect = np.zeros_like(y)
    for iy in range(cfg.ny):
        for ix in range(cfg.nx):
            jdy, jdx = y0 - iy + R, x0 - ix + R
            if 0 <= jdy < cfg.f and 0 <= jdx < cfg.f:
                for j in range(taps.shape[-1]):
                    t = t0[z0, jdy, jdx] + j
                    if 0 <= t < cfg.nt:
                        expect[:, iy, ix, t] = S[z0, :, s0] * taps[z0, jdy, jdx, j]
    np.testing.assert_allclose(y, expect, rtol=1e-13, atol=1e-18)


def test_identity_special_case():
    """F = 1, Nt = Nz, h[z][0][0][t] = delta_tz and S = I give A = I."""
    rng = np.random.default_rng(5)
    nz = 7
    t0 = np.arange(nz, dtype=np.int32).reshape(nz, 1, 1)
    taps = np.zeros((nz, 1, 1, 3), dtype=np.float32)
    taps[:, 0, 0, 0] = 1.0
    S = np.broadcast_to(np.eye(2), (nz, 2, 2)).copy()
    c = rng.standard_normal((2, 4, 5, nz))
    np.testing.assert_array_equal(oracle.apply_A(c, S, t0, taps, nz), c)
    np.testing.assert_array_equal(oracle.apply_AT(c, S, t0, taps, nz), c)


def test_lateral_translation_equivariance():
    c, _, S, t0, taps, nt, nz = _tiny(seed=7, ny=12, nx=12, nz=3, per_voxel=False)
    c[:] = 0
    rng = np.random.default_rng(1)
    c[:, 4:6, 4:7, :] = rng.standard_normal((c.shape[0], 2, 3, nz))
    cs = np.roll(np.roll(c, 2, axis=1), 3, axis=2)
    y = oracle.apply_A(c, S, t0, taps, nt)
    ys = oracle.apply_A(cs, S, t0, taps, nt)
    np.testing.assert_allclose(ys[:, 3:10, 4:12], y[:, 1:8, 1:9], rtol=1e-13, atol=1e-15)


def test_sampled_outputs_match_full_operator():
    c, y, S, t0, taps, nt, nz = _tiny(seed=11, ny=8, nx=9, nz=4, nt=20, f=5, width=5)
    scans = [(0, 0), (3, 4), (7, 8), (2, 8)]
    full = oracle.apply_A(c, S, t0, taps, nt)
    part = oracle.apply_A_scans(c, S, t0, taps, nt, scans)
    for n, (iy, ix) in enumerate(scans):
        np.testing.assert_allclose(part[n], full[:, iy, ix, :], rtol=1e-12, atol=1e-13)
    fullT = oracle.apply_AT(y, S, t0, taps, nz)
    partT = oracle.apply_AT_columns(y, S, t0, taps, nz, scans)
    for n, (jy, jx) in enumerate(scans):
        np.testing.assert_allclose(partT[n], fullT[:, jy, jx, :], rtol=1e-12, atol=1e-13)
    # per-depth S as well
    _, _, Sd, _, _, _, _ = _tiny(seed=11, ny=8, nx=9, nz=4, nt=20, f=5, width=5, per_voxel=False)
    fulld = oracle.apply_A(c, Sd, t0, taps, nt)
    partd = oracle.apply_A_scans(c, Sd, t0, taps, nt, scans)
    np.testing.assert_allclose(partd[1], fulld[:, 3, 4, :], rtol=1e-12, atol=1e-13)


def test_power_iteration_matches_lapack():
    c, _, S, t0, taps, nt, nz = _tiny(seed=13)
    K = S.shape[-2]
    M = oracle.dense_A(c.shape, K, nt, S, t0, taps)
    lam_exact = np.linalg.eigvalsh(M.T @ M)[-1]
    v0 = np.random.default_rng(2).standard_normal(c.shape)
    lam = oracle.power_iteration(lambda v: oracle.apply_A(v, S, t0, taps, nt),
                                 lambda w: oracle.apply_AT(w, S, t0, taps, nz), v0, 300)
    assert lam == pytest.approx(lam_exact, rel=1e-6)
    # identity operator: eigenvalue 1
    lam1 = oracle.power_iteration(lambda v: v, lambda v: v, v0, 3)
    assert lam1 == pytest.approx(1.0, rel=1e-14)


def test_power_iteration_is_a_lower_bound_on_the_32x32x16_problem():
    """The step of Alg. alg:prox-outer needs eig_max(A^T A); the power
    iteration's Rayleigh quotients approach it from below, never decreasing
    (A^T A is positive semidefinite), so a finite run underestimates it.  On
    the 32x32x16 workload (its seeded Gaussian start) against ARPACK's
    implicitly restarted Lanczos (scipy eigsh), a different method: the 10-,
    30- and 100-step estimates are ordered, below the Lanczos value, and the
    100-step one within 0.5% of it.  The top eigenvalues sit close together
    here, which is why 30 steps fall a few percent short."""
    from scipy.sparse.linalg import LinearOperator, eigsh
    cfg = synth.C1
    _, t0, taps, phi, sp, _, v0 = synth.inputs(cfg)
    S = oracle.switching_matrix(np.asarray(phi, np.float64), sp.a, sp.b, sp.tau, sp.gamma,
                                cfg.n_pulses)

    def A(v):
        return oracle.apply_A(v, S, t0, taps, cfg.nt)

    def AT(w):
        return oracle.apply_AT(w, S, t0, taps, cfg.nz)

    n = int(np.prod(cfg.c_shape))
    op = LinearOperator((n, n), dtype=np.float64,
                        matvec=lambda x: AT(A(x.reshape(cfg.c_shape))).ravel())
    lam_max = float(eigsh(op, k=3, which="LA", tol=1e-12, return_eigenvectors=False).max())
    est = [oracle.power_iteration(A, AT, v0, k) for k in (10, 30, 100)]
    assert est[0] <= est[1] <= est[2] <= lam_max * (1 + 1e-10)
    assert est[2] >= lam_max * (1 - 5e-3)


@pytest.mark.parametrize("per_voxel", [True, False])
def test_separable_switching_factorisation(per_voxel):
    """With a fluence-independent rate (gamma = 0) the switching block is
    S_v[k][s] = phi_v T[k][s], T[k][s] = a_s + b_s exp(-k / tau_s), so
    A c = sum_s T[:, s] (x) H(phi c_s) and (A^T y)_s = phi H^T(sum_k T[k][s] y_k):
    the contraction runs over S volumes instead of K (checked against the
    general A and A^T built from the full switching matrix)."""
    rng = np.random.default_rng(4)
    ns, ny, nx, nz, K, nt, f = 3, 4, 5, 4, 6, 12, 3
    t0, taps = synth.random_table(nz, f, nt, 4, rng, t0_lo=-2, t0_hi=nt - 1)
    phi = rng.uniform(0.3, 1.0, size=(ny, nx, nz) if per_voxel else nz)
    sp = synth.species(ns, gamma=0.0)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, K)
    T = np.asarray(sp.a)[None, :] + np.asarray(sp.b)[None, :] * np.exp(
        -np.arange(K)[:, None] / np.asarray(sp.tau)[None, :])
    c = rng.standard_normal((ns, ny, nx, nz))
    y = rng.standard_normal((K, ny, nx, nt))
    ph = np.broadcast_to(phi, (ny, nx, nz))
    h = oracle.apply_H(c * ph[None], t0, taps, nt)                  # [S][Ny][Nx][Nt]
    np.testing.assert_allclose(np.einsum("ks,syxt->kyxt", T, h),
                               oracle.apply_A(c, S, t0, taps, nt), rtol=1e-12, atol=1e-14)
    rt = np.einsum("ks,kyxt->syxt", T, y)
    g = ph[None] * oracle.apply_HT(rt, t0, taps, nz)
    np.testing.assert_allclose(g, oracle.apply_AT(y, S, t0, taps, nz), rtol=1e-12, atol=1e-14)
