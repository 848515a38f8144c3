"""Pins of the oracle's full one-step regulariser with the TV(S c) term
(eq. reg-tv-l1-one with the stacked operator L and the dual iteration of
Alg. alg:prox-inner): the dual step bound against LAPACK, the converged
iteration against an exact bounded least-squares solve (SciPy BVLS) of the
dual it iterates on, followed by the algorithm's final clamp, the
reductions S = I (TV(S c) is then TV(c)) and theta_tvs = 0 (the exact
composition of the TV prox and the clamped shrink), and monotone descent of
the proximal-gradient iteration with that prox on a tiny dense problem."""
import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle


def _grad_matrix(shape):
    n = int(np.prod(shape))
    G = np.zeros((3 * n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        G[:, j] = oracle.grad(e.reshape(shape)).ravel()
    return G


def _s_matrix(S, shape_c):
    """apply_S as a dense matrix [K*V, S*V], column by column."""
    n = int(np.prod(shape_c))
    cols = []
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        cols.append(oracle.apply_S(e.reshape(shape_c), S).ravel())
    return np.stack(cols, axis=1)


def _random_S(rng, vol, n_k, n_s, per_voxel=True):
    shape = tuple(vol) + (n_k, n_s) if per_voxel else (vol[-1], n_k, n_s)
    return rng.uniform(0.1, 1.0, size=shape)


def _exact_prox_then_clamp(z, S, th_tv, th_tvs, th_l1):
    """max(x*, 0) with x* = argmin 1/2|x - z|^2 + th_tv |G x|_1 +
    th_tvs |G_K S x|_1 + th_l1 |x|_1 (no sign constraint), through its dual:
    x* = z - G^T U - (G_K S)^T V - W with |U| <= th_tv, |V| <= th_tvs,
    |W| <= th_l1 minimising |x*|^2 (BVLS).  The printed dual iteration
    projects onto these boxes only and clamps at the end, so this is what it
    converges to; with S mixing species it differs from the prox of the
    regulariser plus the nonnegativity indicator."""
    shape_c = z.shape
    n_k = S.shape[-2]
    G = _grad_matrix(shape_c)
    GK = _grad_matrix((n_k,) + shape_c[1:])
    GS = GK @ _s_matrix(S, shape_c)
    n = z.size
    M = np.hstack([-G.T, -GS.T, -np.eye(n)])
    bnd = np.concatenate([np.full(G.shape[0], th_tv), np.full(GS.shape[0], th_tvs),
                          np.full(n, th_l1)])
    sol = lsq_linear(M, -z.ravel(), bounds=(-bnd, bnd), method="bvls", tol=1e-14)
    return np.maximum((z.ravel() + M @ sol.x).reshape(shape_c), 0.0)


@pytest.mark.parametrize("per_voxel", [True, False])
def test_r3_dual_step_bound_against_lapack(per_voxel):
    """The steps use sum_b theta_b^2 m_b >= eig_max(L^T L) of the stacked
    L = [theta_tv G; theta_tvs G_K S; theta_l1 I]."""
    rng = np.random.default_rng(3)
    shape_c = (2, 2, 3, 3)
    S = _random_S(rng, shape_c[1:], 3, 2, per_voxel)
    th = (0.3, 0.7, 0.2)
    G = _grad_matrix(shape_c)
    GK = _grad_matrix((3,) + shape_c[1:])
    L = np.vstack([th[0] * G, th[1] * GK @ _s_matrix(S, shape_c), th[2] * np.eye(G.shape[1])])
    lam = np.linalg.eigvalsh(L.T @ L)[-1]
    s1, s2, s3 = oracle.r3_dual_steps(shape_c[1:], S, *th)
    bound = th[0] ** 2 / s1
    assert bound >= lam * (1 - 1e-12)
    assert s2 == pytest.approx(th[1] ** 2 / bound) and s3 == pytest.approx(th[2] ** 2 / bound)
    # the switching norm is the largest singular value over voxels (LAPACK)
    blocks = S.reshape(-1, 3, 2)
    assert oracle.switching_norm2(S) == pytest.approx(
        max(np.linalg.eigvalsh(b.T @ b)[-1] for b in blocks), rel=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_prox_r3_converges_to_exact_prox_then_clamp(seed):
    rng = np.random.default_rng(40 + seed)
    shape_c = (2, 2, 2, 3)
    S = _random_S(rng, shape_c[1:], 3, 2, per_voxel=seed == 0)
    z = rng.standard_normal(shape_c) + 0.4
    th = (0.15, 0.1, 0.05)
    exact = _exact_prox_then_clamp(z, S, *th)
    x = oracle.prox_r3(z, S, *th, 30000)
    np.testing.assert_allclose(x, exact, atol=2e-6)
    assert x.min() >= 0.0


def test_prox_r3_with_identity_switching_is_tv_of_c_twice():
    """S_v = I (K = S): TV(S c) = TV(c), so the prox is that of
    (theta_tv + theta_tvs) TV + theta_l1 l1 + nonnegativity."""
    rng = np.random.default_rng(5)
    shape_c = (2, 3, 2, 3)
    S = np.broadcast_to(np.eye(2), (3, 2, 2)).copy()   # per-depth table [Nz][K][S]
    z = rng.standard_normal(shape_c) + 0.3
    x = oracle.prox_r3(z, S, 0.1, 0.15, 0.05, 30000)
    ref = oracle.prox_w(z, 0.25, 0.05, 30000)
    np.testing.assert_allclose(x, ref, atol=2e-6)


def test_prox_r3_without_tvs_matches_the_composition():
    """theta_tvs = 0: the stacked iteration (TV and l1 blocks) converges to the
    exact composition max(prox_TV(z) - theta_l1, 0)."""
    rng = np.random.default_rng(6)
    shape_c = (1, 3, 3, 4)
    S = _random_S(rng, shape_c[1:], 4, 1)
    z = rng.standard_normal(shape_c) + 0.2
    x = oracle.prox_r3(z, S, 0.2, 0.0, 0.1, 30000)
    np.testing.assert_allclose(x, oracle.prox_w(z, 0.2, 0.1, 30000), atol=2e-6)


def test_prox_r3_zero_weights_is_the_clamp():
    rng = np.random.default_rng(8)
    z = rng.standard_normal((2, 2, 3, 2))
    S = _random_S(rng, (2, 3, 2), 3, 2)
    np.testing.assert_array_equal(oracle.prox_r3(z, S, 0.0, 0.0, 0.0, 7), np.maximum(z, 0.0))


def test_ista_with_r3_prox_descends():
    """Proximal gradient without momentum at step 1/L with a converged prox
    does not increase F = 1/2|A c - p|^2 + l_tv TV(c) + l_1 |c|_1 + l_tvs TV(S c)
    (the objective includes the TV(S c) term)."""
    rng = np.random.default_rng(11)
    shape_c = (2, 2, 2, 3)
    n = int(np.prod(shape_c))
    S = _random_S(rng, shape_c[1:], 3, 2)
    Am = rng.standard_normal((30, n))
    A = lambda v: Am @ np.asarray(v).ravel()
    AT = lambda w: (Am.T @ w).reshape(shape_c)
    p = rng.standard_normal(30)
    alpha1 = 1.0 / np.linalg.eigvalsh(Am.T @ Am)[-1]
    tr = []
    oracle.fista(p, A, AT, alpha1, 0.3, 0.2, 25, 3000, momentum=False, trace=tr,
                 shape_c=shape_c, lam_tvs=0.4, S=S)
    assert all(b <= a + 1e-9 * abs(a) for a, b in zip(tr, tr[1:]))
    # and the TV(S c) term is part of it
    c = rng.uniform(0, 1, shape_c)
    f0 = oracle.objective(c, p, A, 0.3, 0.2)
    f1 = oracle.objective(c, p, A, 0.3, 0.2, 0.4, S)
    assert f1 - f0 == pytest.approx(0.4 * np.abs(oracle.grad(oracle.apply_S(c, S))).sum())
