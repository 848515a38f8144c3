"""Pins of the oracle's regulariser pieces: gradient/adjoint, the dual step
constant, soft-thresholding, the dual-FISTA TV prox and the combined prox,
against closed forms, LAPACK and an exact bounded least-squares solve (SciPy
BVLS) of the dual problem."""
import math

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


def test_grad_adjoint_and_constants():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 5, 6))
    p = rng.standard_normal((3, 2, 4, 5, 6))
    assert np.vdot(oracle.grad(x), p) == pytest.approx(np.vdot(x, oracle.grad_T(p)), rel=1e-13)
    np.testing.assert_array_equal(oracle.grad(np.full((1, 3, 4, 5), 2.5)), 0.0)
    # explicit forward differences with a zero last difference
    v = np.arange(5.0) ** 2
    g = oracle.grad(v.reshape(1, 1, 1, 5))[2].ravel()
    np.testing.assert_array_equal(g, [1, 3, 5, 7, 0])


@pytest.mark.parametrize("shape", [(1, 1, 5), (2, 3, 4), (3, 3, 3), (1, 4, 1)])
def test_tv_step_constant_matches_lapack(shape):
    G = _grad_matrix((1,) + shape)
    lam = np.linalg.eigvalsh(G.T @ G)[-1]
    assert oracle.tv_step_constant(shape) == pytest.approx(lam, rel=1e-12, abs=1e-12)
    assert oracle.tv_step_constant(shape) < 12.0


def test_prox_l1_closed_form():
    z = np.array([-2.0, -0.5, 0.0, 0.3, 0.5, 0.7, 3.0])
    np.testing.assert_allclose(oracle.prox_l1(z, 0.5, nonneg=False), [-1.5, 0, 0, 0, 0, 0.2, 2.5])
    np.testing.assert_allclose(oracle.prox_l1(z, 0.5, nonneg=True), [0, 0, 0, 0, 0, 0.2, 2.5])
    # tie |z| = thresh gives exactly 0
    assert oracle.prox_l1(np.array([0.5]), 0.5, nonneg=False)[0] == 0.0


@pytest.mark.parametrize("a,b,theta", [(3.0, 1.0, 0.4), (3.0, 1.0, 2.0), (1.0, 1.2, 0.05), (-1.0, 2.0, 10.0)])
def test_prox_tv_two_voxels_closed_form(a, b, theta):
    """min 1/2((x1-a)^2 + (x2-b)^2) + theta|x2 - x1|: the two values meet at
    the mean when |a - b| <= 2 theta, else each moves theta toward the other."""
    z = np.array([a, b]).reshape(1, 1, 1, 2)
    x = oracle.prox_tv(z, theta, 400).ravel()
    if abs(a - b) <= 2 * theta:
        np.testing.assert_allclose(x, [(a + b) / 2] * 2, atol=1e-9)
    else:
        s = math.copysign(1.0, a - b)
        np.testing.assert_allclose(x, [a - s * theta, b + s * theta], atol=1e-9)


def test_prox_tv_fixed_points_and_limits():
    rng = np.random.default_rng(1)
    const = np.full((2, 3, 4, 5), 1.75)
    np.testing.assert_allclose(oracle.prox_tv(const, 0.3, 20), const, atol=1e-15)
    z = rng.standard_normal((1, 3, 3, 4))
    # theta -> infinity: the constant volume at the mean (Neumann boundary)
    x = oracle.prox_tv(z, 1e6, 3000)
    np.testing.assert_allclose(x, np.full_like(z, z.mean()), atol=1e-6)
    # theta = 0: identity
    np.testing.assert_allclose(oracle.prox_tv(z, 0.0, 5), z, atol=0)


def _bvls_prox(z, theta_tv, theta_l1=None):
    """Exact prox via its dual, solved by bounded-variable least squares.
    TV only:   min_u 1/2|z - G^T u|^2, |u| <= theta           ->  x = z - G^T u
    TV+l1+>=0: min_{u,m} 1/2|(z - th1) - G^T u + m|^2, |u|<=theta, m>=0
                                                          ->  x = (z - th1) - G^T u + m"""
    shape = z.shape
    G = _grad_matrix(shape)
    zr = z.ravel()
    if theta_l1 is None:
        sol = lsq_linear(-G.T, -zr, bounds=(-theta_tv, theta_tv), method="bvls", tol=1e-14)
        return (zr - G.T @ sol.x).reshape(shape)
    n = zr.size
    Mx = np.hstack([-G.T, np.eye(n)])
    lo = np.concatenate([np.full(G.shape[0], -theta_tv), np.zeros(n)])
    hi = np.concatenate([np.full(G.shape[0], theta_tv), np.full(n, np.inf)])
    w = zr - theta_l1
    sol = lsq_linear(Mx, -w, bounds=(lo, hi), method="bvls", tol=1e-14)
    return (w + Mx @ sol.x).reshape(shape)


@pytest.mark.parametrize("shape,theta", [((1, 1, 1, 9), 0.3), ((1, 3, 4, 3), 0.25), ((2, 2, 3, 3), 0.6)])
def test_prox_tv_converges_to_exact_dual_solution(shape, theta):
    rng = np.random.default_rng(sum(shape))
    z = rng.standard_normal(shape)
    exact = _bvls_prox(z, theta)
    x = oracle.prox_tv(z, theta, 4000)
    np.testing.assert_allclose(x, exact, atol=2e-6)


def test_prox_w_matches_exact_constrained_prox():
    """TV + l1 + nonnegativity, against the BVLS solve of its own dual (which
    does not use the composition the oracle relies on)."""
    rng = np.random.default_rng(7)
    z = rng.standard_normal((1, 3, 3, 4)) + 0.3
    exact = _bvls_prox(z, 0.2, theta_l1=0.15)
    x = oracle.prox_w(z, 0.2, 0.15, 4000)
    np.testing.assert_allclose(x, exact, atol=2e-6)
    assert x.min() >= 0.0


def test_prox_tv_dual_optimality():
    """At convergence x = z - G^T u with |u| <= theta, and u_e = theta*sign(Gx)_e
    wherever the difference (Gx)_e is nonzero (subgradient condition)."""
    rng = np.random.default_rng(9)
    z = rng.standard_normal((1, 4, 4, 4))
    theta = 0.2
    x, u = oracle.prox_tv(z, theta, 6000, return_dual=True)
    assert np.abs(u).max() <= theta + 1e-15
    g = oracle.grad(x)
    big = np.abs(g) > 1e-5
    np.testing.assert_allclose(u[big], theta * np.sign(g[big]), atol=1e-6)


def test_literal_momentum_option_differs_but_converges():
    rng = np.random.default_rng(4)
    z = rng.standard_normal((1, 2, 3, 4))
    a = oracle.prox_tv(z, 0.3, 5)
    b = oracle.prox_tv(z, 0.3, 5, literal_momentum=True)
    assert np.abs(a - b).max() > 0
    exact = _bvls_prox(z, 0.3)
    np.testing.assert_allclose(oracle.prox_tv(z, 0.3, 4000, literal_momentum=True), exact, atol=2e-6)
