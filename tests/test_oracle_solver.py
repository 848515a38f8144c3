"""Pins of the oracle's solver: FISTA without regularisation converges to the
nonnegative least-squares solution (SciPy's Lawson-Hanson NNLS), proximal
gradient without momentum and with an exact prox never increases the
objective, A = I reaches the prox of p in one step, the stopping tests, and
the momentum-step recurrence for A c that the GPU solver's objective uses."""
import numpy as np
import pytest
from scipy.optimize import nnls

import oracle
import synth


def _tiny_problem(seed=0):
    rng = np.random.default_rng(seed)
    ns, ny, nx, nz, K, nt, f, width = 2, 3, 3, 3, 4, 12, 3, 4
    t0, taps = synth.random_table(nz, f, nt, width, rng, t0_lo=0, t0_hi=nt - width)
    phi = rng.uniform(0.4, 1.0, size=nz)
    sp = synth.species(ns, gamma=1.0)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, K) * 100.0
    M = oracle.dense_A((ns, ny, nx, nz), K, nt, S, t0, taps)
    c_true = np.maximum(rng.standard_normal((ns, ny, nx, nz)), 0)
    p = (M @ c_true.ravel()) + 0.05 * rng.standard_normal(M.shape[0])
    return M, p, (ns, ny, nx, nz)


def test_fista_unregularised_reaches_nnls():
    M, p, shape = _tiny_problem()
    A = lambda v: M @ v.ravel()
    AT = lambda w: (M.T @ w).reshape(shape)
    lam = np.linalg.eigvalsh(M.T @ M)[-1]
    c, it = oracle.fista(p, A, AT, 1.0 / lam, 0.0, 0.0, 20000, 1, shape_c=shape)
    ref, _ = nnls(M, p, maxiter=5000)
    assert it == 20000
    np.testing.assert_allclose(c.ravel(), ref, atol=1e-6 * max(1.0, np.abs(ref).max()))


def test_ista_objective_never_increases():
    """Proximal gradient at step 1/L with an exact prox (l1 + nonnegativity,
    no TV) is a descent method."""
    M, p, shape = _tiny_problem(1)
    A = lambda v: M @ v.ravel()
    AT = lambda w: (M.T @ w).reshape(shape)
    lam = np.linalg.eigvalsh(M.T @ M)[-1]
    trace = []
    oracle.fista(p, A, AT, 1.0 / lam, 0.0, 0.3, 60, 1, momentum=False, trace=trace, shape_c=shape)
    d = np.diff(trace)
    assert np.all(d <= 1e-12 * np.abs(np.array(trace[:-1])))
    assert trace[-1] < trace[0]


def test_identity_operator_one_step_is_prox_of_p():
    rng = np.random.default_rng(2)
    shape = (1, 3, 4, 5)
    p = rng.standard_normal(shape)
    c, _ = oracle.fista(p, lambda v: v, lambda v: v, 1.0, 0.2, 0.1, 1, 30, shape_c=shape)
    np.testing.assert_allclose(c, oracle.prox_w(p, 0.2, 0.1, 30), atol=0)


def test_stopping_rules_fire():
    M, p, shape = _tiny_problem(3)
    A = lambda v: M @ v.ravel()
    AT = lambda w: (M.T @ w).reshape(shape)
    lam = np.linalg.eigvalsh(M.T @ M)[-1]
    _, it1 = oracle.fista(p, A, AT, 1.0 / lam, 0.0, 0.0, 5000, 1, eps1=1e-8, shape_c=shape)
    _, it2 = oracle.fista(p, A, AT, 1.0 / lam, 0.0, 0.0, 5000, 1, eps2=1e-4, shape_c=shape)
    assert 3 <= it1 < 5000 and 3 <= it2 < 5000


def test_fista_trace_reported_and_ends_below_start():
    M, p, shape = _tiny_problem(4)
    A = lambda v: M @ v.ravel()
    AT = lambda w: (M.T @ w).reshape(shape)
    lam = np.linalg.eigvalsh(M.T @ M)[-1]
    trace = []
    oracle.fista(p, A, AT, 1.0 / (1.01 * lam), 0.05, 0.05, 50, 20, trace=trace, shape_c=shape)
    assert len(trace) == 50 and trace[-1] < trace[0]


def test_unmixing_step_converges_to_per_voxel_nnls():
    """The two-step method's unmixing (eq. unmixing) run by the same FISTA with
    A = S (block diagonal over voxels) and no regulariser reaches, voxel by
    voxel, the nonnegative least-squares solution (SciPy NNLS)."""
    from scipy.optimize import nnls
    rng = np.random.default_rng(12)
    ns, ny, nx, nz, K = 3, 2, 3, 2, 7
    phi = rng.uniform(0.3, 1.0, size=(ny, nx, nz))
    sp = synth.species(ns, gamma=1.0)
    S = oracle.switching_matrix(phi, sp.a, sp.b, sp.tau, sp.gamma, K)
    b = rng.uniform(0.0, 1.0, size=(K, ny, nx, nz)) * 1e-2
    A = lambda c: oracle.apply_S(c, S)
    AT = lambda r: oracle.apply_ST(r, S)
    alpha1 = 1.0 / oracle.switching_norm2(S)
    c, _ = oracle.fista(b, A, AT, alpha1, 0.0, 0.0, 60000, 1, shape_c=(ns, ny, nx, nz))
    for iy in range(ny):
        for ix in range(nx):
            for iz in range(nz):
                ref, _ = nnls(S[iy, ix, iz], b[:, iy, ix, iz])
                # the per-voxel blocks are ill-conditioned (similar switching
                # curves), so the iteration is compared at a 1e-4 relative level
                np.testing.assert_allclose(c[:, iy, ix, iz], ref, rtol=1e-4, atol=1e-6)


def test_objective_recurrence_of_the_momentum_step():
    """A c_{k+1} = (A xi_{k+1} + beta_k A c_k) / (1 + beta_k), chained from
    A c_0 = A xi_0 (xi_0 = c_0), reproduces the direct data term of every
    iterate of Alg. alg:prox-outer (here with the nonnegativity prox), since
    xi_{k+1} = c_{k+1} + beta_k (c_{k+1} - c_k) and A is linear; the same
    chain with the next step's weight beta_{k+1} does not."""
    M, p, shape = _tiny_problem(3)
    lam = np.linalg.eigvalsh(M.T @ M)[-1]
    alpha = 1.0 / lam
    c = np.zeros(M.shape[1])
    xi = c.copy()
    t = 1.0
    yc = M @ xi                      # A c_0
    yc_wrong = yc.copy()
    betas, direct, rec, wrong = [], [], [], []
    for k in range(12):
        c_next = np.maximum(xi - alpha * (M.T @ (M @ xi - p)), 0.0)
        t, beta = oracle.fista_momentum(t)
        betas.append(beta)
        xi = c_next + beta * (c_next - c)
        c = c_next
        y_xi = M @ xi                # what H computes at xi_{k+1}
        yc = (y_xi + beta * yc) / (1.0 + beta)
        direct.append(0.5 * float(np.sum((M @ c - p) ** 2)))
        rec.append(0.5 * float(np.sum((yc - p) ** 2)))
        bw = oracle.fista_momentum(t)[1]   # beta_{k+1}: the wrong index
        yc_wrong = (y_xi + bw * yc_wrong) / (1.0 + bw)
        wrong.append(0.5 * float(np.sum((yc_wrong - p) ** 2)))
    assert betas[0] == 0.0 and betas[-1] > 0.3
    np.testing.assert_allclose(rec, direct, rtol=1e-12)
    assert max(abs(a - b) / b for a, b in zip(wrong, direct)) > 1e-4
