"""Pins of the oracle's msMINRES (Appendix C) against SciPy's MINRES, a brute
force least-squares solve, the residual identity and the paper's bounds."""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import kernels as kk
from oracle import msminres as ms
from oracle import quadrature as qd


def _spd(n, seed, noise=1e-2, ls=0.3):
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3))
    return kk.kernel_matrix("rbf", x, [ls], 1.0, noise), rng


@pytest.mark.parametrize("j", [1, 2, 5, 12])
def test_matches_scipy_minres_iterates(j):
    K, rng = _spd(48, 1)
    b = rng.standard_normal((48, 3))
    t, _ = qd.hht_quadrature(1e-2, float(np.linalg.eigvalsh(K)[-1]), 6)
    X, info = ms.msminres(lambda v: K @ v, b, t, j, 0.0)
    assert info.iters == j
    for qi in range(t.size):
        for s in range(3):
            ref, _ = sla.minres(K, b[:, s], shift=-t[qi], maxiter=j, rtol=0.0)
            assert np.linalg.norm(X[qi, :, s] - ref) <= 1e-10 * np.linalg.norm(ref)


@pytest.mark.parametrize("j", [1, 3, 8, 20, 30])
def test_matches_bruteforce_argmin(j):
    # well-conditioned (kappa ~ 14) so the Krylov basis stays numerically
    # independent up to j = N and the brute force is itself accurate
    rng = np.random.default_rng(2)
    K = kk.kernel_matrix("rbf", rng.random((30, 3)), [0.15], 1.0, 0.2)
    b = rng.standard_normal(30)
    for t in [0.0, 1e-3, 0.5, 40.0]:
        X, _ = ms.msminres(lambda v: K @ v, b, [t], j, 0.0)
        ref = ms.minres_dense_argmin(K, b, t, j)
        assert np.linalg.norm(X[0] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_residual_identity_and_monotone():
    K, rng = _spd(80, 3)
    b = rng.standard_normal((80, 2))
    t = np.array([1e-3, 0.1, 3.0])
    prev = None
    for j in range(1, 25):
        X, info = ms.msminres(lambda v: K @ v, b, t, j, 0.0)
        for qi in range(3):
            r = (K + t[qi] * np.eye(80)) @ X[qi] - b
            true = np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)
            np.testing.assert_allclose(info.rel_residual[qi], true, rtol=1e-8, atol=1e-14)
        if prev is not None:
            assert np.all(info.rel_residual <= prev * (1 + 1e-12) + 1e-15)
        prev = info.rel_residual


def test_exact_after_n_iterations():
    rng = np.random.default_rng(4)
    K = kk.kernel_matrix("rbf", rng.random((16, 3)), [0.15], 1.0, 0.2)
    b = rng.standard_normal(16)
    t = [0.0, 0.2]
    X, _ = ms.msminres(lambda v: K @ v, b, t, 16, 0.0)
    for qi, tq in enumerate(t):
        ref = np.linalg.solve(K + tq * np.eye(16), b)
        assert np.linalg.norm(X[qi] - ref) <= 1e-11 * np.linalg.norm(ref)


def test_minres_rate_lemma():
    K, rng = _spd(120, 5, noise=5e-2)
    lam = np.linalg.eigvalsh(K)
    kappa = lam[-1] / lam[0]
    rho = (math.sqrt(kappa) - 1) / (math.sqrt(kappa) + 1)
    b = rng.standard_normal(120)
    t = np.array([1e-4, 1e-2, 1.0])
    for J in [2, 5, 10, 20]:
        _, info = ms.msminres(lambda v: K @ v, b, t, J, 0.0)
        # the Chebyshev bound carries a factor 2 (Greenbaum, Ch. 3) that the
        # lemma's statement drops; without it J = 2 already violates it here
        assert np.all(info.rel_residual <= 2 * rho ** J + 1e-13)


def test_diagonal_few_distinct_values_is_exact():
    d = np.array([0.5] * 10 + [2.0] * 7 + [9.0] * 5)
    K = np.diag(d)
    b = np.random.default_rng(6).standard_normal((22, 2))
    t = np.array([0.01, 1.0, 7.0])
    X, info = ms.msminres(lambda v: K @ v, b, t, 50, 1e-12)
    assert info.iters <= 3
    for qi in range(3):
        np.testing.assert_allclose(X[qi], b / (d + t[qi])[:, None], rtol=1e-10)


def test_zero_column_and_freeze():
    # moderate kappa: convergence to 1e-6 well before the Krylov space is
    # exhausted, where finite-precision runs of different codes stay close
    K, rng = _spd(40, 7, noise=0.2, ls=0.15)
    b = rng.standard_normal((40, 3))
    b[:, 1] = 0.0
    t = np.array([1e-2, 1.0])
    X, info = ms.msminres(lambda v: K @ v, b, t, 200, 1e-6)
    assert np.all(X[:, :, 1] == 0.0)
    assert info.converged.all()
    assert np.all(info.rel_residual <= 1e-6)
    # a frozen shift keeps the iterate of the iteration it converged at:
    # compare with SciPy at exactly that many iterations
    for qi in range(2):
        x1, i1 = ms.msminres(lambda v: K @ v, b[:, :1], t[qi:qi + 1], 200, 1e-6)
        j = int(i1.col_iters[0])
        ref, _ = sla.minres(K, b[:, 0], shift=-t[qi], maxiter=j, rtol=0.0)
        assert np.linalg.norm(x1[0, :, 0] - ref) <= 1e-9 * np.linalg.norm(ref)
        # and the two-shift run froze this shift at that same iterate
        assert np.linalg.norm(X[qi, :, 0] - ref) <= 1e-9 * np.linalg.norm(ref)


def test_shift_invariance():
    # msMINRES on K with shift t == MINRES on (K + tI) with no shift
    K, rng = _spd(50, 8, noise=0.2, ls=0.15)
    b = rng.standard_normal(50)
    for t in [1e-3, 0.7]:
        X1, _ = ms.msminres(lambda v: K @ v, b, [t], 15, 0.0)
        Kt = K + t * np.eye(50)
        X2, _ = ms.msminres(lambda v: Kt @ v, b, [0.0], 15, 0.0)
        assert np.linalg.norm(X1[0] - X2[0]) <= 1e-10 * np.linalg.norm(X2[0])


def test_planted_mistake_is_caught():
    # a sign slip on the shift (a plausible mistake) must break agreement with SciPy
    K, rng = _spd(30, 9)
    b = rng.standard_normal(30)
    X, _ = ms.msminres(lambda v: K @ v, b, [0.1], 10, 0.0)
    ref, _ = sla.minres(K, b, shift=-0.1, maxiter=10, rtol=0.0)
    assert np.linalg.norm(X[0] - ref) <= 1e-10 * np.linalg.norm(ref)
    Xbad, _ = ms.msminres(lambda v: K @ v, b, [-0.1], 10, 0.0)
    assert np.linalg.norm(Xbad[0] - ref) > 1e-3 * np.linalg.norm(ref)
