"""Pins of the oracle's kernel matrices against scikit-learn's independent
implementations and finite differences."""
import numpy as np
import pytest
from sklearn.gaussian_process import kernels as skk

from oracle import kernels as kk


@pytest.mark.parametrize("ard", [False, True])
def test_rbf_and_matern_vs_sklearn(ard):
    rng = np.random.default_rng(0)
    x = rng.random((50, 4))
    ls = rng.uniform(0.1, 1.0, 4) if ard else np.array([0.3])
    l_sk = ls if ard else float(ls[0])
    np.testing.assert_allclose(kk.kernel_matrix("rbf", x, ls, 2.0, 0.0),
                               2.0 * skk.RBF(length_scale=l_sk)(x), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(kk.kernel_matrix("matern52", x, ls, 1.5, 0.0),
                               1.5 * skk.Matern(length_scale=l_sk, nu=2.5)(x), rtol=1e-11, atol=1e-14)
    K = kk.kernel_matrix("rbf", x, ls, 1.0, 0.25)
    np.testing.assert_allclose(np.diag(K), 1.25)


def test_blocked_mvm_and_rows():
    rng = np.random.default_rng(1)
    x = rng.random((301, 6))
    v = rng.standard_normal((301, 5))
    for kind in ["rbf", "matern52"]:
        K = kk.kernel_matrix(kind, x, [0.3], 1.2, 1e-3)
        np.testing.assert_allclose(kk.kernel_mvm_blocked(kind, x, [0.3], 1.2, 1e-3, v, block=64),
                                   K @ v, rtol=1e-12, atol=1e-12)
        rows = np.array([0, 17, 300])
        np.testing.assert_allclose(kk.kernel_rows(kind, x, [0.3], 1.2, 1e-3, rows), K[rows], rtol=1e-13)


@pytest.mark.parametrize("kind", ["rbf", "matern52"])
def test_lengthscale_grad_fd(kind):
    rng = np.random.default_rng(2)
    x = rng.random((20, 3))
    ls = np.array([0.3, 0.5, 0.8])
    g = kk.kernel_lengthscale_grad(kind, x, ls, 1.7)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3); e[d] = h
        fd = (kk.kernel_matrix(kind, x, ls + e, 1.7, 0.0) - kk.kernel_matrix(kind, x, ls - e, 1.7, 0.0)) / (2 * h)
        np.testing.assert_allclose(g[d], fd, rtol=1e-6, atol=1e-8)
