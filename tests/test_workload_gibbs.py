"""The image-model operator of the Gibbs workload (Sec. 5.3, App. F) against
SciPy's image filters and the model's algebra: blur and Laplacian equal
scipy.ndimage correlation with reflected boundaries, the decimation covers
every pixel once (D^T D = I), and the precision is symmetric positive
definite with the stated composition."""
import numpy as np
import pytest
from scipy import ndimage

from workloads import gibbs


@pytest.mark.parametrize("n", [8, 17, 24])
def test_filters_match_ndimage(n):
    img = np.random.default_rng(n).random((n, n))
    B = gibbs.correlation_matrix(n, gibbs.gaussian_filter())
    ref = ndimage.correlate(img, gibbs.gaussian_filter(), mode="reflect")
    assert np.abs((B @ img.ravel()).reshape(n, n) - ref).max() < 1e-14
    Lf = gibbs.correlation_matrix(n, gibbs.LAPLACE_FILTER)
    ref = ndimage.correlate(img, gibbs.LAPLACE_FILTER, mode="reflect")
    assert np.abs((Lf @ img.ravel()).reshape(n, n) - ref).max() < 1e-14
    w = gibbs.gaussian_filter()
    assert abs(w.sum() - 1.0) < 1e-15 and w.shape == (5, 5)


def test_decimation_and_precision():
    n = 24
    D = gibbs.decimation_matrix(n)
    assert D.shape == (4 * (n // 2) ** 2, n * n)
    assert np.abs((D.T @ D).toarray() - np.eye(n * n)).max() == 0.0
    g_obs, g_prior = 1.0, 0.01
    Lam = gibbs.gibbs_precision(n, g_obs, g_prior).toarray()
    B = gibbs.correlation_matrix(n, gibbs.gaussian_filter()).toarray()
    Lp = -gibbs.correlation_matrix(n, gibbs.LAPLACE_FILTER).toarray()
    A = D.toarray() @ B
    assert np.abs(Lam - (g_obs * A.T @ A + g_prior * Lp)).max() < 1e-14
    assert np.abs(Lam - Lam.T).max() == 0.0
    lam = np.linalg.eigvalsh(Lam)
    assert lam[0] > 0
    # the prior alone annihilates constants (reflected boundaries), the blur keeps them
    assert np.abs(Lp @ np.ones(n * n)).max() < 1e-14
    assert np.abs(B @ np.ones(n * n) - 1.0).max() < 1e-14
