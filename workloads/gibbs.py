"""Input operator of the image-reconstruction Gibbs sampler (Sec. 5.3,
App. F): the conditional precision of the high-resolution image,

    Lam = g_obs A^T A + g_prior Lp,   A = D B,

as an explicit sparse matrix. This builds the problem's operator (like the
points of the kernel workloads); it contains none of CIQ's arithmetic.

Readings of the model (the paper gives sizes and filters, not the indexing):
* B: 5 x 5 Gaussian blur with standard deviation 2.5 pixels, weights
  normalised to sum 1, applied by correlation with reflected (half-sample
  symmetric) boundaries: index -1 -> 0, -2 -> 1, N -> N-1, N+1 -> N-2.
* D: the K = 4 low-resolution M x M images (M = N/2) are the four 2 x 2
  sub-lattices of the blurred image, image (p, q) taking pixels
  (2a + p, 2b + q) -- a binary decimation matrix of K M^2 rows.
* Lp: the isotropic 3 x 3 filter of App. F with reflected boundaries,
  negated so that the prior precision is positive semi-definite (the filter
  as printed has -12/12 at its centre and is negative semi-definite).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

LAPLACE_FILTER = np.array([[1.0, 2.0, 1.0], [2.0, -12.0, 2.0], [1.0, 2.0, 1.0]]) / 12.0


def reflect(i: int, n: int) -> int:
    """Half-sample symmetric boundary: ... b a | a b c ... (period 2n)."""
    i = i % (2 * n)
    return i if i < n else 2 * n - 1 - i


def correlation_matrix(n: int, w: np.ndarray) -> sp.csr_matrix:
    """The n^2 x n^2 matrix of 2-D correlation with the odd-sized filter w and
    reflected boundaries (row-major pixel index r * n + c)."""
    h = w.shape[0] // 2
    rows, cols, vals = [], [], []
    for r in range(n):
        for c in range(n):
            i = r * n + c
            for dr in range(-h, h + 1):
                for dc in range(-h, h + 1):
                    j = reflect(r + dr, n) * n + reflect(c + dc, n)
                    rows.append(i)
                    cols.append(j)
                    vals.append(w[dr + h, dc + h])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n * n, n * n))


def gaussian_filter(size: int = 5, sigma: float = 2.5) -> np.ndarray:
    h = size // 2
    g = np.exp(-(np.arange(-h, h + 1) ** 2) / (2.0 * sigma * sigma))
    w = np.outer(g, g)
    return w / w.sum()


def decimation_matrix(n: int) -> sp.csr_matrix:
    """K = 4 images of (n/2)^2 pixels: image (p, q) row a * (n/2) + b takes
    pixel (2a + p, 2b + q)."""
    m = n // 2
    rows, cols = [], []
    k = 0
    for p in range(2):
        for q in range(2):
            for a in range(m):
                for b in range(m):
                    rows.append(k * m * m + a * m + b)
                    cols.append((2 * a + p) * n + (2 * b + q))
            k += 1
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(4 * m * m, n * n))


def gibbs_precision(n: int = 160, g_obs: float = 1.0, g_prior: float = 0.01) -> sp.csr_matrix:
    """Lam (n^2 x n^2, CSR, FP64, sorted column indices, exactly symmetric)."""
    B = correlation_matrix(n, gaussian_filter())
    A = decimation_matrix(n) @ B
    Lp = -correlation_matrix(n, LAPLACE_FILTER)
    Lam = (g_obs * (A.T @ A) + g_prior * Lp).tocsr()
    Lam = (0.5 * (Lam + Lam.T)).tocsr()
    Lam.sum_duplicates()
    Lam.sort_indices()
    return Lam
