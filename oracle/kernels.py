"""Kernel matrices K = o^2 k(X, X) + sigma^2 I (oracle, FP64).

The paper uses RBF and Matern-5/2 kernels (Sec. 4 figures, App. E/F
experiment details) but never writes the formulas. Reading used here (the
GPyTorch conventions the paper's experiments ran with):

    r^2      = sum_d (x_d - x'_d)^2 / l_d^2          (l isotropic or ARD)
    RBF      k = exp(-r^2 / 2)
    Matern52 k = (1 + sqrt5 r + 5 r^2 / 3) exp(-sqrt5 r)
    K        = o^2 k(X, X) + sigma^2 I               (o^2 = "outputscale")

Noise/jitter sigma^2 sits only on the diagonal.
"""
from __future__ import annotations

import numpy as np

RBF = "rbf"
MATERN52 = "matern52"
SQRT5 = np.sqrt(5.0)


def _ls(lengthscale, d: int) -> np.ndarray:
    ls = np.asarray(lengthscale, dtype=np.float64).reshape(-1)
    if ls.size == 1:
        ls = np.full(d, ls[0])
    if ls.size != d:
        raise ValueError("lengthscale must have 1 or d entries")
    return ls


def scaled_sqdist(x1: np.ndarray, x2: np.ndarray, lengthscale) -> np.ndarray:
    """r^2_ij = sum_d (x1_id - x2_jd)^2 / l_d^2, by explicit differences."""
    x1 = np.asarray(x1, dtype=np.float64)
    x2 = np.asarray(x2, dtype=np.float64)
    ls = _ls(lengthscale, x1.shape[1])
    r2 = np.zeros((x1.shape[0], x2.shape[0]))
    for d in range(x1.shape[1]):
        diff = (x1[:, d][:, None] - x2[:, d][None, :]) / ls[d]
        r2 += diff * diff
    return r2


def unit_kernel(kind: str, r2: np.ndarray) -> np.ndarray:
    """k(r) with unit outputscale, as a function of the scaled r^2."""
    if kind == RBF:
        return np.exp(-0.5 * r2)
    if kind == MATERN52:
        r = np.sqrt(r2)
        return (1.0 + SQRT5 * r + (5.0 / 3.0) * r2) * np.exp(-SQRT5 * r)
    raise ValueError(f"unknown kernel {kind}")


def kernel_matrix(kind, x, lengthscale, outputscale, noise) -> np.ndarray:
    """Dense K = o^2 k(X, X) + sigma^2 I (N x N, FP64)."""
    r2 = scaled_sqdist(x, x, lengthscale)
    K = outputscale * unit_kernel(kind, r2)
    K[np.diag_indices_from(K)] += noise
    return K


def kernel_mvm_blocked(kind, x, lengthscale, outputscale, noise, v, block=256):
    """K V without storing K: rows of K are generated ``block`` at a time.

    The partitioned ("map-reduce") MVM the paper relies on for O(N) memory
    (Sec. 3.2 and Property 1).
    """
    x = np.asarray(x, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    squeeze = v.ndim == 1
    if squeeze:
        v = v[:, None]
    y = np.empty_like(v)
    for i0 in range(0, x.shape[0], block):
        i1 = min(i0 + block, x.shape[0])
        kb = outputscale * unit_kernel(kind, scaled_sqdist(x[i0:i1], x, lengthscale))
        y[i0:i1] = kb @ v
    y += noise * v
    return y[:, 0] if squeeze else y


def kernel_rows(kind, x, lengthscale, outputscale, noise, rows) -> np.ndarray:
    """Selected rows of K (len(rows) x N), for spot checks at large N."""
    x = np.asarray(x, dtype=np.float64)
    rows = np.asarray(rows)
    kb = outputscale * unit_kernel(kind, scaled_sqdist(x[rows], x, lengthscale))
    kb[np.arange(rows.size), rows] += noise
    return kb


def kernel_lengthscale_grad(kind, x, lengthscale, outputscale) -> np.ndarray:
    """dK_ij / dl_d for every ARD dimension d: array (d, N, N).

    RBF:      dK/dl_d = o^2 k (x_d - x'_d)^2 / l_d^3
    Matern52: dK/dl_d = o^2 (5/3)(1 + sqrt5 r) exp(-sqrt5 r) (x_d - x'_d)^2 / l_d^3
    (chain rule through r^2; for an isotropic lengthscale sum over d).
    """
    x = np.asarray(x, dtype=np.float64)
    ls = _ls(lengthscale, x.shape[1])
    r2 = scaled_sqdist(x, x, ls)
    if kind == RBF:
        dk_dr2 = -0.5 * np.exp(-0.5 * r2)
    elif kind == MATERN52:
        r = np.sqrt(r2)
        dk_dr2 = -(5.0 / 6.0) * (1.0 + SQRT5 * r) * np.exp(-SQRT5 * r)
    else:
        raise ValueError(kind)
    out = np.empty((x.shape[1],) + r2.shape)
    for d in range(x.shape[1]):
        diff2 = (x[:, d][:, None] - x[:, d][None, :]) ** 2
        # d r^2 / d l_d = -2 diff^2 / l_d^3
        out[d] = outputscale * dk_dr2 * (-2.0 * diff2 / ls[d] ** 3)
    return out
