"""CIQ composition and exact references (oracle, FP64).

Sec. 3 (rational approximation): K^{-1/2} ~= sum_q w_q (t_q I + K)^{-1} and
K^{1/2} ~= K sum_q w_q (t_q I + K)^{-1}; Alg. S1 forms the inverse root as
the w-weighted sum of the msMINRES solves, and the square root multiplies
that sum by K once more.
"""
from __future__ import annotations

import numpy as np

from . import msminres as _ms
from . import quadrature as _quad


def ciq(mvm, B, lambda_min, lambda_max, q, max_iter, tol, mode="invsqrt",
        return_solves=False):
    """msMINRES-CIQ (Alg. S1). mode 'invsqrt' -> K^{-1/2}B, 'sqrt' -> K^{1/2}B."""
    t, w = _quad.hht_quadrature(lambda_min, lambda_max, q)
    X, info = _ms.msminres(mvm, B, t, max_iter, tol)
    A = np.tensordot(w, X, axes=1)              # sum_q w_q x^{(q)}
    out = mvm(A) if mode == "sqrt" else A
    if return_solves:
        return out, info, t, w, X
    return out, info


def eig_apply(K: np.ndarray, B: np.ndarray, f) -> np.ndarray:
    """U f(Lambda) U^T B for K = U Lambda U^T (dense eigh)."""
    lam, U = np.linalg.eigh(K)
    B = np.asarray(B, dtype=np.float64)
    out = U @ (f(lam)[:, None] * (U.T @ B.reshape(K.shape[0], -1)))
    return out.reshape(B.shape)


def exact_power(K: np.ndarray, B: np.ndarray, p: float) -> np.ndarray:
    """K^p B through the eigendecomposition (the plain definition)."""
    return eig_apply(K, B, lambda lam: lam ** p)


def exact_rational(K: np.ndarray, B: np.ndarray, t, w, mode="invsqrt") -> np.ndarray:
    """CIQ with exact shifted solves: U r_Q(Lambda) U^T B (times Lambda for sqrt)."""
    t = np.asarray(t); w = np.asarray(w)
    if mode == "sqrt":
        return eig_apply(K, B, lambda lam: lam * _quad.rational(t, w, lam))
    return eig_apply(K, B, lambda lam: _quad.rational(t, w, lam))


def rel_err(a: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-column relative 2-norm error ||a_s - ref_s|| / ||ref_s||."""
    a = np.asarray(a, dtype=np.float64).reshape(ref.shape[0], -1)
    ref = np.asarray(ref, dtype=np.float64).reshape(ref.shape[0], -1)
    return np.linalg.norm(a - ref, axis=0) / np.linalg.norm(ref, axis=0)
