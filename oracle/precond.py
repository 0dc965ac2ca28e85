"""Pivoted-Cholesky preconditioned msMINRES-CIQ (oracle, FP64).

THIS MODULE IS TEST INFRASTRUCTURE (see the package header).

Sec. 3.4 and Appendix D. With a preconditioner P ~ K and
A = P^{-1/2} K P^{-1/2}, the shifted solves of msMINRES run on A; one
Lanczos process still serves every shift, because A + t_q I keeps the shift
structure. The outputs

    R' b = P^{-1/2} A^{-1/2} P^{-1/2} (P^{1/2} b)      (~ K^{-1/2} b)
    R  b = K R' b                                       (~ K^{1/2} b)

satisfy R' R'^T = K^{-1} and R R^T = K, so they equal K^{-1/2} b and
K^{1/2} b up to an orthogonal rotation (Appendix D). Equivalently
R'^T K R' = I, the identity the tests check at sizes with no dense
reference. Convergence follows kappa(P^{-1} K) instead of kappa(K).

The preconditioner is the one Appendix D uses: P = Lbar Lbar^T + sigma^2 I,
Lbar the rank-R partial pivoted Cholesky factor of the noise-free kernel
matrix Ktil = o^2 k(X, X) (the greedy largest-diagonal rule of Harbrecht,
Peters and Schneider 2012). Readings where the paper is silent:

* Stop rule of the factorisation: after R columns, or earlier once the
  largest remaining residual diagonal is <= 1e-10 * max_i Ktil_ii (the
  numerical rank is reached); the remaining columns of Lbar are zero. Ties
  in the largest diagonal go to the smallest row index.
* P^{-1} by the matrix inversion lemma (Appendix D names it):
      P^{-1} x = (x - Lbar (sigma^2 I + Lbar^T Lbar)^{-1} Lbar^T x) / sigma^2.
* P^{1/2} b in closed form instead of a second CIQ run (Appendix D allows
  either; the low-rank-plus-diagonal form decomposes exactly): with
  Lbar^T Lbar = V diag(lam) V^T,
      P^{1/2} x = sigma x + Lbar V diag(1 / (sqrt(lam + sigma^2) + sigma)) V^T Lbar^T x,
  which is sigma I + U (sqrt(Lam + sigma^2) - sigma) U^T for the left
  singular vectors U = Lbar V Lam^{-1/2}, written without the cancellation.
* Eigenvalue bounds of A: preconditioned Lanczos as in Appendix B.2, with
  the known floor 1 in the role sigma^2 plays for K (K - P = Ktil - Lbar
  Lbar^T is a Schur complement, positive semi-definite, so A >= I).
"""
from __future__ import annotations

import numpy as np

from . import kernels as _k
from . import lanczos as _lz
from . import msminres as _ms
from . import quadrature as _quad

STOP_RTOL = 1e-10


def pivoted_cholesky(kind, x, lengthscale, outputscale, rank: int):
    """Rank-``rank`` partial pivoted Cholesky of Ktil = o^2 k(X, X).

    Returns (Lbar (N x rank), piv (pivots chosen, length <= rank), d (the
    residual diagonal diag(Ktil - Lbar Lbar^T))). Each step picks the row with
    the largest residual diagonal, takes its kernel row, removes the previous
    columns' contribution and scales by the square root of that diagonal.
    """
    x = np.asarray(x, dtype=np.float64)
    N = x.shape[0]
    d = np.full(N, float(outputscale))           # k(x, x) = o^2 for both kernels
    dmax0 = float(outputscale)
    L = np.zeros((N, rank))
    piv = []
    chosen = np.zeros(N, dtype=bool)
    for m in range(rank):
        cand = np.where(chosen, -np.inf, d)
        p = int(np.argmax(cand))                 # first maximum = smallest index
        if not (cand[p] > STOP_RTOL * dmax0):
            break
        piv.append(p)
        row = _k.kernel_rows(kind, x, lengthscale, outputscale, 0.0, [p])[0]
        lp = np.sqrt(d[p])
        col = (row - L[:, :m] @ L[p, :m]) / lp
        col[chosen] = 0.0
        col[p] = lp
        L[:, m] = col
        chosen[p] = True
        d = d - col * col
        d[chosen] = 0.0
    return L, np.array(piv, dtype=np.int64), d


class Preconditioner:
    """P = Lbar Lbar^T + sigma^2 I with the two operations Appendix D needs."""

    def __init__(self, L: np.ndarray, noise: float):
        if not noise > 0:
            raise ValueError("the preconditioner needs sigma^2 > 0")
        self.L = np.asarray(L, dtype=np.float64)
        self.s2 = float(noise)
        self.gram = self.L.T @ self.L
        self.lam, self.V = np.linalg.eigh(self.gram)
        self.lam = np.maximum(self.lam, 0.0)

    def inv(self, X: np.ndarray) -> np.ndarray:
        """P^{-1} X by the matrix inversion lemma."""
        R = self.L.shape[1]
        inner = np.linalg.solve(self.s2 * np.eye(R) + self.gram, self.L.T @ X)
        return (X - self.L @ inner) / self.s2

    def sqrt(self, X: np.ndarray) -> np.ndarray:
        """P^{1/2} X in the closed form above."""
        s = np.sqrt(self.s2)
        g = 1.0 / (np.sqrt(self.lam + self.s2) + s)
        T = self.V.T @ (self.L.T @ X)
        T = (g[:, None] * T) if T.ndim == 2 else g * T
        return s * X + self.L @ (self.V @ T)

    def dense(self) -> np.ndarray:
        return self.L @ self.L.T + self.s2 * np.eye(self.L.shape[0])


def eig_bounds(mvm, pre: Preconditioner, v0: np.ndarray, steps: int):
    """Bounds of the spectrum of A = P^{-1/2} K P^{-1/2} from preconditioned
    Lanczos (floor 1, see the module header)."""
    return _lz.eig_bounds(mvm, v0, steps, 1.0, pinv=pre.inv)


def ciq_pc(mvm, pre: Preconditioner, B, lambda_min, lambda_max, q, max_iter, tol, mode="invsqrt",
           return_solves=False):
    """Preconditioned msMINRES-CIQ: R' B (mode 'invsqrt') or R B ('sqrt').

    [lambda_min, lambda_max] bound the spectrum of A. The solves run on the
    start vectors C = P^{1/2} B; msMINRES with P^{-1} returns
    x^{(q)} = P^{-1/2} (A + t_q I)^{-1} P^{-1/2} C, and the quadrature sum of
    those is R' B.
    """
    t, w = _quad.hht_quadrature(lambda_min, lambda_max, q)
    C = pre.sqrt(np.asarray(B, dtype=np.float64))
    X, info = _ms.msminres(mvm, C, t, max_iter, tol, pinv=pre.inv)
    A = np.tensordot(w, X, axes=1)
    out = mvm(A) if mode == "sqrt" else A
    if return_solves:
        return out, info, t, w, X
    return out, info


def dense_reference(K: np.ndarray, pre: Preconditioner, B: np.ndarray, f):
    """P^{-1/2} f(A) P^{-1/2} P^{1/2} B = P^{-1/2} f(A) B by dense
    eigendecompositions (small N), for f(A) = A^{-1/2} or a rational r_Q(A)."""
    lp, Up = np.linalg.eigh(pre.dense())
    Pmh = (Up / np.sqrt(lp)) @ Up.T
    A = Pmh @ K @ Pmh
    A = 0.5 * (A + A.T)
    la, Ua = np.linalg.eigh(A)
    return Pmh @ (Ua @ (f(la)[:, None] * (Ua.T @ B)))
