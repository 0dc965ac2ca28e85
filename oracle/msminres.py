"""Multi-shift MINRES (oracle, FP64).

Computes, for every column b_s of B and every shift t_q,

    x_J^{(q,s)} = argmin_{x in K_J(K, b_s)} || (K + t_q I) x - b_s ||_2      (*)

(Appendix C.2, the shifted least-squares problem through the QR of the
shifted tridiagonal [T_J + t_q I; beta_{J+1} e_J^T], and the proof of the
msMINRES residual lemma in Appendix G). All shifts share one Lanczos run on K
(the shift-invariance observation of Appendix C.2), so J iterations cost J
products with K whatever Q is (Property 1).

The recurrence is the standard Paige-Saunders one that Appendix C.1 derives
(QR of the growing tridiagonal by Givens rotations; only the last two
rotations and the last two columns of Q_J R_J^{-1} are kept). The printed
listings (Alg. S3/S4) contain typesetting slips; this follows the
derivation, in the paper's roles: alpha_j = T(j, j) (the listing's gamma),
beta_{j+1} = T(j+1, j) (the listing's delta), and per shift the three
nonzeros (eps_j, delta_j, gamma_j) of column j of R, the step tau_j and the
residual scalar phibar_{j+1}:

    Lanczos:  v = K q_j - beta_j q_{j-1};  alpha_j = q_j^T v;  v -= alpha_j q_j
              beta_{j+1} = ||v||;  q_{j+1} = v / beta_{j+1}
    per shift t (rotations G_{j-2}, G_{j-1} from earlier steps, identity at start):
              eps_j   = s_{j-2} beta_j          dhat = c_{j-2} beta_j
              delta_j = c_{j-1} dhat + s_{j-1} (alpha_j + t)
              gbar    = -s_{j-1} dhat + c_{j-1} (alpha_j + t)
              gamma_j = sqrt(gbar^2 + beta_{j+1}^2); c_j = gbar/gamma_j; s_j = beta_{j+1}/gamma_j
              tau_j = c_j phibar_j;  phibar_{j+1} = -s_j phibar_j   (phibar_1 = ||b||)
              m_j = (q_j - delta_j m_{j-1} - eps_j m_{j-2}) / gamma_j
              x_j = x_{j-1} + tau_j m_j
    and ||(K + t I) x_j - b|| = |phibar_{j+1}|.

Stopping rule (the paper stops at a relative residual, Sec. 4 and App. E):
shift (q, s) is frozen once |phibar_{j+1}| <= tol ||b_s|| (its x keeps the
value just reached); column s stops once all its shifts are frozen or its
Lanczos run breaks down (beta_{j+1} <= breakdown_rtol ||K q_j||, an exact
solve); everything stops after ``max_iter`` products with K. A zero column
b_s gives x = 0 and counts as converged at once. The initial guess is zero.

Preconditioned form (Appendix D; ``pinv`` = the map x -> P^{-1} x). The
Lanczos process runs on A = P^{-1/2} K P^{-1/2} without forming P^{-1/2}:
it keeps z_j = P^{1/2} qt_j and p_j = P^{-1} z_j = P^{-1/2} qt_j for the
orthonormal Lanczos vectors qt_j of A started from P^{-1/2} b, so

    v = K p_j - beta_j z_{j-1};  alpha_j = p_j^T v;  v -= alpha_j z_j
    pt = P^{-1} v;  beta_{j+1} = sqrt(v^T pt);  z_{j+1} = v / beta_{j+1};  p_{j+1} = pt / beta_{j+1}

(beta_1 = sqrt(b^T P^{-1} b)), the Givens stage is unchanged and the
direction recurrence consumes p_j in place of q_j. Then
x_j^{(q)} = P^{-1/2} y_j^{(q)} with y_j^{(q)} the MINRES iterate of
(A + t_q I) y = P^{-1/2} b, and |phibar_{j+1}| is that system's residual.
The breakdown test uses sqrt(alpha_j^2 + beta_j^2 + beta_{j+1}^2), the
A-norm of A qt_j, in place of ||K q_j||.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class MinresInfo:
    iters: int                 # products with K performed
    col_iters: np.ndarray      # (S,) iterations each column ran
    converged: np.ndarray      # (Q, S) bool
    rel_residual: np.ndarray   # (Q, S) |phibar_{j+1}| / ||b_s|| at the final iterate
    alpha: list                # per iteration, (S,) Lanczos diagonal (for inspection)
    beta: list                 # per iteration, (S,) beta_{j+1}


def msminres(mvm, B: np.ndarray, shifts, max_iter: int, tol: float,
             breakdown_rtol: float = 1e-13, pinv=None):
    """Returns X with X[q] ~= (K + t_q I)^{-1} B, and a MinresInfo. With
    ``pinv``, X[q] ~= P^{-1/2} (A + t_q I)^{-1} P^{-1/2} B (see the header)."""
    B = np.asarray(B, dtype=np.float64)
    squeeze = B.ndim == 1
    if squeeze:
        B = B[:, None]
    t = np.asarray(shifts, dtype=np.float64).reshape(-1)
    N, S = B.shape
    Qn = t.size

    if pinv is None:
        beta1 = np.linalg.norm(B, axis=0)             # ||b_s||
    else:
        PB = pinv(B)
        beta1 = np.sqrt(np.maximum(np.sum(B * PB, axis=0), 0.0))
    X = np.zeros((Qn, N, S))
    m1 = np.zeros((Qn, N, S))                          # m_{j-1}
    m2 = np.zeros((Qn, N, S))                          # m_{j-2}
    nz = beta1 > 0
    q = np.zeros_like(B)
    q[:, nz] = B[:, nz] / beta1[nz]
    q_prev = np.zeros_like(B)
    if pinv is not None:                               # p_j = P^{-1} z_j (q holds z_j)
        pq = np.zeros_like(B)
        pq[:, nz] = PB[:, nz] / beta1[nz]
    else:
        pq = q
    beta_j = np.zeros(S)                               # beta_j (0 for j = 1)

    c1 = np.ones((Qn, S)); s1 = np.zeros((Qn, S))      # G_{j-1}
    c2 = np.ones((Qn, S)); s2 = np.zeros((Qn, S))      # G_{j-2}
    phibar = np.tile(beta1, (Qn, 1))

    frozen = np.tile(~nz, (Qn, 1))
    active = nz.copy()
    col_iters = np.zeros(S, dtype=int)
    rel_res = np.where(frozen, 0.0, 1.0)
    alphas, betas = [], []
    iters = 0

    for _ in range(max_iter):
        if not active.any():
            break
        iters += 1
        y = mvm(pq)                                    # K q_j (all columns share it)
        v = y - beta_j * q_prev
        alpha = np.sum(pq * v, axis=0)
        v = v - alpha * q
        if pinv is None:
            beta_next = np.linalg.norm(v, axis=0)
            scale = np.linalg.norm(y, axis=0)
        else:
            pv = pinv(v)
            beta_next = np.sqrt(np.maximum(np.sum(v * pv, axis=0), 0.0))
            scale = np.sqrt(alpha ** 2 + beta_j ** 2 + beta_next ** 2)
        broke = beta_next <= breakdown_rtol * scale
        beta_next = np.where(broke, 0.0, beta_next)
        alphas.append(alpha.copy())
        betas.append(beta_next.copy())

        a = alpha[None, :] + t[:, None]
        eps = s2 * beta_j[None, :]
        dhat = c2 * beta_j[None, :]
        delta = c1 * dhat + s1 * a
        gbar = -s1 * dhat + c1 * a
        gamma = np.hypot(gbar, beta_next[None, :])
        c = gbar / gamma
        s = beta_next[None, :] / gamma
        tau = c * phibar
        phibar_next = -s * phibar

        m = (pq[None] - delta[:, None, :] * m1 - eps[:, None, :] * m2) / gamma[:, None, :]
        upd = active[None, :] & ~frozen                # (Q, S) shifts still moving
        X += np.where(upd[:, None, :], tau[:, None, :] * m, 0.0)

        act = active[None, :]
        m2 = np.where(act[:, None, :], m1, m2)
        m1 = np.where(act[:, None, :], m, m1)
        c2 = np.where(act, c1, c2); s2 = np.where(act, s1, s2)
        c1 = np.where(act, c, c1); s1 = np.where(act, s, s1)
        phibar = np.where(act, phibar_next, phibar)
        with np.errstate(invalid="ignore", divide="ignore"):
            rr = np.abs(phibar) / np.where(nz, beta1, 1.0)[None, :]
        rel_res = np.where(upd, rr, rel_res)
        frozen = frozen | (upd & (rr <= tol))
        col_iters += active.astype(int)

        done = np.all(frozen, axis=0) | broke
        cont = active & ~done
        qn = np.zeros_like(q)
        qn[:, cont] = v[:, cont] / beta_next[cont]
        q_prev = np.where(cont[None, :], q, q_prev)
        q = np.where(cont[None, :], qn, q)
        if pinv is None:
            pq = q
        else:
            pn = np.zeros_like(q)
            pn[:, cont] = pv[:, cont] / beta_next[cont]
            pq = np.where(cont[None, :], pn, pq)
        beta_j = np.where(cont, beta_next, beta_j)
        frozen = frozen | (broke & active)[None, :]
        active = cont

    info = MinresInfo(iters, col_iters, frozen.copy(), rel_res, alphas, betas)
    if squeeze:
        X = X[:, :, 0]
    return X, info


def minres_dense_argmin(K: np.ndarray, b: np.ndarray, t: float, j: int) -> np.ndarray:
    """Brute force of (*) for tiny N: an orthonormal basis of K_j(K, b) by
    QR of the Krylov matrix with full re-orthogonalisation, then a dense
    least-squares solve. Independent of the recurrence above."""
    N = b.size
    basis = []
    v = b / np.linalg.norm(b)
    for _ in range(j):
        for u in basis:                    # twice is enough (Kahan-Parlett)
            v = v - (u @ v) * u
        for u in basis:
            v = v - (u @ v) * u
        nv = np.linalg.norm(v)
        if nv < 1e-13:
            break
        v = v / nv
        basis.append(v)
        v = K @ v
    V = np.stack(basis, axis=1)
    A = (K + t * np.eye(N)) @ V
    y, *_ = np.linalg.lstsq(A, b, rcond=None)
    return V @ y
