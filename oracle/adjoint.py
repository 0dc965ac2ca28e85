"""Backward pass of CIQ (oracle, FP64) and its two independent references.

Sec. 3.3: differentiating each term of the rational approximation,

    d<V, K^{-1/2}B>/dK ~= -1/2 sum_q w_q (t_q I + K)^{-1} (V B^T + B V^T) (t_q I + K)^{-1}
                       = -1/2 sum_q w_q (g_q a_q^T + a_q g_q^T),

with a_q = (t_q I + K)^{-1} B (the forward solves, saved) and
g_q = (t_q I + K)^{-1} V (one more msMINRES run on V). The gradient with
respect to B is sum_q w_q g_q (K symmetric). For the square root,
out = K A with A = sum_q w_q a_q: the upstream gradient is first pulled
through K (g <- K V) and the direct term 1/2 (V A^T + A V^T) is added.

Reading: ``ciq_vjp`` is the exact vector-Jacobian product of the quadrature
rule evaluated with the given solves; the gap to the derivative of the true
K^{-1/2} is the quadrature + solver error, checked separately.
"""
from __future__ import annotations

import numpy as np

from . import kernels as _k
from . import msminres as _ms


def ciq_vjp(mvm, A_solves, G, t, w, max_iter, tol, mode="invsqrt"):
    """Returns (dB, dK) for loss <G, out>; dK is the dense symmetric N x N gradient."""
    G = np.asarray(G, dtype=np.float64)
    w = np.asarray(w)
    Gin = mvm(G) if mode == "sqrt" else G
    Gq, _ = _ms.msminres(mvm, Gin, t, max_iter, tol)
    dB = np.tensordot(w, Gq, axes=1)
    dK = np.zeros((G.shape[0], G.shape[0]))
    for qi in range(len(w)):
        P = Gq[qi] @ A_solves[qi].T
        dK -= 0.5 * w[qi] * (P + P.T)
    if mode == "sqrt":
        A = np.tensordot(w, A_solves, axes=1)
        P = G @ A.T
        dK += 0.5 * (P + P.T)
    return dB, dK


def hyper_grads(kind, x, lengthscale, outputscale, dK):
    """Contract dL/dK with dK/dtheta: (d lengthscale [1 or d], d outputscale, d noise)."""
    x = np.asarray(x, dtype=np.float64)
    ls = np.asarray(lengthscale, dtype=np.float64).reshape(-1)
    dKdl = _k.kernel_lengthscale_grad(kind, x, ls, outputscale)
    g_ls = np.array([np.sum(dK * dKdl[d]) for d in range(x.shape[1])])
    if ls.size == 1:
        g_ls = np.array([g_ls.sum()])
    ku = _k.unit_kernel(kind, _k.scaled_sqdist(x, x, ls))
    return g_ls, float(np.sum(dK * ku)), float(np.trace(dK))


def daleckii_krein_vjp(K, B, G, divided_difference):
    """d<G, f(K) B>/dK = U (F o (U^T G B^T U)) U^T, symmetrised, with
    F_ij = (f(l_i) - f(l_j)) / (l_i - l_j) (f'(l_i) on the diagonal), supplied
    by ``divided_difference(l_i, l_j)`` as a stable closed form."""
    lam, U = np.linalg.eigh(K)
    E = U.T @ np.asarray(G, dtype=np.float64).reshape(K.shape[0], -1) \
        @ np.asarray(B, dtype=np.float64).reshape(K.shape[0], -1).T @ U
    F = divided_difference(lam[:, None], lam[None, :])
    D = U @ (F * E) @ U.T
    return 0.5 * (D + D.T)


def dd_invsqrt(li, lj):
    """Divided difference of f(l) = l^{-1/2}: -1 / (sqrt(li) sqrt(lj) (sqrt(li) + sqrt(lj)))."""
    a, b = np.sqrt(li), np.sqrt(lj)
    return -1.0 / (a * b * (a + b))


def dd_rational(t, w):
    """Divided difference of r_Q(l) = sum w_q/(t_q + l): -sum w_q / ((t_q + li)(t_q + lj))."""
    t = np.asarray(t); w = np.asarray(w)

    def f(li, lj):
        out = np.zeros(np.broadcast(li, lj).shape)
        for tq, wq in zip(t, w):
            out -= wq / ((tq + li) * (tq + lj))
        return out
    return f
