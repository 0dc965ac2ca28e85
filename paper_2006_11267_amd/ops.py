"""Python entry points with the C ABI's names (include/ciq.h), taking torch
tensors for device memory and torch's current stream. Marshalling only."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


def _stream() -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t: torch.Tensor, precision: Optional[str]) -> int:
    if precision is not None:
        return L.DTYPES[precision]
    if t.dtype == torch.float64:
        return L.CIQ_F64
    if t.dtype == torch.float32:
        return L.CIQ_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _elem_dtype(code: int) -> torch.dtype:
    return torch.float64 if code == L.CIQ_F64 else torch.float32


@dataclass
class Problem:
    """K = outputscale * k(X, X) + noise * I with X a device tensor (n x d)."""

    x: torch.Tensor
    kernel: str = "rbf"
    lengthscale: Sequence[float] = (1.0,)
    outputscale: float = 1.0
    noise: float = 0.0

    def c_struct(self):
        x = self.x
        if not (x.is_cuda and x.dim() == 2 and x.is_contiguous()):
            raise ValueError("x must be a contiguous 2-D device tensor")
        ls = np.ascontiguousarray(np.asarray(self.lengthscale, dtype=np.float64).reshape(-1))
        arr = (ctypes.c_double * ls.size)(*ls.tolist())
        p = L.ciq_problem(
            n=x.shape[0], d=x.shape[1], x=ctypes.c_void_p(x.data_ptr()), kernel=L.KERNELS[self.kernel],
            n_lengthscale=ls.size, lengthscale=ctypes.cast(arr, ctypes.POINTER(ctypes.c_double)),
            outputscale=float(self.outputscale), noise=float(self.noise))
        return p, arr  # keep arr alive with p


BASIS_MODES = {"auto": 0, "off": 1}


def _opts(dtype_code, q, max_iter, tol, lanczos_steps=0, seed=0, bounds=None, check_every=0, profile=False,
          kernel_cache="auto", cache_budget_mib=0, graph=False, precond_rank=0, krylov_basis="auto"):
    o = L.ciq_opts()
    o.dtype = dtype_code
    o.q = int(q)
    o.max_iter = int(max_iter)
    o.tol = float(tol)
    o.lanczos_steps = int(lanczos_steps)
    o.seed = int(seed)
    if bounds is not None:
        o.lambda_min, o.lambda_max = float(bounds[0]), float(bounds[1])
    o.check_every = int(check_every)
    o.profile = 1 if profile else 0
    o.kernel_cache = L.CACHE_MODES[kernel_cache]
    o.cache_budget_mib = int(cache_budget_mib)
    o.graph = 1 if graph else 0
    o.precond_rank = int(precond_rank)
    o.krylov_basis = BASIS_MODES[krylov_basis]
    return o


def ciq_version() -> int:
    return L.load().ciq_version()


def ciq_release_workspace(device: Optional[int] = None) -> None:
    """Free the device memory the library keeps between calls (resident Krylov
    basis chunks, their logs, the iteration scratch) on `device` (default: the
    current one)."""
    dev = torch.cuda.current_device() if device is None else int(device)
    L.check(L.load().ciq_release_workspace(dev), "ciq_release_workspace")


def ciq_setup(lambda_min: float, lambda_max: float, q: int):
    """HHT shifts t (ascending) and weights w (host FP64)."""
    lib = L.load()
    t = (ctypes.c_double * q)()
    w = (ctypes.c_double * q)()
    L.check(lib.ciq_setup(float(lambda_min), float(lambda_max), int(q), t, w), "ciq_setup")
    return np.array(t[:]), np.array(w[:])


def ciq_kernel_mvm(problem: Problem, v: torch.Tensor, precision: Optional[str] = None) -> torch.Tensor:
    """Y = K V (on the current stream, asynchronous)."""
    lib = L.load()
    code = _dtype_code(problem.x, precision)
    v2 = v if v.dim() == 2 else v.reshape(-1, 1)
    y = torch.empty(v2.shape, dtype=_elem_dtype(code), device=v.device)
    p, keep = problem.c_struct()
    L.check(lib.ciq_kernel_mvm(ctypes.byref(p), code, ctypes.c_void_p(v2.data_ptr()), v2.shape[1],
                               v2.stride(0), ctypes.c_void_p(y.data_ptr()), y.stride(0), _stream()),
            "ciq_kernel_mvm")
    del keep
    return y.reshape(v.shape)


def ciq_kernel_mvm_noalloc(problem: Problem, v: torch.Tensor, y: torch.Tensor,
                           precision: Optional[str] = None) -> torch.Tensor:
    """Y = K V into the caller's y with no device allocation inside the call
    (static scratch; on the current stream, asynchronous)."""
    lib = L.load()
    code = _dtype_code(problem.x, precision)
    v2 = v if v.dim() == 2 else v.reshape(-1, 1)
    y2 = y if y.dim() == 2 else y.reshape(-1, 1)
    if y2.shape != v2.shape or y2.dtype != _elem_dtype(code) or not y2.is_cuda:
        raise ValueError("y must be a device tensor of v's shape and the dtype's element type")
    p, keep = problem.c_struct()
    L.check(lib.ciq_kernel_mvm_noalloc(ctypes.byref(p), code, ctypes.c_void_p(v2.data_ptr()), v2.shape[1],
                                       v2.stride(0), ctypes.c_void_p(y2.data_ptr()), y2.stride(0), _stream()),
            "ciq_kernel_mvm_noalloc")
    del keep
    return y


def ciq_kernel_mvm_resident(problem: Problem, v: torch.Tensor, precision: Optional[str] = None) -> torch.Tensor:
    """Y = K V through the solvers' resident-matrix product (K written once for
    the call, then streamed); synchronous."""
    lib = L.load()
    code = _dtype_code(problem.x, precision)
    v2 = v if v.dim() == 2 else v.reshape(-1, 1)
    y = torch.empty(v2.shape, dtype=_elem_dtype(code), device=v.device)
    p, keep = problem.c_struct()
    L.check(lib.ciq_kernel_mvm_resident(ctypes.byref(p), code, ctypes.c_void_p(v2.data_ptr()), v2.shape[1],
                                        v2.stride(0), ctypes.c_void_p(y.data_ptr()), y.stride(0), _stream()),
            "ciq_kernel_mvm_resident")
    del keep
    return y.reshape(v.shape)


def ciq_eig_bounds(problem: Problem, steps: int = 20, v0: Optional[torch.Tensor] = None, seed: int = 0,
                   precision: Optional[str] = None):
    lib = L.load()
    code = _dtype_code(problem.x, precision)
    p, keep = problem.c_struct()
    lo, hi = ctypes.c_double(), ctypes.c_double()
    vp = ctypes.c_void_p(v0.data_ptr()) if v0 is not None else None
    L.check(lib.ciq_eig_bounds(ctypes.byref(p), code, int(steps), vp, int(seed), ctypes.byref(lo),
                               ctypes.byref(hi), _stream()), "ciq_eig_bounds")
    del keep
    return lo.value, hi.value


def _solve(fn_name, problem, b, q, max_iter, tol, precision, bounds, keep_solves, lanczos_steps, seed,
           check_every, profile, kernel_cache, cache_budget_mib, graph, precond_rank, krylov_basis="auto"):
    lib = L.load()
    code = _dtype_code(problem.x, precision)
    b2 = b if b.dim() == 2 else b.reshape(-1, 1)
    if b2.stride(1) != 1:
        b2 = b2.contiguous()
    n, s = b2.shape
    out = torch.empty((n, s), dtype=_elem_dtype(code), device=b.device)
    solves = torch.empty((n, q, s), dtype=_elem_dtype(code), device=b.device) if keep_solves else None
    p, keep = problem.c_struct()
    o = _opts(code, q, max_iter, tol, lanczos_steps, seed, bounds, check_every, profile, kernel_cache,
              cache_budget_mib, graph, precond_rank, krylov_basis)
    info = L.ciq_info()
    fn = getattr(lib, fn_name)
    L.check(fn(ctypes.byref(p), ctypes.byref(o), ctypes.c_void_p(b2.data_ptr()), s, b2.stride(0),
               ctypes.c_void_p(out.data_ptr()), out.stride(0),
               ctypes.c_void_p(solves.data_ptr()) if solves is not None else None, ctypes.byref(info), _stream()),
            fn_name)
    del keep
    return out.reshape(b.shape), info.as_dict(), solves


def ciq_invsqrt_mvm(problem: Problem, b: torch.Tensor, q: int = 15, max_iter: int = 200, tol: float = 1e-4,
                    precision: Optional[str] = None, bounds=None, keep_solves: bool = False,
                    lanczos_steps: int = 0, seed: int = 0, check_every: int = 0, profile: bool = False,
                    kernel_cache: str = "auto", cache_budget_mib: int = 0, graph: bool = False,
                    precond_rank: int = 0, krylov_basis: str = "auto"):
    """K^{-1/2} B -> (out, info, solves or None). With precond_rank > 0 the
    output is R' B, R' R'^T = K^{-1} (K^{-1/2} B up to a rotation)."""
    return _solve("ciq_invsqrt_mvm", problem, b, q, max_iter, tol, precision, bounds, keep_solves,
                  lanczos_steps, seed, check_every, profile, kernel_cache, cache_budget_mib, graph, precond_rank,
                  krylov_basis)


def ciq_sqrt_mvm(problem: Problem, b: torch.Tensor, q: int = 15, max_iter: int = 200, tol: float = 1e-4,
                 precision: Optional[str] = None, bounds=None, keep_solves: bool = False,
                 lanczos_steps: int = 0, seed: int = 0, check_every: int = 0, profile: bool = False,
                 kernel_cache: str = "auto", cache_budget_mib: int = 0, graph: bool = False,
                 precond_rank: int = 0, krylov_basis: str = "auto"):
    """K^{1/2} B -> (out, info, solves or None). With precond_rank > 0 the
    output is R B, R R^T = K (K^{1/2} B up to a rotation)."""
    return _solve("ciq_sqrt_mvm", problem, b, q, max_iter, tol, precision, bounds, keep_solves,
                  lanczos_steps, seed, check_every, profile, kernel_cache, cache_budget_mib, graph, precond_rank,
                  krylov_basis)


def ciq_posterior_mvm(candidates: Problem, x_obs: torch.Tensor, obs_noise: float, b: torch.Tensor,
                      mode: str = "sqrt", q: int = 15, max_iter: int = 200, tol: float = 1e-4,
                      precision: Optional[str] = None, bounds=None, lanczos_steps: int = 0, seed: int = 0,
                      check_every: int = 0, profile: bool = False, kernel_cache: str = "auto",
                      cache_budget_mib: int = 0, graph: bool = False, krylov_basis: str = "auto"):
    """Sigma^{1/2} B (mode "sqrt") or Sigma^{-1/2} B ("invsqrt") for the GP
    posterior covariance at the candidates given observations at x_obs
    (candidates.noise is the jitter) -> (out, info)."""
    lib = L.load()
    code = _dtype_code(candidates.x, precision)
    if not (x_obs.is_cuda and x_obs.dim() == 2 and x_obs.is_contiguous() and x_obs.dtype == candidates.x.dtype):
        raise ValueError("x_obs must be a contiguous 2-D device tensor of the candidates' dtype")
    b2 = b if b.dim() == 2 else b.reshape(-1, 1)
    if b2.stride(1) != 1:
        b2 = b2.contiguous()
    n, s = b2.shape
    out = torch.empty((n, s), dtype=_elem_dtype(code), device=b.device)
    p, keep = candidates.c_struct()
    o = _opts(code, q, max_iter, tol, lanczos_steps, seed, bounds, check_every, profile, kernel_cache,
              cache_budget_mib, graph, krylov_basis=krylov_basis)
    info = L.ciq_info()
    mode_code = L.CIQ_SQRT if mode == "sqrt" else L.CIQ_INVSQRT
    L.check(lib.ciq_posterior_mvm(ctypes.byref(p), ctypes.c_void_p(x_obs.data_ptr()), x_obs.shape[0],
                                  float(obs_noise), mode_code, ctypes.byref(o), ctypes.c_void_p(b2.data_ptr()), s,
                                  b2.stride(0), ctypes.c_void_p(out.data_ptr()), out.stride(0), ctypes.byref(info),
                                  _stream()), "ciq_posterior_mvm")
    del keep
    return out.reshape(b.shape), info.as_dict()


def ciq_csr_mvm(row_ptr: torch.Tensor, col_idx: torch.Tensor, val: torch.Tensor, b: torch.Tensor,
                mode: str = "invsqrt", q: int = 15, max_iter: int = 400, tol: float = 1e-4, bounds=None,
                lanczos_steps: int = 0, seed: int = 0, check_every: int = 0, profile: bool = False,
                graph: bool = False, krylov_basis: str = "auto"):
    """A^{-1/2} B ("invsqrt") or A^{1/2} B ("sqrt") for a sparse symmetric
    positive-definite A given in CSR form (int32 indices, float64 values,
    device tensors) -> (out, info)."""
    lib = L.load()
    for t_, dt in ((row_ptr, torch.int32), (col_idx, torch.int32), (val, torch.float64), (b, torch.float64)):
        if not (t_.is_cuda and t_.dtype == dt):
            raise ValueError("row_ptr/col_idx: int32, val/b: float64, all device tensors")
    n = row_ptr.numel() - 1
    b2 = b if b.dim() == 2 else b.reshape(-1, 1)
    if b2.stride(1) != 1:
        b2 = b2.contiguous()
    s = b2.shape[1]
    out = torch.empty((n, s), dtype=torch.float64, device=b.device)
    a = L.ciq_csr(n=n, nnz=col_idx.numel(), row_ptr=ctypes.c_void_p(row_ptr.data_ptr()),
                  col_idx=ctypes.c_void_p(col_idx.data_ptr()), val=ctypes.c_void_p(val.data_ptr()))
    o = _opts(L.CIQ_F64, q, max_iter, tol, lanczos_steps, seed, bounds, check_every, profile, graph=graph,
              krylov_basis=krylov_basis)
    info = L.ciq_info()
    mode_code = L.CIQ_SQRT if mode == "sqrt" else L.CIQ_INVSQRT
    L.check(lib.ciq_csr_mvm(ctypes.byref(a), mode_code, ctypes.byref(o), ctypes.c_void_p(b2.data_ptr()), s,
                            b2.stride(0), ctypes.c_void_p(out.data_ptr()), out.stride(0), ctypes.byref(info),
                            _stream()), "ciq_csr_mvm")
    return out.reshape(b.shape), info.as_dict()


def ciq_svgp_predict(inducing: Problem, x: torch.Tensor, theta: torch.Tensor, Theta: torch.Tensor, q: int = 15,
                     max_iter: int = 200, tol: float = 1e-4, precision: Optional[str] = None, bounds=None,
                     solve_max_iter: int = 1000, solve_tol: float = 1e-8, want_a: bool = False,
                     kernel_cache: str = "auto", seed: int = 0):
    """Whitened SVGP predictive mean and variance at x from natural parameters
    (theta, Theta) -> (mean, var, a or None, info, info_solve)."""
    lib = L.load()
    code = _dtype_code(inducing.x, precision)
    if not (x.is_cuda and x.dim() == 2 and x.is_contiguous() and x.dtype == inducing.x.dtype):
        raise ValueError("x must be a contiguous 2-D device tensor of the inducing points' dtype")
    M, nb = inducing.x.shape[0], x.shape[0]
    th = theta.to(torch.float64).contiguous()
    Th = Theta.to(torch.float64).contiguous()
    mean = torch.empty(nb, dtype=torch.float64, device=x.device)
    var = torch.empty(nb, dtype=torch.float64, device=x.device)
    a = torch.empty((M, nb), dtype=torch.float64, device=x.device) if want_a else None
    p, keep = inducing.c_struct()
    o = _opts(code, q, max_iter, tol, 0, seed, bounds, 0, False, kernel_cache)
    info, info_s = L.ciq_info(), L.ciq_info()
    L.check(lib.ciq_svgp_predict(ctypes.byref(p), ctypes.c_void_p(x.data_ptr()), nb, ctypes.c_void_p(th.data_ptr()),
                                 ctypes.c_void_p(Th.data_ptr()), ctypes.byref(o), int(solve_max_iter),
                                 float(solve_tol), ctypes.c_void_p(mean.data_ptr()), ctypes.c_void_p(var.data_ptr()),
                                 ctypes.c_void_p(a.data_ptr()) if a is not None else None, ctypes.byref(info),
                                 ctypes.byref(info_s), _stream()), "ciq_svgp_predict")
    del keep
    return mean, var, a, info.as_dict(), info_s.as_dict()


def ciq_svgp_ngd_step(a: torch.Tensor, mean: torch.Tensor, c_mean: torch.Tensor, c_var: torch.Tensor,
                      theta: torch.Tensor, Theta: torch.Tensor, scale: float, step: float):
    """One App. E natural-gradient step, updating theta (M) and Theta (M x M)
    in place from a (M x nb), mean, c_mean, c_var (nb); all float64 device
    tensors. Returns (theta, Theta)."""
    lib = L.load()
    M, nb = a.shape
    for t, shape in ((a, (M, nb)), (mean, (nb,)), (c_mean, (nb,)), (c_var, (nb,)), (theta, (M,)), (Theta, (M, M))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError("float64 contiguous device tensors of the documented shapes are required")
    L.check(lib.ciq_svgp_ngd_step(M, nb, ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(mean.data_ptr()),
                                  ctypes.c_void_p(c_mean.data_ptr()), ctypes.c_void_p(c_var.data_ptr()),
                                  float(scale), float(step), ctypes.c_void_p(theta.data_ptr()),
                                  ctypes.c_void_p(Theta.data_ptr()), _stream()), "ciq_svgp_ngd_step")
    return theta, Theta


def ciq_pivoted_cholesky(problem: Problem, rank: int):
    """Rank-`rank` partial pivoted Cholesky factor of outputscale * k(X, X):
    (Lbar as an n x rank float64 device tensor, pivots (numpy, -1 after a
    stop), trace of the residual)."""
    lib = L.load()
    n = problem.x.shape[0]
    code = L.CIQ_F64 if problem.x.dtype == torch.float64 else L.CIQ_F32
    lbar = torch.empty((n, int(rank)), dtype=torch.float64, device=problem.x.device)
    piv = (ctypes.c_int * int(rank))()
    tr = ctypes.c_double()
    p, keep = problem.c_struct()
    L.check(lib.ciq_pivoted_cholesky(ctypes.byref(p), code, int(rank), ctypes.c_void_p(lbar.data_ptr()), piv,
                                     ctypes.byref(tr), _stream()), "ciq_pivoted_cholesky")
    del keep
    return lbar, np.array(piv[:], dtype=np.int64), tr.value


def ciq_invsqrt_mvm_batched(problems: Sequence[Problem], bs: Sequence[torch.Tensor], q: int = 12,
                            max_iter: int = 1000, tol: float = 1e-4, bounds=None, lanczos_steps: int = 0,
                            seed: int = 0, check_every: int = 0, profile: bool = False, graph: bool = True,
                            kernel_cache: str = "auto"):
    """[K_p^{-1/2} B_p] for independent problems in one run -> (outs, infos).
    The iteration's kernels (one persistent product over all problems' row
    blocks, inner products, scalar stage, update) are replayed from a HIP
    graph unless graph=False or profile=True."""
    lib = L.load()
    P = len(problems)
    s = bs[0].shape[1]
    structs, keeps = [], []
    for pr in problems:
        c, k = pr.c_struct()
        structs.append(c)
        keeps.append(k)
    parr = (L.ciq_problem * P)(*structs)
    bcont = [b.contiguous() for b in bs]
    outs = [torch.empty_like(b) for b in bcont]
    bp = (ctypes.c_void_p * P)(*[b.data_ptr() for b in bcont])
    op = (ctypes.c_void_p * P)(*[o.data_ptr() for o in outs])
    infos = (L.ciq_info * P)()
    o = _opts(L.CIQ_F32, q, max_iter, tol, lanczos_steps, seed, bounds, check_every, profile, graph=graph,
              kernel_cache=kernel_cache)
    L.check(lib.ciq_invsqrt_mvm_batched(P, parr, ctypes.byref(o), bp, s, op, infos, _stream()),
            "ciq_invsqrt_mvm_batched")
    del keeps
    return outs, [i.as_dict() for i in infos]


def ciq_backward(problem: Problem, g: torch.Tensor, t, w, solves: torch.Tensor, mode: str = "invsqrt",
                 max_iter: int = 200, tol: float = 1e-4, precision: Optional[str] = None, want_b: bool = True,
                 want_hyper: bool = True, check_every: int = 0, kernel_cache: str = "auto"):
    """VJP of a forward call: returns (dB or None, dlengthscale, doutputscale, dnoise, info)."""
    lib = L.load()
    code = _dtype_code(problem.x, precision)
    g2 = g if g.dim() == 2 else g.reshape(-1, 1)
    if g2.stride(1) != 1:
        g2 = g2.contiguous()
    n, s = g2.shape
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64))
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64))
    q = t.size
    tc = (ctypes.c_double * q)(*t.tolist())
    wc = (ctypes.c_double * q)(*w.tolist())
    db = torch.empty((n, s), dtype=_elem_dtype(code), device=g.device) if want_b else None
    nls = np.asarray(problem.lengthscale).size
    dls = (ctypes.c_double * nls)()
    do2 = ctypes.c_double()
    dn = ctypes.c_double()
    p, keep = problem.c_struct()
    o = _opts(code, q, max_iter, tol, check_every=check_every, kernel_cache=kernel_cache)
    info = L.ciq_info()
    mode_code = L.CIQ_SQRT if mode == "sqrt" else L.CIQ_INVSQRT
    sol = solves.contiguous()
    L.check(lib.ciq_backward(ctypes.byref(p), ctypes.byref(o), mode_code, tc, wc, ctypes.c_void_p(sol.data_ptr()),
                             ctypes.c_void_p(g2.data_ptr()), s, g2.stride(0),
                             ctypes.c_void_p(db.data_ptr()) if db is not None else None, s,
                             dls if want_hyper else None, ctypes.byref(do2) if want_hyper else None,
                             ctypes.byref(dn) if want_hyper else None, ctypes.byref(info), _stream()),
            "ciq_backward")
    del keep
    dB = db.reshape(g.shape) if db is not None else None
    if not want_hyper:
        return dB, None, None, None, info.as_dict()
    return dB, np.array(dls[:]), do2.value, dn.value, info.as_dict()
