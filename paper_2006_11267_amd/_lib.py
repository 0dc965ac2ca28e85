"""ctypes binding of libciq (see include/ciq.h). Argument marshalling only:
every step of the computation runs in the HIP library. If the built library
is missing this module raises; there is no CPU fallback."""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libciq.so")

CIQ_OK, CIQ_EINVAL, CIQ_ENOMEM, CIQ_EHIP, CIQ_ENOTSUP, CIQ_ENUMERIC = range(6)
CIQ_KERNEL_RBF, CIQ_KERNEL_MATERN52 = 0, 1
CIQ_F64, CIQ_F32, CIQ_BF16X3, CIQ_F16X3 = 0, 1, 2, 3
CIQ_INVSQRT, CIQ_SQRT = 0, 1
CIQ_CACHE_AUTO, CIQ_CACHE_OFF, CIQ_CACHE_ON = 0, 1, 2
CACHE_MODES = {"auto": CIQ_CACHE_AUTO, "off": CIQ_CACHE_OFF, "on": CIQ_CACHE_ON}
CIQ_MAX_Q = 64
CIQ_MAX_D = 16
CIQ_MAX_RANK = 1024
CIQ_MAX_OBS = 4096
CIQ_NOALLOC_SCRATCH_BYTES = 64 << 20

KERNELS = {"rbf": CIQ_KERNEL_RBF, "matern52": CIQ_KERNEL_MATERN52}
DTYPES = {"f64": CIQ_F64, "f32": CIQ_F32, "bf16x3": CIQ_BF16X3, "f16x3": CIQ_F16X3}


class ciq_problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("d", ctypes.c_int32),
        ("x", ctypes.c_void_p),
        ("kernel", ctypes.c_int32),
        ("n_lengthscale", ctypes.c_int32),
        ("lengthscale", ctypes.POINTER(ctypes.c_double)),
        ("outputscale", ctypes.c_double),
        ("noise", ctypes.c_double),
    ]


class ciq_csr(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("nnz", ctypes.c_int32),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
    ]


class ciq_opts(ctypes.Structure):
    _fields_ = [
        ("dtype", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("tol", ctypes.c_double),
        ("lanczos_steps", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("check_every", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("kernel_cache", ctypes.c_int32),
        ("cache_budget_mib", ctypes.c_int32),
        ("graph", ctypes.c_int32),
        ("precond_rank", ctypes.c_int32),
        ("krylov_basis", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class ciq_info(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("converged", ctypes.c_int32),
        ("q", ctypes.c_int32),
        ("mvm_count", ctypes.c_int32),
        ("max_rel_residual", ctypes.c_double),
        ("lambda_min", ctypes.c_double),
        ("lambda_max", ctypes.c_double),
        ("t", ctypes.c_double * CIQ_MAX_Q),
        ("w", ctypes.c_double * CIQ_MAX_Q),
        ("mvm_ms", ctypes.c_double),
        ("mvm_timed", ctypes.c_int32),
        ("kernel_cached", ctypes.c_int32),
        ("precond_rank", ctypes.c_int32),
        ("precond_trace", ctypes.c_double),
        ("setup_ms", ctypes.c_double),
        ("krylov_basis", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        q = self.q
        return {
            "iters": self.iters,
            "converged": bool(self.converged),
            "q": q,
            "mvm_count": self.mvm_count,
            "max_rel_residual": self.max_rel_residual,
            "lambda_min": self.lambda_min,
            "lambda_max": self.lambda_max,
            "t": np.array(self.t[:q]),
            "w": np.array(self.w[:q]),
            "mvm_ms": self.mvm_ms,
            "mvm_timed": self.mvm_timed,
            "kernel_cached": bool(self.kernel_cached),
            "precond_rank": self.precond_rank,
            "precond_trace": self.precond_trace,
            "setup_ms": self.setup_ms,
            "krylov_basis": bool(self.krylov_basis),
        }


# Exported symbols and their prototypes (mirrors include/ciq.h).
_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
PROTOTYPES = {
    "ciq_version": (_I, []),
    "ciq_strerror": (ctypes.c_char_p, [_I]),
    "ciq_release_workspace": (_I, [_I]),
    "ciq_setup": (_I, [_D, _D, _I, _PD, _PD]),
    "ciq_kernel_mvm": (_I, [ctypes.POINTER(ciq_problem), _I, _VP, _I, _I, _VP, _I, _VP]),
    "ciq_kernel_mvm_resident": (_I, [ctypes.POINTER(ciq_problem), _I, _VP, _I, _I, _VP, _I, _VP]),
    "ciq_kernel_mvm_noalloc": (_I, [ctypes.POINTER(ciq_problem), _I, _VP, _I, _I, _VP, _I, _VP]),
    "ciq_eig_bounds": (_I, [ctypes.POINTER(ciq_problem), _I, _I, _VP, ctypes.c_uint64, _PD, _PD, _VP]),
    "ciq_invsqrt_mvm": (_I, [ctypes.POINTER(ciq_problem), ctypes.POINTER(ciq_opts), _VP, _I, _I, _VP, _I,
                             _VP, ctypes.POINTER(ciq_info), _VP]),
    "ciq_sqrt_mvm": (_I, [ctypes.POINTER(ciq_problem), ctypes.POINTER(ciq_opts), _VP, _I, _I, _VP, _I,
                          _VP, ctypes.POINTER(ciq_info), _VP]),
    "ciq_backward": (_I, [ctypes.POINTER(ciq_problem), ctypes.POINTER(ciq_opts), _I, _PD, _PD, _VP, _VP, _I,
                          _I, _VP, _I, _PD, _PD, _PD, ctypes.POINTER(ciq_info), _VP]),
    "ciq_invsqrt_mvm_batched": (_I, [_I, ctypes.POINTER(ciq_problem), ctypes.POINTER(ciq_opts),
                                     ctypes.POINTER(_VP), _I, ctypes.POINTER(_VP),
                                     ctypes.POINTER(ciq_info), _VP]),
    "ciq_pivoted_cholesky": (_I, [ctypes.POINTER(ciq_problem), _I, _I, _VP, ctypes.POINTER(ctypes.c_int), _PD,
                                  _VP]),
    "ciq_csr_mvm": (_I, [ctypes.POINTER(ciq_csr), _I, ctypes.POINTER(ciq_opts), _VP, _I, _I, _VP, _I,
                         ctypes.POINTER(ciq_info), _VP]),
    "ciq_svgp_predict": (_I, [ctypes.POINTER(ciq_problem), _VP, _I, _VP, _VP, ctypes.POINTER(ciq_opts), _I, _D, _VP,
                              _VP, _VP, ctypes.POINTER(ciq_info), ctypes.POINTER(ciq_info), _VP]),
    "ciq_svgp_ngd_step": (_I, [_I, _I, _VP, _VP, _VP, _VP, _D, _D, _VP, _VP, _VP]),
    "ciq_posterior_mvm": (_I, [ctypes.POINTER(ciq_problem), _VP, _I, _D, _I, ctypes.POINTER(ciq_opts), _VP, _I, _I,
                               _VP, _I, ctypes.POINTER(ciq_info), _VP]),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libciq.so (built in-tree by paper_2006_11267_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libciq is not built ({path} missing); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    for name, (res, args) in PROTOTYPES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class CIQError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        super().__init__(f"{where}: {lib.ciq_strerror(status).decode()}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != CIQ_OK:
        raise CIQError(status, where)
