"""msMINRES-CIQ on MI355X (gfx950): K^{1/2} B and K^{-1/2} B for Gaussian-process
kernel matrices through a C-ABI HIP library (include/ciq.h, libciq.so).

The Python layer only marshals arguments (torch tensors supply device memory
and the current stream); all computation runs in the library.
"""
from ._lib import CIQError, load  # noqa: F401
from .ops import (  # noqa: F401
    Problem,
    ciq_csr_mvm,
    ciq_eig_bounds,
    ciq_invsqrt_mvm,
    ciq_invsqrt_mvm_batched,
    ciq_kernel_mvm,
    ciq_kernel_mvm_noalloc,
    ciq_kernel_mvm_resident,
    ciq_pivoted_cholesky,
    ciq_posterior_mvm,
    ciq_release_workspace,
    ciq_setup,
    ciq_sqrt_mvm,
    ciq_svgp_ngd_step,
    ciq_svgp_predict,
    ciq_version,
    ciq_backward,
)
from .autograd import CIQFunction, ciq_apply  # noqa: F401
