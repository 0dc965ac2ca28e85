// FP64 MFMA kernel product, CIQ_KERNEL_MATERN52, isotropic lengthscale.
#include "mvm_mfma.h"

namespace ciq {
hipError_t launch_mvm_f64_m52_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f64m_k<CIQ_KERNEL_MATERN52, false>(a, nsb, grid_x, st);
}
}  // namespace ciq
