// FP32 MFMA kernel product, CIQ_KERNEL_RBF, isotropic lengthscale.
#include "mvm_mfma.h"

namespace ciq {
hipError_t launch_mvm_f32_rbf_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f32_k<CIQ_KERNEL_RBF, false>(a, nsb, grid_x, st);
}
}  // namespace ciq
