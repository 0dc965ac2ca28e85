// FP64 MFMA kernel product, CIQ_KERNEL_RBF, per-dimension lengthscale.
#include "mvm_mfma.h"

namespace ciq {
hipError_t launch_mvm_f64_rbf_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f64m_k<CIQ_KERNEL_RBF, true>(a, nsb, grid_x, st);
}
}  // namespace ciq
