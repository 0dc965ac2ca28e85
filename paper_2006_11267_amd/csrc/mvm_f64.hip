// FP64 MFMA kernel products with entries evaluated on the fly: RBF and
// Matern-5/2, isotropic and per-dimension lengthscales.
#include "mvm_mfma.h"

namespace ciq {
hipError_t launch_mvm_f64_rbf_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f64m_k<CIQ_KERNEL_RBF, false>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_f64_rbf_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f64m_k<CIQ_KERNEL_RBF, true>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_f64_m52_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f64m_k<CIQ_KERNEL_MATERN52, false>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_f64_m52_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f64m_k<CIQ_KERNEL_MATERN52, true>(a, nsb, grid_x, st);
}
}  // namespace ciq
