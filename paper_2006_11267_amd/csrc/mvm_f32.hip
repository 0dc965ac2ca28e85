// FP32 MFMA kernel products with entries evaluated on the fly: RBF and
// Matern-5/2, isotropic and per-dimension lengthscales (one instantiation
// of the mvm_mfma.h kernels each).
#include "mvm_mfma.h"

namespace ciq {
hipError_t launch_mvm_f32_rbf_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f32_k<CIQ_KERNEL_RBF, false>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_f32_rbf_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f32_k<CIQ_KERNEL_RBF, true>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_f32_m52_iso(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f32_k<CIQ_KERNEL_MATERN52, false>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_f32_m52_ard(const MvmArgs& a, int nsb, int grid_x, hipStream_t st) {
    return mfma::launch_f32_k<CIQ_KERNEL_MATERN52, true>(a, nsb, grid_x, st);
}
}  // namespace ciq
