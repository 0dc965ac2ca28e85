// Split-operand BF16 / FP16 kernel products: RBF and Matern-5/2.
#include "mvm_x3.h"

namespace ciq {
hipError_t launch_mvm_x3_rbf(const MvmArgs& a, int nsb, int grid_x, bool half, hipStream_t st) {
    if (half)
        return a.ard ? x3::launch_x3_k<CIQ_KERNEL_RBF, true, true>(a, nsb, grid_x, st)
                     : x3::launch_x3_k<CIQ_KERNEL_RBF, false, true>(a, nsb, grid_x, st);
    return a.ard ? x3::launch_x3_k<CIQ_KERNEL_RBF, true, false>(a, nsb, grid_x, st)
                 : x3::launch_x3_k<CIQ_KERNEL_RBF, false, false>(a, nsb, grid_x, st);
}

hipError_t launch_mvm_x3_m52(const MvmArgs& a, int nsb, int grid_x, bool half, hipStream_t st) {
    if (half)
        return a.ard ? x3::launch_x3_k<CIQ_KERNEL_MATERN52, true, true>(a, nsb, grid_x, st)
                     : x3::launch_x3_k<CIQ_KERNEL_MATERN52, false, true>(a, nsb, grid_x, st);
    return a.ard ? x3::launch_x3_k<CIQ_KERNEL_MATERN52, true, false>(a, nsb, grid_x, st)
                 : x3::launch_x3_k<CIQ_KERNEL_MATERN52, false, false>(a, nsb, grid_x, st);
}
}  // namespace ciq
