// Kernel instantiation for one storage precision (see lbm_kernels_impl.h).
#include "lbm_kernels_impl.h"

namespace lbm {
LBM_INSTANTIATE(f32, float, float)
}  // namespace lbm
