// Kernel instantiation for one storage precision (see lbm_kernels_impl.h).
#include "lbm_kernels_impl.h"

namespace lbm {
LBM_INSTANTIATE(f16, _Float16, float)
}  // namespace lbm
