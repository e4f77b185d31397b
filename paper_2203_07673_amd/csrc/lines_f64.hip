// Line-kernel instantiations for float64 (the gradient-check path).
#include "fmm_launch.hpp"

namespace fmm {
FMM_INSTANTIATE(OP_SDDMM, double, double, double, double)
FMM_INSTANTIATE(OP_SPMM1, double, double, double, double)
FMM_INSTANTIATE(OP_SPMM2, double, double, double, double)
FMM_INSTANTIATE(OP_FUSED1, double, double, double, double)
FMM_INSTANTIATE(OP_FUSED2, double, double, double, double)
FMM_INSTANTIATE(OP_FUSED1S, double, double, double, double)
}  // namespace fmm
