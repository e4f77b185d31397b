// Line-kernel instantiations for float32 storage (every operand float32).
#include "fmm_launch.hpp"

namespace fmm {
FMM_INSTANTIATE(OP_SDDMM, float, float, float, float)
FMM_INSTANTIATE(OP_SPMM1, float, float, float, float)
FMM_INSTANTIATE(OP_SPMM2, float, float, float, float)
FMM_INSTANTIATE(OP_FUSED1, float, float, float, float)
FMM_INSTANTIATE(OP_FUSED2, float, float, float, float)
FMM_INSTANTIATE(OP_FUSED1S, float, float, float, float)
FMM_INSTANTIATE(OP_CG, float, float, float, float)
}  // namespace fmm
