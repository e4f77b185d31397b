// Line-kernel instantiations for bfloat16 storage of A and B (float32 values,
// gradients and outputs): the forward and unfused-baseline operand combinations.
#include "fmm_launch.hpp"

namespace fmm {
FMM_INSTANTIATE(OP_SDDMM, bf16_t, bf16_t, bf16_t, float)
FMM_INSTANTIATE(OP_SDDMM, float, bf16_t, bf16_t, float)
FMM_INSTANTIATE(OP_SDDMM, bf16_t, float, float, float)
FMM_INSTANTIATE(OP_SPMM1, bf16_t, bf16_t, bf16_t, float)
FMM_INSTANTIATE(OP_SPMM2, bf16_t, bf16_t, float, float)
}  // namespace fmm
