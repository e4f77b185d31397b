// Line-kernel instantiations for bfloat16 storage of A and B: the fused passes.
#include "fmm_launch.hpp"

namespace fmm {
FMM_INSTANTIATE(OP_FUSED1, bf16_t, bf16_t, bf16_t, float)
FMM_INSTANTIATE(OP_FUSED1, float, bf16_t, bf16_t, float)
FMM_INSTANTIATE(OP_FUSED2, bf16_t, bf16_t, float, float)
FMM_INSTANTIATE(OP_FUSED2, bf16_t, bf16_t, bf16_t, float)  // bfloat16 upstream gradient
FMM_INSTANTIATE(OP_FUSED1S, float, bf16_t, bf16_t, float)
FMM_INSTANTIATE(OP_CG, float, bf16_t, bf16_t, float)
}  // namespace fmm
