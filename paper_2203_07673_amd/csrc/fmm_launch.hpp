// Launcher for the line kernels: picks the compiled (L, NV, VW, U) variant for r,
// sizes the grid (chunk blocks first, then line blocks) and runs the merge of split
// lines.  Included only by the per-dtype instantiation units.
#pragma once

#include "fmm_internal.hpp"

namespace fmm {

// Entries loaded ahead per group: enough gathers in flight without spilling.  A lane
// holds U * NV vectors of 16 bytes per gathered matrix.
// Batch depth of class CLS (1 deep, 2 medium, 3 shallow): entries per batch for the
// one-row passes, half that for the two-row passes, divided by the vectors per lane.
template <int OP, int NV, int CLS> constexpr int unroll_for() {
    constexpr bool two = (OP == OP_SPMM2 || OP == OP_FUSED2);
    constexpr int one = CLS == 1 ? 8 : CLS == 2 ? 4 : 2;
    constexpr int u = (two ? one / 2 : one) / NV;
    return u < 1 ? 1 : u;
}

template <int OP, class TH, class TG1, class TG2, class Acc, int L, int NV, int VW, int U>
hipError_t launch_one(const LineArgs &a, hipStream_t stream)
{
    constexpr int GPB = kBlock / L;
    const int64_t nb_chunk = a.n_chunks > 0 ? ((int64_t)a.n_chunks + GPB - 1) / GPB : 0;
    const int64_t nb_line = ((int64_t)a.nlines + GPB - 1) / GPB;
    const int64_t nb = nb_chunk + nb_line;
    if (nb == 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((line_kernel<OP, TH, TG1, TG2, Acc, L, NV, VW, U>), dim3((unsigned)nb), dim3(kBlock), 0,
                       stream, a, (int32_t)nb_chunk);
    return hipGetLastError();
}

#define FMM_SHAPE_CASE(Lv, NVv)                                                                  \
    if (shape.L == Lv && shape.NV == NVv) {                                                      \
        if (a.uclass == 1) return launch_one<OP, TH, TG1, TG2, Acc, Lv, NVv, VW, unroll_for<OP, NVv, 1>()>(a, stream); \
        if (a.uclass == 2) return launch_one<OP, TH, TG1, TG2, Acc, Lv, NVv, VW, unroll_for<OP, NVv, 2>()>(a, stream); \
        return launch_one<OP, TH, TG1, TG2, Acc, Lv, NVv, VW, unroll_for<OP, NVv, 3>()>(a, stream);                    \
    }

template <int OP, class TH, class TG1, class TG2, class Acc, int VW>
hipError_t launch_shape(const LineArgs &a, Shape shape, hipStream_t stream)
{
    FMM_SHAPE_CASE(1, 1)
    FMM_SHAPE_CASE(2, 1)
    FMM_SHAPE_CASE(4, 1)
    FMM_SHAPE_CASE(8, 1)
    FMM_SHAPE_CASE(16, 1)
    FMM_SHAPE_CASE(32, 1)
    FMM_SHAPE_CASE(64, 1)
    FMM_SHAPE_CASE(16, 2)
    FMM_SHAPE_CASE(32, 2)
    FMM_SHAPE_CASE(64, 2)
    FMM_SHAPE_CASE(64, 4)
    return hipErrorInvalidValue;
}
#undef FMM_SHAPE_CASE

// Smallest element size among the operands decides the vector width (16-byte loads).
template <class TH, class TG1, class TG2> constexpr int vector_width() {
    constexpr int a = (int)sizeof(TH), b = (int)sizeof(TG1), c = (int)sizeof(TG2);
    constexpr int mn = a < b ? (a < c ? a : c) : (b < c ? b : c);
    return 16 / mn;
}

template <int OP, class TH, class TG1, class TG2, class Acc>
hipError_t launch_lines(const LineArgs &a, int32_t n_splits, const int32_t *splits, Shape hint,
                        hipStream_t stream)
{
    constexpr int VWV = vector_width<TH, TG1, TG2>();
    constexpr bool has_bf16 = sizeof(TH) == 2 || sizeof(TG1) == 2 || sizeof(TG2) == 2;
    const bool vector_path = (a.r % VWV) == 0;
    const int vw = vector_path ? VWV : 1;
    const Shape shape = shape_supported(hint, a.r, vw) ? hint : default_shape(a.r, vw);
    if (!shape_supported(shape, a.r, vw)) return hipErrorInvalidValue;
    hipError_t e;
    if (vector_path) {
        e = launch_shape<OP, TH, TG1, TG2, Acc, VWV>(a, shape, stream);
    } else {
        if constexpr (has_bf16) {
            return hipErrorInvalidValue;  // bfloat16 storage has no scalar path
        } else {
            e = launch_shape<OP, TH, TG1, TG2, Acc, 1>(a, shape, stream);
        }
    }
    if (e != hipSuccess) return e;
    if (OP != OP_SDDMM && n_splits > 0 && a.out != nullptr) {
        const int64_t total = (int64_t)n_splits * a.r;
        const int64_t nb = (total + kBlock - 1) / kBlock;
        hipLaunchKernelGGL((merge_kernel<Acc>), dim3((unsigned)nb), dim3(kBlock), 0, stream, splits, n_splits, a.r,
                           static_cast<const Acc *>(a.partial), static_cast<Acc *>(a.out), a.beta);
        e = hipGetLastError();
    }
    return e;
}

#define FMM_INSTANTIATE(OP, TH, TG1, TG2, Acc)                                                   \
    template hipError_t launch_lines<OP, TH, TG1, TG2, Acc>(const LineArgs &, int32_t, const int32_t *, \
                                                            Shape, hipStream_t);

}  // namespace fmm
