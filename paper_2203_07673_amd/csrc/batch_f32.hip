// Batched persistent kernels, float32 storage.
#include "batch_kernels.hpp"

namespace fmm {

template <class TS, class TD, int L> static BatchKernelFn pick(int rw, int cw)
{
    constexpr int VW = 16 / (int)sizeof(TS);
    constexpr int W = 64 / L;
    if (!rw && !cw) return batch_kernel<TS, TD, L, VW, 1, 1>;
    if (!rw && cw) return batch_kernel<TS, TD, L, VW, 1, W>;
    if (rw && !cw) return batch_kernel<TS, TD, L, VW, W, 1>;
    return batch_kernel<TS, TD, L, VW, W, W>;
}

template <class TS, class TD, int L> static BatchQueueKernelFn pick_queue(int rw, int cw)
{
    constexpr int VW = 16 / (int)sizeof(TS);
    constexpr int W = 64 / L;
    if (!rw && !cw) return batch_queue_kernel<TS, TD, L, VW, 1, 1>;
    if (!rw && cw) return batch_queue_kernel<TS, TD, L, VW, 1, W>;
    if (rw && !cw) return batch_queue_kernel<TS, TD, L, VW, W, 1>;
    return batch_queue_kernel<TS, TD, L, VW, W, W>;
}

template <> BatchKernelFn batch_kernel_for<float, float>(int L, int rw, int cw)
{
    switch (L) {
    case 4: return pick<float, float, 4>(rw, cw);
    case 8: return pick<float, float, 8>(rw, cw);
    case 16: return pick<float, float, 16>(rw, cw);
    case 32: return pick<float, float, 32>(rw, cw);
    case 64: return pick<float, float, 64>(rw, cw);
    default: return nullptr;
    }
}

template <> BatchQueueKernelFn batch_queue_kernel_for<float, float>(int L, int rw, int cw)
{
    switch (L) {
    case 4: return pick_queue<float, float, 4>(rw, cw);
    case 8: return pick_queue<float, float, 8>(rw, cw);
    case 16: return pick_queue<float, float, 16>(rw, cw);
    case 32: return pick_queue<float, float, 32>(rw, cw);
    case 64: return pick_queue<float, float, 64>(rw, cw);
    default: return nullptr;
    }
}

}  // namespace fmm
