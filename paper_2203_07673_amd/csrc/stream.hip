// Plain streaming kernels that measure the HBM rate this GPU reaches on contiguous
// traffic: a copy (read + write) and a read-only pass.  The line kernels' rates are read
// against these ceilings as well as against the 8 TB/s specification.  A third probe
// gathers whole rows at listed indices, the access shape of the line kernels, so that
// hardware counters can be calibrated on a gather of known size.
#include <hip/hip_runtime.h>

#include "fmm_internal.hpp"

namespace fmm {
namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;      // 16-byte vectors in flight per lane (copy)
constexpr int kReadUnroll = 8;  // (read)

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kThreads) void stream_copy_kernel(const uint4 *__restrict__ src,
                                                               uint4 *__restrict__ dst, size_t n)
{
    const size_t step = (size_t)gridDim.x * kThreads * kUnroll;
    for (size_t base = (size_t)blockIdx.x * kThreads * kUnroll + threadIdx.x; base < n; base += step) {
        uint4 v[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const size_t i = base + (size_t)u * kThreads;
            if (i < n) v[u] = src[i];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const size_t i = base + (size_t)u * kThreads;
            if (i < n) dst[i] = v[u];
        }
    }
}

// Folds every loaded word into one value so that no load can be dropped; the value is
// stored only when it equals `key`, which keeps the pass free of writes in practice.
// Streaming (nontemporal) loads: data read once should not allocate in the caches, and
// on MI355X they reach a higher rate than default-policy loads.
__global__ __launch_bounds__(kThreads) void stream_read_kernel(const u32x4_t *__restrict__ src, size_t n,
                                                               uint32_t key, uint32_t *__restrict__ sink)
{
    const size_t step = (size_t)gridDim.x * kThreads * kReadUnroll;
    uint32_t acc = 0;
    for (size_t base = (size_t)blockIdx.x * kThreads * kReadUnroll + threadIdx.x; base < n; base += step) {
        u32x4_t v[kReadUnroll];
#pragma unroll
        for (int u = 0; u < kReadUnroll; ++u) {
            const size_t i = base + (size_t)u * kThreads;
            v[u] = i < n ? __builtin_nontemporal_load(src + i) : u32x4_t{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int u = 0; u < kReadUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    if (acc == key) sink[0] = acc;
}

// Rows of ROWV 16-byte vectors at the listed indices: one lane group of ROWV lanes per
// row, each lane one vector, default cache policy (as the line kernels' gathers).  Every
// loaded word is folded into one value, stored only when it equals `key`.
template <int ROWV>
__global__ __launch_bounds__(kThreads) void gather_rows_kernel(const u32x4_t *__restrict__ src,
                                                               const int32_t *__restrict__ rows, int64_t n_rows,
                                                               uint32_t key, uint32_t *__restrict__ sink)
{
    constexpr int kRowsPerBlock = kThreads / ROWV;
    const int lane = threadIdx.x % ROWV;
    const int64_t step = (int64_t)gridDim.x * kRowsPerBlock;
    uint32_t acc = 0;
    for (int64_t k = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / ROWV; k < n_rows; k += step) {
        const u32x4_t v = src[(size_t)rows[k] * ROWV + lane];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (acc == key) sink[0] = acc;
}

hipError_t stream_grid(size_t n, int unroll, unsigned *blocks)
{
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t per_block = (size_t)kThreads * unroll;
    const size_t need = (n + per_block - 1) / per_block;
    const size_t cap = (size_t)(cus > 0 ? cus : 1) * 16;  // 16 workgroups per compute unit
    *blocks = (unsigned)(need < cap ? need : cap);
    return hipSuccess;
}

fmm_status stream_status(hipError_t e)
{
    if (e == hipSuccess) return FMM_OK;
    set_last_hip_error((int32_t)e);
    return FMM_ERR_HIP;
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" {

fmm_status fmm_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t stream)
{
    if (bytes == 0) return FMM_OK;
    if (!src || !dst) return FMM_ERR_NULL;
    if (bytes % 16 != 0) return FMM_ERR_DIM;
    if ((uintptr_t)src % 16 != 0 || (uintptr_t)dst % 16 != 0) return FMM_ERR_UNSUPPORTED;
    const size_t n = bytes / 16;
    unsigned blocks = 0;
    hipError_t e = stream_grid(n, kUnroll, &blocks);
    if (e != hipSuccess) return stream_status(e);
    hipLaunchKernelGGL(stream_copy_kernel, dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const uint4 *>(src), static_cast<uint4 *>(dst), n);
    return stream_status(hipGetLastError());
}

fmm_status fmm_stream_read(const void *src, size_t bytes, uint32_t key, uint32_t *sink, hipStream_t stream)
{
    if (bytes == 0) return FMM_OK;
    if (!src || !sink) return FMM_ERR_NULL;
    if (bytes % 16 != 0) return FMM_ERR_DIM;
    if ((uintptr_t)src % 16 != 0) return FMM_ERR_UNSUPPORTED;
    const size_t n = bytes / 16;
    unsigned blocks = 0;
    hipError_t e = stream_grid(n, kReadUnroll, &blocks);
    if (e != hipSuccess) return stream_status(e);
    hipLaunchKernelGGL(stream_read_kernel, dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const u32x4_t *>(src), n, key, sink);
    return stream_status(hipGetLastError());
}

fmm_status fmm_stream_gather(const void *src, size_t row_bytes, const int32_t *rows, int64_t n_rows, uint32_t key,
                             uint32_t *sink, hipStream_t stream)
{
    if (n_rows == 0) return FMM_OK;
    if (!src || !rows || !sink) return FMM_ERR_NULL;
    if (n_rows < 0) return FMM_ERR_DIM;
    if ((uintptr_t)src % 16 != 0) return FMM_ERR_UNSUPPORTED;
    const int rowv = (int)(row_bytes / 16);
    if (row_bytes % 16 != 0 || rowv < 1 || rowv > 64 || (rowv & (rowv - 1)) != 0) return FMM_ERR_DIM;
    unsigned blocks = 0;
    hipError_t e = stream_grid((size_t)n_rows * rowv, 1, &blocks);
    if (e != hipSuccess) return stream_status(e);
    const u32x4_t *s = static_cast<const u32x4_t *>(src);
    switch (rowv) {
    case 1: hipLaunchKernelGGL(gather_rows_kernel<1>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    case 2: hipLaunchKernelGGL(gather_rows_kernel<2>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    case 4: hipLaunchKernelGGL(gather_rows_kernel<4>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    case 8: hipLaunchKernelGGL(gather_rows_kernel<8>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    case 16: hipLaunchKernelGGL(gather_rows_kernel<16>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    case 32: hipLaunchKernelGGL(gather_rows_kernel<32>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    default: hipLaunchKernelGGL(gather_rows_kernel<64>, dim3(blocks), dim3(kThreads), 0, stream, s, rows, n_rows, key, sink); break;
    }
    return stream_status(hipGetLastError());
}

}  // extern "C"
