// Alternating least squares support (Section VI-E of the paper): batched conjugate
// gradients whose query vectors M p for every line come from one pass over the sparse
// pattern (the batching of Zhao and Canny the paper adopts), and the Frobenius residual
// ||C~ - SDDMM(A, B, S)|| over the stored entries.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "fmm.h"
#include "fmm_internal.hpp"

namespace fmm {
namespace {

fmm_status hipfail(hipError_t e)
{
    set_last_hip_error((int32_t)e);
    return FMM_ERR_HIP;
}

template <int VW> struct F32v;
template <> struct F32v<1> {
    static __device__ __forceinline__ void ld(const float *p, float *o) { o[0] = p[0]; }
    static __device__ __forceinline__ void st(float *p, const float *o) { p[0] = o[0]; }
};
template <> struct F32v<4> {
    static __device__ __forceinline__ void ld(const float *p, float *o) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
    static __device__ __forceinline__ void st(float *p, const float *o) {
        *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
    }
};

// Start of CG for every line: R = rhs - (Q + lambda X) with Q = (sum_j F_j F_j^T) X,
// P = R, rr = <R, R>.
template <int L, int NV, int VW>
__global__ __launch_bounds__(kBlock) void cg_start_kernel(int32_t n, int32_t r, const float *__restrict__ rhs,
                                                          const float *__restrict__ Q, const float *__restrict__ X,
                                                          float lambda, float *__restrict__ R, float *__restrict__ P,
                                                          float *__restrict__ rr)
{
    const int lane = threadIdx.x % L;
    const int64_t row = (int64_t)blockIdx.x * (kBlock / L) + threadIdx.x / L;
    if (row >= n) return;
    const int C = r / VW;
    float dot = 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int c = v * L + lane;
        if (c >= C) continue;
        const int64_t o = row * r + c * VW;
        float b[VW], q[VW], x[VW], res[VW];
        F32v<VW>::ld(rhs + o, b);
        F32v<VW>::ld(Q + o, q);
        F32v<VW>::ld(X + o, x);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            res[e] = b[e] - (q[e] + lambda * x[e]);
            dot += res[e] * res[e];
        }
        F32v<VW>::st(R + o, res);
        F32v<VW>::st(P + o, res);
    }
    dot = group_sum<L>(dot);
    if (lane == 0) rr[row] = dot;
}

// One CG step for every line, given Q = (sum_j F_j F_j^T) P:
//   alpha = rr / <P, Q + lambda P>;  X += alpha P;  R -= alpha (Q + lambda P);
//   beta = <R, R>_new / rr;  P = R + beta P;  rr = <R, R>_new.
// A line whose residual or curvature is zero keeps its iterate (alpha = beta = 0).
template <int L, int NV, int VW>
__global__ __launch_bounds__(kBlock) void cg_step_kernel(int32_t n, int32_t r, float lambda, float *__restrict__ X,
                                                         float *__restrict__ R, float *__restrict__ P,
                                                         const float *__restrict__ Q, float *__restrict__ rr)
{
    constexpr int E = NV * VW;
    const int lane = threadIdx.x % L;
    const int64_t row = (int64_t)blockIdx.x * (kBlock / L) + threadIdx.x / L;
    if (row >= n) return;
    const int C = r / VW;
    float p[E], mq[E];
    float pq = 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int c = v * L + lane;
        float q[VW];
        if (c < C) {
            F32v<VW>::ld(P + row * r + c * VW, p + v * VW);
            F32v<VW>::ld(Q + row * r + c * VW, q);
        } else {
#pragma unroll
            for (int e = 0; e < VW; ++e) p[v * VW + e] = q[e] = 0.f;
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            mq[v * VW + e] = q[e] + lambda * p[v * VW + e];
            pq += p[v * VW + e] * mq[v * VW + e];
        }
    }
    pq = group_sum<L>(pq);
    const float rr_old = rr[row];
    const float alpha = (rr_old > 0.f && pq > 0.f) ? rr_old / pq : 0.f;
    float res[E];
    float rrn = 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int c = v * L + lane;
        if (c >= C) {
#pragma unroll
            for (int e = 0; e < VW; ++e) res[v * VW + e] = 0.f;
            continue;
        }
        const int64_t o = row * r + c * VW;
        float x[VW], rv[VW];
        F32v<VW>::ld(X + o, x);
        F32v<VW>::ld(R + o, rv);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            x[e] += alpha * p[v * VW + e];
            res[v * VW + e] = rv[e] - alpha * mq[v * VW + e];
            rrn += res[v * VW + e] * res[v * VW + e];
        }
        F32v<VW>::st(X + o, x);
        F32v<VW>::st(R + o, res + v * VW);
    }
    rrn = group_sum<L>(rrn);
    const float beta = rr_old > 0.f ? rrn / rr_old : 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int c = v * L + lane;
        if (c >= C) continue;
        float np[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) np[e] = res[v * VW + e] + beta * p[v * VW + e];
        F32v<VW>::st(P + row * r + c * VW, np);
    }
    if (lane == 0) rr[row] = rrn;
}

// Per-block partial sums of (val[p] - R[p])^2 in float64, then one block adds the
// partials in block order: a fixed summation order, so the result is reproducible.
__global__ __launch_bounds__(256) void residual_partial_kernel(int64_t nnz, const float *__restrict__ val,
                                                               const float *__restrict__ R, double *__restrict__ part)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * 256) {
        const double d = (double)(val ? val[p] : 1.f) - (double)R[p];
        acc += d * d;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void residual_final_kernel(int32_t nparts, const double *__restrict__ part,
                                                             double *__restrict__ out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += 256) acc += part[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

constexpr int kResidualBlocks = 1024;

template <int L, int NV, int VW>
hipError_t launch_cg(bool start, int32_t n, int32_t r, const float *rhs, const float *Q, float *X, float lambda,
                     float *R, float *P, float *rr, hipStream_t st)
{
    const unsigned nb = (unsigned)(((int64_t)n + kBlock / L - 1) / (kBlock / L));
    if (nb == 0) return hipSuccess;
    if (start)
        hipLaunchKernelGGL((cg_start_kernel<L, NV, VW>), dim3(nb), dim3(kBlock), 0, st, n, r, rhs, Q, X, lambda, R, P,
                           rr);
    else
        hipLaunchKernelGGL((cg_step_kernel<L, NV, VW>), dim3(nb), dim3(kBlock), 0, st, n, r, lambda, X, R, P, Q, rr);
    return hipGetLastError();
}

template <int VW>
hipError_t dispatch_cg(Shape sh, bool start, int32_t n, int32_t r, const float *rhs, const float *Q, float *X,
                       float lambda, float *R, float *P, float *rr, hipStream_t st)
{
#define CG_CASE(Lv, NVv)                                                                         \
    if (sh.L == Lv && sh.NV == NVv) return launch_cg<Lv, NVv, VW>(start, n, r, rhs, Q, X, lambda, R, P, rr, st);
    CG_CASE(1, 1) CG_CASE(2, 1) CG_CASE(4, 1) CG_CASE(8, 1) CG_CASE(16, 1) CG_CASE(32, 1) CG_CASE(64, 1)
    CG_CASE(64, 2) CG_CASE(64, 4)
#undef CG_CASE
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" {

fmm_status fmm_cg_work_size(int32_t nmajor, int32_t r, size_t *bytes)
{
    if (!bytes) return FMM_ERR_NULL;
    if (nmajor < 0 || r < 1) return FMM_ERR_DIM;
    *bytes = (3 * (size_t)nmajor * r + (size_t)nmajor) * sizeof(float);
    return FMM_OK;
}

fmm_status fmm_cg_lines(const fmm_sparse *S, const void *F, int32_t r, int32_t dtype, const float *rhs, float lambda,
                        int32_t iters, float *X, float *work, size_t work_bytes, void *ws, size_t ws_bytes,
                        hipStream_t stream)
{
    if (!S) return FMM_ERR_NULL;
    if (S->orient != FMM_CSR && S->orient != FMM_CSC) return FMM_ERR_ORIENT;
    const int32_t n = S->orient == FMM_CSR ? S->rows : S->cols;
    const int32_t minor = S->orient == FMM_CSR ? S->cols : S->rows;
    if (n < 0 || minor < 0 || r < 1 || iters < 0 || !(lambda >= 0.f)) return FMM_ERR_DIM;
    if (dtype != FMM_F32 && dtype != FMM_BF16) return FMM_ERR_DTYPE;
    if (n > 0 && (!rhs || !X || !work)) return FMM_ERR_NULL;
    if (minor > 0 && !F) return FMM_ERR_NULL;
    size_t need = 0;
    fmm_cg_work_size(n, r, &need);
    if (work_bytes < need) return FMM_ERR_WORKSPACE;
    const int vw = r % 4 == 0 ? 4 : 1;
    if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
    if (vw == 4 && ((uintptr_t)rhs % 16 || (uintptr_t)X % 16 || (uintptr_t)work % 16)) return FMM_ERR_UNSUPPORTED;
    float *R = work, *P = work + (size_t)n * r, *Q = work + 2 * (size_t)n * r, *rr = work + 3 * (size_t)n * r;
    const Shape sh = default_shape(r, vw);
    fmm_status s = gram_apply(S, X, F, r, dtype, Q, ws, ws_bytes, stream);
    if (s != FMM_OK) return s;
    hipError_t e = vw == 4 ? dispatch_cg<4>(sh, true, n, r, rhs, Q, X, lambda, R, P, rr, stream)
                           : dispatch_cg<1>(sh, true, n, r, rhs, Q, X, lambda, R, P, rr, stream);
    if (e != hipSuccess) return hipfail(e);
    for (int32_t it = 0; it < iters; ++it) {
        if (S->n_chunks == 0) {  // the step fused into the Gram pass: q never reaches memory
            s = gram_cg_step(S, P, F, r, dtype, lambda, X, R, rr, stream);
            if (s != FMM_OK) return s;
            continue;
        }
        s = gram_apply(S, P, F, r, dtype, Q, ws, ws_bytes, stream);
        if (s != FMM_OK) return s;
        e = vw == 4 ? dispatch_cg<4>(sh, false, n, r, rhs, Q, X, lambda, R, P, rr, stream)
                    : dispatch_cg<1>(sh, false, n, r, rhs, Q, X, lambda, R, P, rr, stream);
        if (e != hipSuccess) return hipfail(e);
    }
    return FMM_OK;
}

fmm_status fmm_residual_workspace(const fmm_sparse *S, size_t *bytes)
{
    if (!S || !bytes) return FMM_ERR_NULL;
    if (S->nnz < 0) return FMM_ERR_DIM;
    *bytes = ((size_t)S->nnz * sizeof(float) + 255) / 256 * 256 + kResidualBlocks * sizeof(double);
    return FMM_OK;
}

fmm_status fmm_sddmm_residual(const fmm_sparse *S_csr, const void *A, const void *B, int32_t r, int32_t dtype,
                              double *out, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!S_csr || !out) return FMM_ERR_NULL;
    if (S_csr->orient != FMM_CSR) return FMM_ERR_ORIENT;
    if (dtype != FMM_F32 && dtype != FMM_BF16) return FMM_ERR_DTYPE;
    size_t need = 0;
    fmm_residual_workspace(S_csr, &need);
    if (!ws || ws_bytes < need || (uintptr_t)ws % 16) return FMM_ERR_WORKSPACE;
    float *R = static_cast<float *>(ws);
    double *part = reinterpret_cast<double *>(static_cast<char *>(ws) + ((size_t)S_csr->nnz * sizeof(float) + 255) /
                                                                             256 * 256);
    fmm_sparse pat = *S_csr;  // the model's prediction uses the pattern alone
    pat.val = nullptr;
    fmm_status s = fmm_sddmm(&pat, A, B, r, dtype, R, 0.0, nullptr, 0, stream);
    if (s != FMM_OK) return s;
    hipLaunchKernelGGL(residual_partial_kernel, dim3(kResidualBlocks), dim3(256), 0, stream, (int64_t)S_csr->nnz,
                       static_cast<const float *>(S_csr->val), (const float *)R, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hipfail(e);
    hipLaunchKernelGGL(residual_final_kernel, dim3(1), dim3(256), 0, stream, kResidualBlocks, (const double *)part,
                       out);
    e = hipGetLastError();
    return e == hipSuccess ? FMM_OK : hipfail(e);
}

}  // extern "C"
