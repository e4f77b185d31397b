// Graph attention on the FusedMM access pattern (Section VI-E of the paper): the
// sampled product is replaced by the attention score a^T (H_i || H_j) = s_i + t_j,
// passed through LeakyReLU, optionally normalised by a softmax over each row's stored
// entries, and the result weights an SpMM with H:
//
//   out_i = sum_j w_ij H_j,   e_ij = LeakyReLU(S_ij (s_i + t_j)),
//   w_ij = e_ij, or w_ij = exp(e_ij - max_k e_ik) / sum_k exp(e_ik - max_k e_ik).
//
// The fused kernel keeps the softmax state of a row (running maximum m, normaliser l
// and the weighted sum) in registers and rescales it when the maximum grows, so a row
// is read once and no edge value is written to memory.  Long rows are split into
// chunks whose (sum, m, l) triples are combined afterwards in chunk order.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <type_traits>

#include "fmm.h"
#include "fmm_internal.hpp"

namespace fmm {
namespace {

template <class Acc> __device__ __forceinline__ Acc exp_acc(Acc x);
template <> __device__ __forceinline__ float exp_acc<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double exp_acc<double>(double x) { return exp(x); }
template <class Acc> __device__ __forceinline__ Acc log_acc(Acc x);
template <> __device__ __forceinline__ float log_acc<float>(float x) { return logf(x); }
template <> __device__ __forceinline__ double log_acc<double>(double x) { return log(x); }
template <class Acc> __device__ __forceinline__ Acc neg_inf();
template <> __device__ __forceinline__ float neg_inf<float>() { return -__builtin_huge_valf(); }
template <> __device__ __forceinline__ double neg_inf<double>() { return -__builtin_huge_val(); }

// s_i = a1 . H_i and t_i = a2 . H_i for every row: one lane group per row.
template <class TH, class Acc, int L, int NV, int VW>
__global__ __launch_bounds__(kBlock) void gat_scores_kernel(const TH *__restrict__ H, int32_t n, int32_t r,
                                                            const Acc *__restrict__ a1, const Acc *__restrict__ a2,
                                                            Acc *__restrict__ s, Acc *__restrict__ t)
{
    constexpr int GPB = kBlock / L;
    const int lane = threadIdx.x % L;
    const int64_t row = (int64_t)blockIdx.x * GPB + threadIdx.x / L;
    if (row >= n) return;
    const int C = r / VW;
    Acc x = Acc(0), y = Acc(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int c = v * L + lane;
        if (c < C) {
            Raw<TH, VW> h;
            h.load(H + row * r + c * VW);
#pragma unroll
            for (int e = 0; e < VW; ++e) {
                x += a1[c * VW + e] * Acc(h.get(e));
                y += a2[c * VW + e] * Acc(h.get(e));
            }
        }
    }
    x = group_sum<L>(x);
    y = group_sum<L>(y);
    if (lane == 0) {
        s[row] = x;
        t[row] = y;
    }
}

// Edge values of every stored entry, in CSR order (the unfused form: written to memory
// for a separate SpMM).  A group of L lanes owns a row; lanes take the row's entries in
// turn.  Softmax: the row maximum and the sum of exponentials are reduced over the group
// (a fixed tree), then every value is rescaled.
template <class Acc, int L>
__global__ __launch_bounds__(kBlock) void gat_edges_kernel(int32_t n, const int32_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ idx, const Acc *__restrict__ val,
                                                           const Acc *__restrict__ s, const Acc *__restrict__ t,
                                                           Acc slope, bool softmax, Acc *__restrict__ w)
{
    const int lane = threadIdx.x % L;
    const int64_t row = (int64_t)blockIdx.x * (kBlock / L) + threadIdx.x / L;
    if (row >= n) return;
    const int32_t b = ptr[row], e = ptr[row + 1];
    const Acc si = s[row];
    Acc mx = neg_inf<Acc>();
    for (int32_t p = b + lane; p < e; p += L) {
        const Acc x = (val ? val[p] : Acc(1)) * (si + t[idx[p]]);
        const Acc v = x >= Acc(0) ? x : slope * x;
        w[p] = v;
        mx = v > mx ? v : mx;
    }
    if (!softmax) return;
    // group maximum: max is exact, so any reduction order gives the same bits
#pragma unroll
    for (int o = 1; o < L; o <<= 1) {
        const Acc y = __shfl_xor(mx, o, L);
        mx = y > mx ? y : mx;
    }
    Acc sum = Acc(0);
    for (int32_t p = b + lane; p < e; p += L) {
        const Acc v = exp_acc<Acc>(w[p] - mx);
        w[p] = v;
        sum += v;
    }
    sum = group_sum<L>(sum);
    const Acc inv = sum > Acc(0) ? Acc(1) / sum : Acc(0);
    for (int32_t p = b + lane; p < e; p += L) w[p] *= inv;
}

struct GatArgs {
    int32_t nlines, r;
    const int32_t *ptr, *idx;
    const void *val;  // S values (Acc) or NULL for a 0/1 adjacency
    const void *s, *t;
    const void *H;
    void *out;
    double slope;
    int32_t long_len, n_chunks;
    const int32_t *chunks;
    void *partial;  // n_chunks x r sums, then n_chunks x 2 (m, l)
    const int32_t *order;  // row processing order, NULL = index order
    void *lse;             // softmax: per-row log-sum-exp of the edge values (Acc), or NULL
};

template <class TH, class Acc, int L, int NV, int VW, int U, bool SOFTMAX>
__global__ __launch_bounds__(kBlock) void gat_kernel(GatArgs a, int32_t nb_chunk_blocks)
{
    constexpr int GPB = kBlock / L;
    constexpr int E = NV * VW;
    const int lane = threadIdx.x % L;
    const int gib = threadIdx.x / L;
    const int r = a.r;
    int32_t line, begin, end, chunk = -1;
    if ((int32_t)blockIdx.x < nb_chunk_blocks) {
        chunk = blockIdx.x * GPB + gib;
        if (chunk >= a.n_chunks) return;
        line = a.chunks[3 * chunk];
        begin = a.chunks[3 * chunk + 1];
        end = a.chunks[3 * chunk + 2];
    } else {
        const int32_t k = (blockIdx.x - nb_chunk_blocks) * GPB + gib;
        if (k >= a.nlines) return;
        line = a.order ? a.order[k] : k;
        begin = a.ptr[line];
        end = a.ptr[line + 1];
        if (a.n_chunks > 0 && end - begin > a.long_len) return;
    }
    const int C = r / VW;
    bool act[NV];
    int off[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        act[v] = v * L + lane < C;
        off[v] = act[v] ? (v * L + lane) * VW : 0;
    }
    const int32_t *__restrict__ idx = a.idx;
    const Acc *__restrict__ val = static_cast<const Acc *>(a.val);
    const Acc *__restrict__ tv = static_cast<const Acc *>(a.t);
    const TH *__restrict__ H = static_cast<const TH *>(a.H);
    const Acc si = static_cast<const Acc *>(a.s)[line];
    const Acc slope = Acc(a.slope);

    Acc acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = Acc(0);
    Acc m = neg_inf<Acc>(), l = Acc(0);

    // Column indices and edge values of the batch at p0; entries past `end` reread the
    // last entry, so every load is in bounds.
    auto load_meta = [&](int32_t p0, int32_t *j, Acc *sc) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t p = p0 + u;
            const int32_t pc = p < end ? p : end - 1;
            j[u] = idx[pc];
            sc[u] = val ? val[pc] : Acc(1);
        }
    };
    int32_t j[U], jn[U];
    Acc sc[U], scn[U];
    if (begin < end) load_meta(begin, j, sc);
    for (int32_t p0 = begin; p0 < end; p0 += U) {
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ok[u] = p0 + u < end;
        Raw<TH, VW> g[U][NV];
        Acc tj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            tj[u] = tv[j[u]];
            if (ok[u]) {
#pragma unroll
                for (int v = 0; v < NV; ++v) g[u][v].load(H + (size_t)j[u] * r + off[v]);
            }
        }
        // the next batch's operands arrive while this batch waits for its rows
        if (p0 + U < end) load_meta(p0 + U, jn, scn);
        // LeakyReLU of the sampled score; entries past the end get weight 0 (softmax: -inf)
        Acc ev[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const Acc x = sc[u] * (si + tj[u]);
            ev[u] = x >= Acc(0) ? x : slope * x;
        }
        Acc w[U];
        if constexpr (SOFTMAX) {
            Acc mb = m;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) mb = ev[u] > mb ? ev[u] : mb;
            const Acc scale = exp_acc<Acc>(m - mb);  // m == -inf on the first batch: 0
            l *= scale;
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] *= scale;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                w[u] = ok[u] ? exp_acc<Acc>(ev[u] - mb) : Acc(0);
                l += w[u];
            }
            m = mb;
        } else {
#pragma unroll
            for (int u = 0; u < U; ++u) w[u] = ok[u] ? ev[u] : Acc(0);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
#pragma unroll
            for (int v = 0; v < NV; ++v)
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[v * VW + e] += w[u] * Acc(g[u][v].get(e));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            j[u] = jn[u];
            sc[u] = scn[u];
        }
    }

    Acc *dst;
    Acc inv = Acc(1);
    if (chunk >= 0) {
        dst = static_cast<Acc *>(a.partial) + (size_t)chunk * r;
        if (lane == 0) {
            Acc *ml = static_cast<Acc *>(a.partial) + (size_t)a.n_chunks * r + 2 * (size_t)chunk;
            ml[0] = m;
            ml[1] = l;
        }
    } else {
        dst = static_cast<Acc *>(a.out) + (size_t)line * r;
        if (SOFTMAX) inv = l > Acc(0) ? Acc(1) / l : Acc(0);
        if (SOFTMAX && a.lse && lane == 0)
            static_cast<Acc *>(a.lse)[line] = l > Acc(0) ? m + log_acc<Acc>(l) : Acc(0);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (!act[v]) continue;
        Acc o[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) o[e] = acc[v * VW + e] * inv;
        St<Acc, VW>::run(dst + off[v], o);
    }
}

// Combine the chunks of each split row, in chunk order: with M the largest chunk maximum,
// sum_c acc_c exp(m_c - M) / sum_c l_c exp(m_c - M) (softmax), or sum_c acc_c.
template <class Acc, bool SOFTMAX>
__global__ __launch_bounds__(kBlock) void gat_merge_kernel(const int32_t *__restrict__ splits, int32_t n_splits,
                                                           int32_t r, int32_t n_chunks,
                                                           const Acc *__restrict__ partial, Acc *__restrict__ out,
                                                           Acc *__restrict__ lse)
{
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (tid >= (int64_t)n_splits * r) return;
    const int32_t sidx = (int32_t)(tid / r), k = (int32_t)(tid % r);
    const int32_t line = splits[3 * sidx], first = splits[3 * sidx + 1], cnt = splits[3 * sidx + 2];
    const Acc *ml = partial + (size_t)n_chunks * r;
    Acc sum = Acc(0);
    if (SOFTMAX) {
        Acc M = neg_inf<Acc>();
        for (int32_t c = 0; c < cnt; ++c) M = ml[2 * (first + c)] > M ? ml[2 * (first + c)] : M;
        Acc L = Acc(0);
        for (int32_t c = 0; c < cnt; ++c) {
            const Acc f = exp_acc<Acc>(ml[2 * (first + c)] - M);
            L += ml[2 * (first + c) + 1] * f;
            sum += partial[(size_t)(first + c) * r + k] * f;
        }
        sum = L > Acc(0) ? sum * (Acc(1) / L) : Acc(0);
        if (lse && k == 0) lse[line] = L > Acc(0) ? M + log_acc<Acc>(L) : Acc(0);
    } else {
        for (int32_t c = 0; c < cnt; ++c) sum += partial[(size_t)(first + c) * r + k];
    }
    out[(size_t)line * r + k] = sum;
}

template <class TH, class Acc, int L, int NV, int VW, int U>
hipError_t launch_gat_shape(const GatArgs &a, bool softmax, hipStream_t st)
{
    constexpr int GPB = kBlock / L;
    const int64_t nbc = a.n_chunks > 0 ? ((int64_t)a.n_chunks + GPB - 1) / GPB : 0;
    const int64_t nbl = ((int64_t)a.nlines + GPB - 1) / GPB;
    if (nbc + nbl == 0) return hipSuccess;
    if (softmax)
        hipLaunchKernelGGL((gat_kernel<TH, Acc, L, NV, VW, U, true>), dim3((unsigned)(nbc + nbl)), dim3(kBlock), 0,
                           st, a, (int32_t)nbc);
    else
        hipLaunchKernelGGL((gat_kernel<TH, Acc, L, NV, VW, U, false>), dim3((unsigned)(nbc + nbl)), dim3(kBlock), 0,
                           st, a, (int32_t)nbc);
    return hipGetLastError();
}

template <class TH, class Acc, int L, int NV, int VW>
hipError_t launch_scores_shape(const TH *H, int32_t n, int32_t r, const Acc *a1, const Acc *a2, Acc *s, Acc *t,
                               hipStream_t st)
{
    constexpr int GPB = kBlock / L;
    const int64_t nb = ((int64_t)n + GPB - 1) / GPB;
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((gat_scores_kernel<TH, Acc, L, NV, VW>), dim3((unsigned)nb), dim3(kBlock), 0, st, H, n, r, a1,
                       a2, s, t);
    return hipGetLastError();
}

#define GAT_SHAPES(X)                                                                            \
    X(1, 1) X(2, 1) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(64, 2) X(64, 4)

template <class TH, class Acc, int VW>
hipError_t dispatch_gat(const GatArgs &a, Shape sh, bool softmax, int uclass, hipStream_t st)
{
#define GAT_CASE(Lv, NVv)                                                                        \
    if (sh.L == Lv && sh.NV == NVv) {                                                            \
        if (uclass == 1) return launch_gat_shape<TH, Acc, Lv, NVv, VW, (8 / NVv > 0 ? 8 / NVv : 1)>(a, softmax, st); \
        return launch_gat_shape<TH, Acc, Lv, NVv, VW, (4 / NVv > 0 ? 4 / NVv : 1)>(a, softmax, st);                   \
    }
    GAT_SHAPES(GAT_CASE)
#undef GAT_CASE
    return hipErrorInvalidValue;
}

template <class TH, class Acc, int VW>
hipError_t dispatch_scores(const TH *H, int32_t n, int32_t r, const Acc *a1, const Acc *a2, Acc *s, Acc *t, Shape sh,
                           hipStream_t st)
{
#define SC_CASE(Lv, NVv)                                                                         \
    if (sh.L == Lv && sh.NV == NVv) return launch_scores_shape<TH, Acc, Lv, NVv, VW>(H, n, r, a1, a2, s, t, st);
    GAT_SHAPES(SC_CASE)
#undef SC_CASE
    return hipErrorInvalidValue;
}

// Shapes for the attention kernels: the default line shape, with NV = 2 rounded up to 4
// only where L = 64 (the compiled set above).
Shape gat_shape(int r, int vw)
{
    Shape s = default_shape(r, vw);
    if (s.NV == 2 && s.L != 64) s = Shape{64, 1};
    return s;
}

fmm_status hipfail(hipError_t e)
{
    set_last_hip_error((int32_t)e);
    return FMM_ERR_HIP;
}

int gat_uclass(const fmm_sparse *S)
{
    if (S->variant == FMM_VARIANT_DEEP) return 1;
    if (S->variant >= FMM_VARIANT_MEDIUM) return 2;
    const double mean = S->rows > 0 ? (double)S->nnz / S->rows : 0.0;
    return mean >= 24.0 ? 1 : 2;
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" {

fmm_status fmm_gat_scores(const void *H, int32_t n, int32_t r, int32_t dtype, const void *a1, const void *a2, void *s,
                          void *t, hipStream_t stream)
{
    if (n < 0 || r < 1) return FMM_ERR_DIM;
    if (n > 0 && (!H || !s || !t)) return FMM_ERR_NULL;
    if (!a1 || !a2) return FMM_ERR_NULL;
    hipError_t e;
    if (dtype == FMM_F32) {
        const int vw = r % 4 == 0 ? 4 : 1;
        if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
        if (vw == 4 && (uintptr_t)H % 16) return FMM_ERR_UNSUPPORTED;
        const Shape sh = gat_shape(r, vw);
        e = vw == 4 ? dispatch_scores<float, float, 4>((const float *)H, n, r, (const float *)a1, (const float *)a2,
                                                       (float *)s, (float *)t, sh, stream)
                    : dispatch_scores<float, float, 1>((const float *)H, n, r, (const float *)a1, (const float *)a2,
                                                       (float *)s, (float *)t, sh, stream);
    } else if (dtype == FMM_BF16) {
        if (r % 8 != 0 || r > 1024) return FMM_ERR_DTYPE;
        if ((uintptr_t)H % 16) return FMM_ERR_UNSUPPORTED;
        e = dispatch_scores<bf16_t, float, 8>((const bf16_t *)H, n, r, (const float *)a1, (const float *)a2,
                                              (float *)s, (float *)t, gat_shape(r, 8), stream);
    } else if (dtype == FMM_F64) {
        const int vw = r % 2 == 0 ? 2 : 1;
        if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
        if (vw == 2 && (uintptr_t)H % 16) return FMM_ERR_UNSUPPORTED;
        const Shape sh = gat_shape(r, vw);
        e = vw == 2 ? dispatch_scores<double, double, 2>((const double *)H, n, r, (const double *)a1,
                                                         (const double *)a2, (double *)s, (double *)t, sh, stream)
                    : dispatch_scores<double, double, 1>((const double *)H, n, r, (const double *)a1,
                                                         (const double *)a2, (double *)s, (double *)t, sh, stream);
    } else {
        return FMM_ERR_DTYPE;
    }
    return e == hipSuccess ? FMM_OK : hipfail(e);
}

fmm_status fmm_gat_forward(const fmm_sparse *S, const void *s, const void *t, const void *H, int32_t r, int32_t dtype,
                           double negative_slope, int32_t flags, void *out, void *lse, void *ws, size_t ws_bytes,
                           hipStream_t stream)
{
    if (!S) return FMM_ERR_NULL;
    if (S->orient != FMM_CSR) return FMM_ERR_ORIENT;
    if (S->rows < 0 || S->rows != S->cols || S->nnz < 0 || r < 1) return FMM_ERR_DIM;
    if (!S->ptr || (S->nnz > 0 && !S->idx)) return FMM_ERR_NULL;
    if (S->rows > 0 && (!s || !t || !H || !out)) return FMM_ERR_NULL;
    if (flags & ~FMM_GAT_SOFTMAX) return FMM_ERR_DIM;
    if (S->n_chunks < 0 || S->n_splits < 0) return FMM_ERR_DIM;
    if (S->n_chunks > 0 && (!S->chunks || !S->splits || S->long_len < 1)) return FMM_ERR_NULL;
    const size_t ob = dtype == FMM_F64 ? 8 : 4;
    const size_t need = S->n_chunks > 0 ? (size_t)S->n_chunks * ((size_t)r + 2) * ob : 0;
    if (need && (!ws || ws_bytes < need || (uintptr_t)ws % 16)) return FMM_ERR_WORKSPACE;
    GatArgs a;
    memset(&a, 0, sizeof(a));
    a.nlines = S->rows;
    a.r = r;
    a.ptr = S->ptr;
    a.idx = S->idx;
    a.val = S->val;
    a.s = s;
    a.t = t;
    a.H = H;
    a.out = out;
    a.slope = negative_slope;
    a.long_len = S->long_len;
    a.n_chunks = S->n_chunks;
    a.chunks = S->chunks;
    a.order = S->order;
    a.partial = ws;
    a.lse = lse;
    const bool softmax = (flags & FMM_GAT_SOFTMAX) != 0;
    const int uc = gat_uclass(S);
    hipError_t e;
    if (dtype == FMM_F32) {
        const int vw = r % 4 == 0 ? 4 : 1;
        if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
        if (vw == 4 && ((uintptr_t)H % 16 || (uintptr_t)out % 16)) return FMM_ERR_UNSUPPORTED;
        e = vw == 4 ? dispatch_gat<float, float, 4>(a, gat_shape(r, 4), softmax, uc, stream)
                    : dispatch_gat<float, float, 1>(a, gat_shape(r, 1), softmax, uc, stream);
    } else if (dtype == FMM_BF16) {
        if (r % 8 != 0 || r > 1024) return FMM_ERR_DTYPE;
        if ((uintptr_t)H % 16 || (uintptr_t)out % 16) return FMM_ERR_UNSUPPORTED;
        e = dispatch_gat<bf16_t, float, 8>(a, gat_shape(r, 8), softmax, uc, stream);
    } else if (dtype == FMM_F64) {
        const int vw = r % 2 == 0 ? 2 : 1;
        if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
        if (vw == 2 && ((uintptr_t)H % 16 || (uintptr_t)out % 16)) return FMM_ERR_UNSUPPORTED;
        e = vw == 2 ? dispatch_gat<double, double, 2>(a, gat_shape(r, 2), softmax, uc, stream)
                    : dispatch_gat<double, double, 1>(a, gat_shape(r, 1), softmax, uc, stream);
    } else {
        return FMM_ERR_DTYPE;
    }
    if (e != hipSuccess) return hipfail(e);
    if (S->n_chunks > 0 && S->n_splits > 0) {
        const int64_t total = (int64_t)S->n_splits * r;
        const unsigned nb = (unsigned)((total + kBlock - 1) / kBlock);
        if (dtype == FMM_F64) {
            if (softmax)
                hipLaunchKernelGGL((gat_merge_kernel<double, true>), dim3(nb), dim3(kBlock), 0, stream, S->splits,
                                   S->n_splits, r, S->n_chunks, (const double *)ws, (double *)out, (double *)lse);
            else
                hipLaunchKernelGGL((gat_merge_kernel<double, false>), dim3(nb), dim3(kBlock), 0, stream, S->splits,
                                   S->n_splits, r, S->n_chunks, (const double *)ws, (double *)out, (double *)lse);
        } else {
            if (softmax)
                hipLaunchKernelGGL((gat_merge_kernel<float, true>), dim3(nb), dim3(kBlock), 0, stream, S->splits,
                                   S->n_splits, r, S->n_chunks, (const float *)ws, (float *)out, (float *)lse);
            else
                hipLaunchKernelGGL((gat_merge_kernel<float, false>), dim3(nb), dim3(kBlock), 0, stream, S->splits,
                                   S->n_splits, r, S->n_chunks, (const float *)ws, (float *)out, (float *)lse);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return hipfail(e);
    }
    return FMM_OK;
}

fmm_status fmm_gat_workspace(const fmm_sparse *S, int32_t r, int32_t dtype, size_t *bytes)
{
    if (!S || !bytes) return FMM_ERR_NULL;
    if (r < 1) return FMM_ERR_DIM;
    if (dtype != FMM_F32 && dtype != FMM_BF16 && dtype != FMM_F64) return FMM_ERR_DTYPE;
    const size_t ob = dtype == FMM_F64 ? 8 : 4;
    *bytes = S->n_chunks > 0 ? (size_t)S->n_chunks * ((size_t)r + 2) * ob : 0;
    return FMM_OK;
}

fmm_status fmm_gat_edge_values(const fmm_sparse *S, const void *s, const void *t, int32_t dtype, double negative_slope,
                               int32_t flags, void *w, hipStream_t stream)
{
    if (!S) return FMM_ERR_NULL;
    if (S->orient != FMM_CSR) return FMM_ERR_ORIENT;
    if (S->rows < 0 || S->rows != S->cols || S->nnz < 0) return FMM_ERR_DIM;
    if (!S->ptr || (S->nnz > 0 && (!S->idx || !w))) return FMM_ERR_NULL;
    if (S->rows > 0 && (!s || !t)) return FMM_ERR_NULL;
    if (flags & ~FMM_GAT_SOFTMAX) return FMM_ERR_DIM;
    const bool softmax = (flags & FMM_GAT_SOFTMAX) != 0;
    constexpr int L = 16;
    const unsigned nb = (unsigned)(((int64_t)S->rows + kBlock / L - 1) / (kBlock / L));
    if (nb == 0) return FMM_OK;
    if (dtype == FMM_F64)
        hipLaunchKernelGGL((gat_edges_kernel<double, L>), dim3(nb), dim3(kBlock), 0, stream, S->rows, S->ptr, S->idx,
                           (const double *)S->val, (const double *)s, (const double *)t, negative_slope, softmax,
                           (double *)w);
    else if (dtype == FMM_F32 || dtype == FMM_BF16)
        hipLaunchKernelGGL((gat_edges_kernel<float, L>), dim3(nb), dim3(kBlock), 0, stream, S->rows, S->ptr, S->idx,
                           (const float *)S->val, (const float *)s, (const float *)t, (float)negative_slope, softmax,
                           (float *)w);
    else
        return FMM_ERR_DTYPE;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? FMM_OK : hipfail(e);
}

}  // extern "C"
