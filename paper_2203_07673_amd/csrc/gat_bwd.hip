// Adjoint of the graph-attention head (the forward is Section VI-E; its gradient follows
// from the definition by the chain rule).  With upstream gradient dO and the forward's
// scores s, t and output out:
//
//   x_ij = S_ij (s_i + t_j),  e = LeakyReLU(x),  w = e or exp(e_ij - lse_i) (row softmax)
//   dw_ij = <dO_i, H_j>
//   de_ij = dw_ij, or w_ij (dw_ij - D_i) with D_i = sum_j w_ij dw_ij = <dO_i, out_i>
//   dx_ij = de_ij (1 if x_ij > 0 else slope)
//   dS_ij = dx_ij (s_i + t_j),  ds_i = sum_j dx_ij S_ij,  dt_j = sum_i dx_ij S_ij
//   dH_j  = sum_i w_ij dO_i + ds_j a1 + dt_j a2,  da1 = H^T ds,  da2 = H^T dt
//
// Passes: (1) a row pass on S_csr (held dO_i and out_i, gathered H_j) for D_i, ds and dS;
// (2) a column pass on the stored transpose (held H_j, gathered dO_i and per-row scalars)
// for dt and dH_j = sum_i w_ij dO_i + ds_j a1 + dt_j a2, both recomputing the edge weight
// (from the forward's per-row log-sum-exp) and dw in registers like the fused adjoints;
// (3) chunk merges in chunk order for split lines, then their rank-one terms; (4) per-block
// partial sums of da1, da2 and (5) their sum in block order.  No atomics anywhere.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <initializer_list>

#include "fmm.h"
#include "fmm_internal.hpp"

namespace fmm {
namespace {

template <class Acc> __device__ __forceinline__ Acc bexp(Acc x);
template <> __device__ __forceinline__ float bexp<float>(float x) { return expf(x); }
template <> __device__ __forceinline__ double bexp<double>(double x) { return exp(x); }
template <class Acc> __device__ __forceinline__ Acc blog(Acc x);
template <> __device__ __forceinline__ float blog<float>(float x) { return logf(x); }
template <> __device__ __forceinline__ double blog<double>(double x) { return log(x); }
template <class Acc> __device__ __forceinline__ Acc bneg_inf();
template <> __device__ __forceinline__ float bneg_inf<float>() { return -__builtin_huge_valf(); }
template <> __device__ __forceinline__ double bneg_inf<double>() { return -__builtin_huge_val(); }

constexpr int kFinishRows = 512;  // rows per block of the rank-one / da pass

// One stored element widened to the accumulation type (bfloat16: the high half of a float).
template <class Acc> __device__ __forceinline__ Acc widen(float x) { return Acc(x); }
template <class Acc> __device__ __forceinline__ Acc widen(double x) { return Acc(x); }
template <class Acc> __device__ __forceinline__ Acc widen(bf16_t x) { return Acc(__uint_as_float((uint32_t)x << 16)); }

// The three per-row scalars the column pass gathers for every entry, packed so that one
// 16-byte (float) or 32-byte (double) load fetches them: s_i, lse_i, D_i.
template <class Acc> struct RowScalars;
template <> struct RowScalars<float> {
    float4 v;
    __device__ __forceinline__ void load(const void *base, int32_t i) { v = static_cast<const float4 *>(base)[i]; }
    static __device__ __forceinline__ void store(void *base, int32_t i, float s, float l, float d) {
        static_cast<float4 *>(base)[i] = make_float4(s, l, d, 0.f);
    }
    __device__ __forceinline__ float s() const { return v.x; }
    __device__ __forceinline__ float lse() const { return v.y; }
    __device__ __forceinline__ float D() const { return v.z; }
};
template <> struct RowScalars<double> {
    double2 a, b;
    __device__ __forceinline__ void load(const void *base, int32_t i) {
        a = static_cast<const double2 *>(base)[2 * i];
        b = static_cast<const double2 *>(base)[2 * i + 1];
    }
    static __device__ __forceinline__ void store(void *base, int32_t i, double s, double l, double d) {
        static_cast<double2 *>(base)[2 * i] = make_double2(s, l);
        static_cast<double2 *>(base)[2 * i + 1] = make_double2(d, 0.0);
    }
    __device__ __forceinline__ double s() const { return a.x; }
    __device__ __forceinline__ double lse() const { return a.y; }
    __device__ __forceinline__ double D() const { return b.x; }
};

struct GatBwdArgs {
    int32_t nlines, r;
    const int32_t *ptr, *idx;
    const void *val;          // S's values in this orientation (Acc), NULL = 1
    const void *s, *t;        // scores (Acc, per node)
    const void *lse;          // per row log-sum-exp from the forward (softmax; Acc)
    void *rs;                 // packed per-row (s_i, lse_i, D_i): written by the row pass, gathered by the column pass
    const void *out;          // forward output (row pass)
    const void *a1, *a2;      // attention vectors (column pass)
    const void *ds;           // ds from the row pass (column pass)
    const void *held;         // held matrix: dO (row pass, Acc) or H (column pass, TH)
    const void *gath;         // gathered matrix: H (row pass, TH) or dO (column pass, Acc)
    double slope;
    int32_t softmax;
    int32_t long_len, n_chunks;
    const int32_t *chunks;
    const int32_t *order;
    void *out_vec;            // column pass: sum_i w_ij dO_i per column (Acc, lines x r)
    void *out_sc;             // per-line scalar: ds (row pass) or dt (column pass)
    void *part_vec, *part_sc; // chunk partials
    void *dS;                 // row pass: dL/dS in CSR order (Acc), or NULL
};

// Line (or chunk) of this lane group, as in the forward kernels.  Returns false when the
// group has no work.
__device__ __forceinline__ bool pick_line(const GatBwdArgs &a, int32_t nb_chunk_blocks, int gpb, int gib,
                                          int32_t &line, int32_t &begin, int32_t &end, int32_t &chunk)
{
    chunk = -1;
    if ((int32_t)blockIdx.x < nb_chunk_blocks) {
        chunk = blockIdx.x * gpb + gib;
        if (chunk >= a.n_chunks) return false;
        line = a.chunks[3 * chunk];
        begin = a.chunks[3 * chunk + 1];
        end = a.chunks[3 * chunk + 2];
        return true;
    }
    const int32_t k = (blockIdx.x - nb_chunk_blocks) * gpb + gib;
    if (k >= a.nlines) return false;
    line = a.order ? a.order[k] : k;
    begin = a.ptr[line];
    end = a.ptr[line + 1];
    return !(a.n_chunks > 0 && end - begin > a.long_len);
}

// Indices and stored values of the batch at p0 (entries past `end` reread the last one).
template <class Acc, int U>
__device__ __forceinline__ void load_entries(const int32_t *__restrict__ idx, const Acc *__restrict__ val, int32_t p0,
                                             int32_t end, int32_t *j, Acc *v)
{
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int32_t pc = p0 + u < end ? p0 + u : end - 1;
        j[u] = idx[pc];
        v[u] = val ? val[pc] : Acc(1);
    }
}

// Per-entry backward scalars from the recomputed forward values.
template <class Acc>
__device__ __forceinline__ void entry_grad(Acc v, Acc score, Acc lse_i, Acc D_i, Acc dw, Acc slope, bool softmax,
                                           Acc &w, Acc &dx)
{
    const Acc x = v * score;
    const Acc e = x >= Acc(0) ? x : slope * x;
    w = softmax ? bexp<Acc>(e - lse_i) : e;
    const Acc de = softmax ? w * (dw - D_i) : dw;
    dx = de * (x > Acc(0) ? Acc(1) : slope);
}

// (2) Row pass on S_csr: held dO_i (stored as TO), gathered H_j.  ds_i = sum_j dx_ij S_ij; dS_ij.
template <class TH, class TO, class Acc, int L, int NV, int VW, int U>
__global__ __launch_bounds__(kBlock) void gat_bwd_rows_kernel(GatBwdArgs a, int32_t nb_chunk_blocks)
{
    constexpr int GPB = kBlock / L;
    constexpr int E = NV * VW;
    const int lane = threadIdx.x % L;
    int32_t line, begin, end, chunk;
    if (!pick_line(a, nb_chunk_blocks, GPB, threadIdx.x / L, line, begin, end, chunk)) return;
    const int r = a.r, C = r / VW;
    const TO *dO = static_cast<const TO *>(a.held);
    const TH *H = static_cast<const TH *>(a.gath);
    const Acc *val = static_cast<const Acc *>(a.val);
    const Acc *t = static_cast<const Acc *>(a.t);
    const Acc *out = static_cast<const Acc *>(a.out);
    const Acc si = static_cast<const Acc *>(a.s)[line];
    const bool softmax = a.softmax != 0;
    const Acc lse_i = softmax ? static_cast<const Acc *>(a.lse)[line] : Acc(0);
    const Acc slope = Acc(a.slope);
    Acc *dS = static_cast<Acc *>(a.dS);
    bool act[NV];
    int off[NV];
    Acc hd[E];
    Acc dd = Acc(0);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        act[v] = v * L + lane < C;
        off[v] = act[v] ? (v * L + lane) * VW : 0;
        Raw<TO, VW> x;
        Raw<Acc, VW> y;
        if (act[v]) {
            x.load(dO + (size_t)line * r + off[v]);
            y.load(out + (size_t)line * r + off[v]);
        } else {
            x.zero();
            y.zero();
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            hd[v * VW + e] = Acc(x.get(e));
            dd += Acc(x.get(e)) * Acc(y.get(e));
        }
    }
    // D_i = <dO_i, out_i> (= sum_j w_ij dw_ij); every chunk of a split row writes the same bits
    const Acc D_i = group_sum<L>(dd);
    if (lane == 0) RowScalars<Acc>::store(a.rs, line, si, lse_i, D_i);
    Acc dsum = Acc(0);
    // indices and values of the next batch are loaded while this batch's rows arrive
    int32_t j[U], jn[U];
    Acc v[U], vn[U];
    if (begin < end) load_entries<Acc, U>(a.idx, val, begin, end, j, v);
    for (int32_t p0 = begin; p0 < end; p0 += U) {
        bool ok[U];
        Acc tj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ok[u] = p0 + u < end;
        Raw<TH, VW> g[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            tj[u] = t[j[u]];
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                if (ok[u] && act[q]) g[u][q].load(H + (size_t)j[u] * r + off[q]);
                else g[u][q].zero();
            }
        }
        if (p0 + U < end) load_entries<Acc, U>(a.idx, val, p0 + U, end, jn, vn);
        Acc dw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Acc x = Acc(0);
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int e = 0; e < VW; ++e) x += hd[q * VW + e] * Acc(g[u][q].get(e));
            dw[u] = group_sum<L>(x);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            const Acc score = si + tj[u];
            Acc w, dx;
            entry_grad<Acc>(v[u], score, lse_i, D_i, dw[u], slope, softmax, w, dx);
            dsum += dx * v[u];
            if (dS && lane == (u % L)) dS[p0 + u] = dx * score;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            j[u] = jn[u];
            v[u] = vn[u];
        }
    }
    if (lane == 0) {
        if (chunk >= 0) static_cast<Acc *>(a.part_sc)[chunk] = dsum;
        else static_cast<Acc *>(a.out_sc)[line] = dsum;
    }
}

// (3) Column pass on the stored transpose: held H_j, gathered dO_i (stored as TO) and the
// row scalars.  dt_j = sum_i dx_ij S_ij and sum_i w_ij dO_i.
template <class TH, class TO, class Acc, int L, int NV, int VW, int U>
__global__ __launch_bounds__(kBlock) void gat_bwd_cols_kernel(GatBwdArgs a, int32_t nb_chunk_blocks)
{
    constexpr int GPB = kBlock / L;
    constexpr int E = NV * VW;
    const int lane = threadIdx.x % L;
    int32_t line, begin, end, chunk;
    if (!pick_line(a, nb_chunk_blocks, GPB, threadIdx.x / L, line, begin, end, chunk)) return;
    const int r = a.r, C = r / VW;
    const TH *H = static_cast<const TH *>(a.held);
    const TO *dO = static_cast<const TO *>(a.gath);
    const Acc *val = static_cast<const Acc *>(a.val);
    const Acc tj = static_cast<const Acc *>(a.t)[line];
    const Acc slope = Acc(a.slope);
    const bool softmax = a.softmax != 0;
    bool act[NV];
    int off[NV];
    Acc hh[E], acc[E];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        act[v] = v * L + lane < C;
        off[v] = act[v] ? (v * L + lane) * VW : 0;
        Raw<TH, VW> x;
        if (act[v]) x.load(H + (size_t)line * r + off[v]);
        else x.zero();
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            hh[v * VW + e] = Acc(x.get(e));
            acc[v * VW + e] = Acc(0);
        }
    }
    Acc dtsum = Acc(0);
    int32_t i[U], in_[U];
    Acc v[U], vn[U];
    if (begin < end) load_entries<Acc, U>(a.idx, val, begin, end, i, v);
    for (int32_t p0 = begin; p0 < end; p0 += U) {
        bool ok[U];
        RowScalars<Acc> rsc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) ok[u] = p0 + u < end;
        Raw<TO, VW> g[U][NV];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            rsc[u].load(a.rs, i[u]);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
                if (ok[u] && act[q]) g[u][q].load(dO + (size_t)i[u] * r + off[q]);
                else g[u][q].zero();
            }
        }
        if (p0 + U < end) load_entries<Acc, U>(a.idx, val, p0 + U, end, in_, vn);
        Acc dw[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            Acc x = Acc(0);
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int e = 0; e < VW; ++e) x += hh[q * VW + e] * Acc(g[u][q].get(e));
            dw[u] = group_sum<L>(x);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!ok[u]) continue;
            Acc w, dx;
            entry_grad<Acc>(v[u], rsc[u].s() + tj, rsc[u].lse(), rsc[u].D(), dw[u], slope, softmax, w, dx);
            dtsum += dx * v[u];
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[q * VW + e] += w * Acc(g[u][q].get(e));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            i[u] = in_[u];
            v[u] = vn[u];
        }
    }
    Acc *dst;
    if (chunk >= 0) {
        dst = static_cast<Acc *>(a.part_vec) + (size_t)chunk * r;
    } else {  // a whole column: add the rank-one terms ds_j a1 + dt_j a2 here
        dst = static_cast<Acc *>(a.out_vec) + (size_t)line * r;
        const Acc dsj = static_cast<const Acc *>(a.ds)[line];
        const Acc *a1 = static_cast<const Acc *>(a.a1);
        const Acc *a2 = static_cast<const Acc *>(a.a2);
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (act[v])
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    acc[v * VW + e] += dsj * a1[off[v] + e] + dtsum * a2[off[v] + e];
    }
#pragma unroll
    for (int v = 0; v < NV; ++v)
        if (act[v]) St<Acc, VW>::run(dst + off[v], acc + v * VW);
    if (lane == 0) {
        if (chunk >= 0) static_cast<Acc *>(a.part_sc)[chunk] = dtsum;
        else static_cast<Acc *>(a.out_sc)[line] = dtsum;
    }
}

// (3) For the split columns, after their merges: dH_j += ds_j a1 + dt_j a2.
template <class Acc>
__global__ __launch_bounds__(kBlock) void gat_bwd_split_finish_kernel(const int32_t *__restrict__ splits,
                                                                      int32_t n_splits, int32_t r,
                                                                      const Acc *__restrict__ a1,
                                                                      const Acc *__restrict__ a2,
                                                                      const Acc *__restrict__ ds,
                                                                      const Acc *__restrict__ dt,
                                                                      Acc *__restrict__ dH)
{
    const int64_t tid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (tid >= (int64_t)n_splits * r) return;
    const int32_t line = splits[3 * (tid / r)];
    const int32_t k = (int32_t)(tid % r);
    dH[(size_t)line * r + k] += ds[line] * a1[k] + dt[line] * a2[k];
}

// (4) Per-block partial sums of ds_j H_j and dt_j H_j over the block's kFinishRows rows
// (in row order).
template <class TH, class Acc>
__global__ __launch_bounds__(kBlock) void gat_bwd_da_kernel(int32_t n, int32_t r, const TH *__restrict__ H,
                                                            const Acc *__restrict__ ds, const Acc *__restrict__ dt,
                                                            Acc *__restrict__ part)
{
    const int64_t r0 = (int64_t)blockIdx.x * kFinishRows;
    const int64_t r1 = r0 + kFinishRows < n ? r0 + kFinishRows : n;
    for (int k = threadIdx.x; k < r; k += kBlock) {
        Acc p1 = Acc(0), p2 = Acc(0);
        int64_t j = r0;
        for (; j + 8 <= r1; j += 8) {  // eight rows' loads in flight, added in row order
            Acc h[8], a[8], b[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                h[u] = widen<Acc>(H[(j + u) * r + k]);
                a[u] = ds[j + u];
                b[u] = dt[j + u];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                p1 += a[u] * h[u];
                p2 += b[u] * h[u];
            }
        }
        for (; j < r1; ++j) {
            const Acc h = widen<Acc>(H[j * r + k]);
            p1 += ds[j] * h;
            p2 += dt[j] * h;
        }
        part[(size_t)blockIdx.x * 2 * r + k] = p1;
        part[(size_t)blockIdx.x * 2 * r + r + k] = p2;
    }
}

// (5) da1 = sum_b part[b][0:r], da2 = sum_b part[b][r:2r], blocks in order.
template <class Acc>
__global__ __launch_bounds__(kBlock) void gat_bwd_reduce_kernel(int32_t nb, int32_t r, const Acc *__restrict__ part,
                                                                Acc *__restrict__ da1, Acc *__restrict__ da2)
{
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= 2 * r) return;
    Acc sum = Acc(0);
    int32_t b = 0;
    for (; b + 8 <= nb; b += 8) {
        Acc x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = part[(size_t)(b + u) * 2 * r + k];
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += x[u];
    }
    for (; b < nb; ++b) sum += part[(size_t)b * 2 * r + k];
    if (k < r) da1[k] = sum;
    else da2[k - r] = sum;
}

inline size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct BwdLayout {
    size_t rs, ds, dt, psc_r, pvec_c, psc_c, pblk, total;
};

BwdLayout bwd_layout(const fmm_sparse *S_csr, const fmm_sparse *S_csc, int32_t r, size_t ob)
{
    const int64_t n = S_csr->rows;
    const int64_t ncr = S_csr->n_chunks > 0 ? S_csr->n_chunks : 0;
    const int64_t ncc = S_csc->n_chunks > 0 ? S_csc->n_chunks : 0;
    const int64_t nb = (n + kFinishRows - 1) / kFinishRows;
    BwdLayout l;
    size_t o = 0;
    l.rs = o; o += al256((size_t)n * 4 * ob);
    l.ds = o; o += al256((size_t)n * ob);
    l.dt = o; o += al256((size_t)n * ob);
    l.psc_r = o; o += al256((size_t)ncr * ob);
    l.pvec_c = o; o += al256((size_t)ncc * r * ob);
    l.psc_c = o; o += al256((size_t)ncc * ob);
    l.pblk = o; o += al256((size_t)nb * 2 * r * ob);
    l.total = o + 256;
    return l;
}

Shape bwd_shape(int r, int vw)
{
    Shape s = default_shape(r, vw);
    if (s.NV == 2 && s.L != 64) s = Shape{64, 1};
    return s;
}

template <class TH, class TO, class Acc, int L, int NV, int VW>
hipError_t run_bwd_shape(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const TH *H, const Acc *a1, const Acc *a2,
                         const Acc *s, const Acc *t, const Acc *out, const Acc *lse, const TO *dO, int32_t r,
                         Acc slope, bool softmax, Acc *dH, Acc *da1, Acc *da2, Acc *dS, char *ws, hipStream_t st)
{
    constexpr int GPB = kBlock / L;
    constexpr int UR = NV == 1 ? 8 : 4;  // batch depth of the row pass
    constexpr int UC = NV == 1 ? 4 : 2;  // and of the column pass (more live registers per entry)
    const int32_t n = S_csr->rows;
    const BwdLayout lay = bwd_layout(S_csr, S_csc, r, sizeof(Acc));
    void *rsb = ws + lay.rs;
    Acc *ds = reinterpret_cast<Acc *>(ws + lay.ds);
    Acc *dt = reinterpret_cast<Acc *>(ws + lay.dt);
    hipError_t e;
    if (n == 0) {  // da1 = da2 = 0
        hipLaunchKernelGGL((gat_bwd_reduce_kernel<Acc>), dim3((unsigned)((2 * r + kBlock - 1) / kBlock)),
                           dim3(kBlock), 0, st, 0, r, (const Acc *)nullptr, da1, da2);
        return hipGetLastError();
    }
    const unsigned nb_rows = (unsigned)(((int64_t)n + GPB - 1) / GPB);

    GatBwdArgs a;
    memset(&a, 0, sizeof(a));
    a.r = r;
    a.s = s;
    a.t = t;
    a.lse = lse;
    a.rs = rsb;
    a.slope = (double)slope;
    a.softmax = softmax ? 1 : 0;
    // (1) row pass: D, ds, dS
    a.nlines = n;
    a.ptr = S_csr->ptr;
    a.idx = S_csr->idx;
    a.val = S_csr->val;
    a.held = dO;
    a.gath = H;
    a.out = out;
    a.long_len = S_csr->long_len;
    a.n_chunks = S_csr->n_chunks;
    a.chunks = S_csr->chunks;
    a.order = S_csr->order;
    a.out_sc = ds;
    a.part_sc = ws + lay.psc_r;
    a.dS = dS;
    int64_t nbc = a.n_chunks > 0 ? ((int64_t)a.n_chunks + GPB - 1) / GPB : 0;
    hipLaunchKernelGGL((gat_bwd_rows_kernel<TH, TO, Acc, L, NV, VW, UR>), dim3((unsigned)(nbc + nb_rows)), dim3(kBlock),
                       0, st, a, (int32_t)nbc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (S_csr->n_chunks > 0 && S_csr->n_splits > 0) {
        const int64_t mb = ((int64_t)S_csr->n_splits + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(merge_kernel<Acc>, dim3((unsigned)mb), dim3(kBlock), 0, st, S_csr->splits, S_csr->n_splits,
                           1, static_cast<const Acc *>(a.part_sc), ds, 0.0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // (2) column pass: dt and dH (whole columns get their rank-one terms here)
    a.nlines = S_csc->cols;
    a.ptr = S_csc->ptr;
    a.idx = S_csc->idx;
    a.val = S_csc->val;
    a.held = H;
    a.gath = dO;
    a.out = nullptr;
    a.a1 = a1;
    a.a2 = a2;
    a.ds = ds;
    a.long_len = S_csc->long_len;
    a.n_chunks = S_csc->n_chunks;
    a.chunks = S_csc->chunks;
    a.order = S_csc->order;
    a.out_vec = dH;
    a.out_sc = dt;
    a.part_vec = ws + lay.pvec_c;
    a.part_sc = ws + lay.psc_c;
    a.dS = nullptr;
    nbc = a.n_chunks > 0 ? ((int64_t)a.n_chunks + GPB - 1) / GPB : 0;
    hipLaunchKernelGGL((gat_bwd_cols_kernel<TH, TO, Acc, L, NV, VW, UC>), dim3((unsigned)(nbc + nb_rows)), dim3(kBlock),
                       0, st, a, (int32_t)nbc);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // (3) split columns: merge their chunks, then add their rank-one terms
    if (S_csc->n_chunks > 0 && S_csc->n_splits > 0) {
        const int64_t mv = ((int64_t)S_csc->n_splits * r + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(merge_kernel<Acc>, dim3((unsigned)mv), dim3(kBlock), 0, st, S_csc->splits, S_csc->n_splits,
                           r, static_cast<const Acc *>(a.part_vec), dH, 0.0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        const int64_t ms = ((int64_t)S_csc->n_splits + kBlock - 1) / kBlock;
        hipLaunchKernelGGL(merge_kernel<Acc>, dim3((unsigned)ms), dim3(kBlock), 0, st, S_csc->splits, S_csc->n_splits,
                           1, static_cast<const Acc *>(a.part_sc), dt, 0.0);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((gat_bwd_split_finish_kernel<Acc>), dim3((unsigned)mv), dim3(kBlock), 0, st,
                           S_csc->splits, S_csc->n_splits, r, a1, a2, (const Acc *)ds, (const Acc *)dt, dH);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // (4), (5) da1 = H^T ds, da2 = H^T dt
    const int64_t nbf = ((int64_t)n + kFinishRows - 1) / kFinishRows;
    Acc *part = reinterpret_cast<Acc *>(ws + lay.pblk);
    hipLaunchKernelGGL((gat_bwd_da_kernel<TH, Acc>), dim3((unsigned)nbf), dim3(kBlock), 0, st, n, r, H,
                       (const Acc *)ds, (const Acc *)dt, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((gat_bwd_reduce_kernel<Acc>), dim3((unsigned)((2 * r + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       st, (int32_t)nbf, r, (const Acc *)part, da1, da2);
    return hipGetLastError();
}

#define BWD_SHAPES(X) X(1, 1) X(2, 1) X(4, 1) X(8, 1) X(16, 1) X(32, 1) X(64, 1) X(64, 2) X(64, 4)

template <class TH, class TO, class Acc, int VW>
hipError_t dispatch_bwd(Shape sh, const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *H, const void *a1,
                        const void *a2, const void *s, const void *t, const void *out, const void *lse,
                        const void *dO, int32_t r,
                        double slope, bool softmax, void *dH, void *da1, void *da2, void *dS, void *ws,
                        hipStream_t st)
{
#define BWD_CASE(Lv, NVv)                                                                        \
    if (sh.L == Lv && sh.NV == NVv)                                                              \
        return run_bwd_shape<TH, TO, Acc, Lv, NVv, VW>(                                          \
            S_csr, S_csc, (const TH *)H, (const Acc *)a1, (const Acc *)a2, (const Acc *)s, (const Acc *)t, \
            (const Acc *)out, (const Acc *)lse, (const TO *)dO, r, (Acc)slope, softmax, (Acc *)dH, (Acc *)da1, (Acc *)da2, \
            (Acc *)dS, (char *)ws, st);
    BWD_SHAPES(BWD_CASE)
#undef BWD_CASE
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace fmm

using namespace fmm;

extern "C" {

fmm_status fmm_gat_backward_workspace(const fmm_sparse *S_csr, const fmm_sparse *S_csc, int32_t r, int32_t dtype,
                                      size_t *bytes)
{
    if (!bytes || !S_csr || !S_csc) return FMM_ERR_NULL;
    if (r < 1 || S_csr->rows < 0) return FMM_ERR_DIM;
    if (dtype != FMM_F32 && dtype != FMM_BF16 && dtype != FMM_F64) return FMM_ERR_DTYPE;
    *bytes = bwd_layout(S_csr, S_csc, r, dtype == FMM_F64 ? 8 : 4).total;
    return FMM_OK;
}

fmm_status fmm_gat_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *H, const void *a1,
                            const void *a2, const void *s, const void *t, const void *out, const void *lse,
                            const void *dO, int32_t r,
                            int32_t dtype, double negative_slope, int32_t flags, void *dH, void *da1, void *da2,
                            void *dS, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!S_csr || !S_csc) return FMM_ERR_NULL;
    if (S_csr->orient != FMM_CSR || S_csc->orient != FMM_CSC) return FMM_ERR_ORIENT;
    const int32_t n = S_csr->rows;
    if (n < 0 || S_csr->cols != n || S_csc->rows != n || S_csc->cols != n || S_csr->nnz != S_csc->nnz ||
        S_csr->nnz < 0 || r < 1)
        return FMM_ERR_DIM;
    if (flags & ~(FMM_GAT_SOFTMAX | FMM_DC_BF16)) return FMM_ERR_DIM;
    const bool do16 = (flags & FMM_DC_BF16) != 0;  // dO stored as bfloat16 (bfloat16 H only)
    if (do16 && dtype != FMM_BF16) return FMM_ERR_UNSUPPORTED;
    if (!S_csr->ptr || !S_csc->ptr || (S_csr->nnz > 0 && (!S_csr->idx || !S_csc->idx))) return FMM_ERR_NULL;
    if (!a1 || !a2 || !da1 || !da2) return FMM_ERR_NULL;
    if (n > 0 && (!H || !s || !t || !out || !dO || !dH)) return FMM_ERR_NULL;
    if (n > 0 && (flags & FMM_GAT_SOFTMAX) && !lse) return FMM_ERR_NULL;
    for (const fmm_sparse *S : {S_csr, S_csc}) {
        if (S->n_chunks < 0 || S->n_splits < 0) return FMM_ERR_DIM;
        if (S->n_chunks > 0 && (!S->chunks || !S->splits || S->long_len < 1)) return FMM_ERR_NULL;
    }
    const size_t ob = dtype == FMM_F64 ? 8 : 4;
    if (!ws || ws_bytes < bwd_layout(S_csr, S_csc, r, ob).total || (uintptr_t)ws % 256 != 0)
        return FMM_ERR_WORKSPACE;
    const bool softmax = (flags & FMM_GAT_SOFTMAX) != 0;
    auto misaligned = [](const void *p) { return ((uintptr_t)p % 16) != 0; };
    hipError_t e;
    if (dtype == FMM_F32) {
        const int vw = r % 4 == 0 ? 4 : 1;
        if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
        if (vw == 4 && (misaligned(H) || misaligned(out) || misaligned(dO) || misaligned(dH)))
            return FMM_ERR_UNSUPPORTED;
        const Shape sh = bwd_shape(r, vw);
        e = vw == 4 ? dispatch_bwd<float, float, float, 4>(sh, S_csr, S_csc, H, a1, a2, s, t, out, lse, dO, r, negative_slope,
                                                    softmax, dH, da1, da2, dS, ws, stream)
                    : dispatch_bwd<float, float, float, 1>(sh, S_csr, S_csc, H, a1, a2, s, t, out, lse, dO, r, negative_slope,
                                                    softmax, dH, da1, da2, dS, ws, stream);
    } else if (dtype == FMM_BF16) {
        if (r % 8 != 0 || r > 1024) return FMM_ERR_DTYPE;
        if (misaligned(H) || misaligned(out) || misaligned(dO) || misaligned(dH)) return FMM_ERR_UNSUPPORTED;
        e = do16 ? dispatch_bwd<bf16_t, bf16_t, float, 8>(bwd_shape(r, 8), S_csr, S_csc, H, a1, a2, s, t, out, lse,
                                                          dO, r, negative_slope, softmax, dH, da1, da2, dS, ws, stream)
                 : dispatch_bwd<bf16_t, float, float, 8>(bwd_shape(r, 8), S_csr, S_csc, H, a1, a2, s, t, out, lse,
                                                         dO, r, negative_slope, softmax, dH, da1, da2, dS, ws, stream);
    } else if (dtype == FMM_F64) {
        const int vw = r % 2 == 0 ? 2 : 1;
        if (r > 64 * 4 * vw) return FMM_ERR_DTYPE;
        if (vw == 2 && (misaligned(H) || misaligned(out) || misaligned(dO) || misaligned(dH)))
            return FMM_ERR_UNSUPPORTED;
        const Shape sh = bwd_shape(r, vw);
        e = vw == 2 ? dispatch_bwd<double, double, double, 2>(sh, S_csr, S_csc, H, a1, a2, s, t, out, lse, dO, r, negative_slope,
                                                      softmax, dH, da1, da2, dS, ws, stream)
                    : dispatch_bwd<double, double, double, 1>(sh, S_csr, S_csc, H, a1, a2, s, t, out, lse, dO, r, negative_slope,
                                                      softmax, dH, da1, da2, dS, ws, stream);
    } else {
        return FMM_ERR_DTYPE;
    }
    if (e != hipSuccess) {
        set_last_hip_error((int32_t)e);
        return FMM_ERR_HIP;
    }
    return FMM_OK;
}

}  // extern "C"
