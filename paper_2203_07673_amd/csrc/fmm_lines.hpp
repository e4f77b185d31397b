// Line kernels of the local FusedMM path for gfx950 (CDNA4, wave64).
//
// Every operation of the path walks the stored entries of S one major line at a
// time (a row of the CSR, or a column of the stored transposed copy), touching for
// each entry p = (line, idx[p]) one row of a "held" dense matrix H (the line's own
// row, kept in registers) and one gathered row of G1 (and G2).  This is the shared
// access pattern of SDDMM and SpMM the paper points out in Section IV-A.  The six
// operations differ only in what they do per entry:
//
//   OP_SDDMM  : R[p]    = beta R[p] + w_p <H_line, G1_j>                  (Eq. (1))
//   OP_SPMM1  : out_line = beta out + sum_p w_p G1_j                       (SpMMA/SpMMB)
//   OP_SPMM2  : out_line = beta out + sum_p (w_p G1_j + w'_p G2_j)         (two SpMMs, one pass)
//   OP_FUSED1 : out_line = beta out + sum_p w_p <H_line, G1_j> G1_j        (FusedMMA row form,
//                                                                           Section IV-B)
//   OP_FUSED2 : out_line = beta out + sum_p w_p (<H,G2_j> G1_j + <H,G1_j> G2_j)
//               (the column pass of the adjoints: both sampled products recomputed)
//   OP_FUSED1S: OP_FUSED1 plus, per entry, V[p] = <H_line, G1_j> <H2_line, G1_j> with a
//               second held row H2 (the gradient with respect to S's values, written with
//               the adjoint row pass; out may be NULL)
//   OP_CG     : OP_FUSED1 on the pattern alone, where the line's sum q = M p is consumed in
//               registers by one conjugate-gradient step of that line (batched CG of the
//               ALS application): X, R, P (= H, updated in place) and rr; nothing else
//               is written
//
// Work decomposition.  A group of L lanes (L | 64) owns one line; lane l holds
// elements k = (v*L + l)*VW + e (v < NV, e < VW) of each r-vector, so one vector
// load per (v, entry) covers a contiguous L*VW-element span: coalesced 16-byte
// loads per lane.  A dot product is a lane-local FMA chain followed by an
// all-reduce over the group with DPP row permutes (quad_perm, row_half_mirror,
// row_mirror) and the gfx950 permlane16/32 swaps; every lane ends with the same
// sum, so no broadcast is needed and no LDS is touched.  U entries are loaded
// before any of them is reduced, to keep U row gathers in flight per group.
//
// Gather hints: with a per-entry hint array, entries whose hint is 0 gather their row
// with the streaming (nontemporal) policy, so rows gathered once do not displace the
// rows of hub lines, which many entries gather, from L2 and the MALL.
//
// Long lines: with a split schedule, lines longer than long_len are skipped by
// the line groups and processed as chunks (line, begin, end) whose partial
// r-vectors go to a workspace; merge_kernel adds them in chunk order.  Chunk
// blocks come first in the grid so the heaviest items start first.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>


namespace fmm {

typedef uint16_t bf16_t;

// Stand-ins for absent per-entry arrays: read with stride 0 they give 1 (weights) or 0.
static __device__ const float kUnitF[1] = {1.0f};
static __device__ const double kUnitD[1] = {1.0};
static __device__ const int32_t kZeroIdx[1] = {0};
static __device__ const uint8_t kHotByte[1] = {1};
template <class Acc> __device__ __forceinline__ const Acc *unit_value();
template <> __device__ __forceinline__ const float *unit_value<float>() { return kUnitF; }
template <> __device__ __forceinline__ const double *unit_value<double>() { return kUnitD; }
__device__ __forceinline__ const int32_t *zero_index() { return kZeroIdx; }

enum { OP_SDDMM = 0, OP_SPMM1 = 1, OP_SPMM2 = 2, OP_FUSED1 = 3, OP_FUSED2 = 4, OP_FUSED1S = 5, OP_CG = 6 };

constexpr int kBlock = 256;

struct LineArgs {
    int32_t nlines;
    int32_t r;
    const int32_t *ptr;
    const int32_t *idx;
    const void *val;      // per-entry weight in orientation order (Acc), NULL = 1
    const void *wv1;      // extra per-entry factor for G1 (Acc), NULL = 1
    const void *wv2;      // extra per-entry factor for G2 (Acc), NULL = 1 (OP_SPMM2)
    const int32_t *wperm; // wv1/wv2 are read at wperm[p] instead of p when non-NULL
    const int32_t *operm; // OP_SDDMM writes R[operm[p]] instead of R[p] when non-NULL
    const void *H;
    const void *G1;
    const void *G2;
    const void *H2;       // second held matrix (TG2 elements), OP_FUSED1S
    void *out;            // lines x r (Acc), or nnz (Acc) for OP_SDDMM; may be NULL for OP_FUSED1S
    void *values;         // nnz per-entry output (Acc) of OP_FUSED1S, through operm when non-NULL
    float *cg_X, *cg_R, *cg_P, *cg_rr;  // OP_CG: iterate, residual, direction (the held rows), <R, R>
    float cg_lambda;                    // OP_CG: ridge term of the line operator
    double beta;
    int32_t long_len;
    int32_t n_chunks;
    const int32_t *chunks;
    void *partial;        // n_chunks x r (Acc)
    int32_t uclass;       // batch depth class, 1 (deep) .. 3 (shallow)
    const int32_t *order; // line processing order (a permutation of the lines), NULL = index order
    const uint8_t *hot;   // per-entry gather hint in orientation order (0: streaming policy), NULL = all 1
};

// ------------------------------------------------------------------ conversions

__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xffff0000u); }
// Two floats that are bfloat16 values (widened exactly) packed back into one word, lo first.
__device__ __forceinline__ uint32_t bf16_pack_exact(float lo, float hi)
{
    return (__float_as_uint(hi) & 0xffff0000u) | (__float_as_uint(lo) >> 16);
}

// c + a.lo * b.lo + a.hi * b.hi over two packed bfloat16 pairs: gfx950's bf16 dot
// instruction (v_dot2c_f32_bf16).  Each product of two bfloat16 values is exact in
// float32, so only the accumulation rounds; it replaces two widenings of b and two FMAs.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c,
                                           false);
}

// Streaming (nontemporal) cache hint for data a pass touches once, so that it does not
// displace gathered rows (the only reused data) from L2 and the MALL.  On by default for
// the held rows (one 16-byte load per lane per line) and the row outputs.  Off for the
// index and weight arrays: they are read with one dword load per entry, and the lines
// that consecutive batches share would be refetched.  Off for the gathered rows, whose
// reuse is the point of the cache.  Every setting gives the same results.
#ifndef FMM_NT_META
#define FMM_NT_META 0
#endif
#ifndef FMM_NT_HELD
#define FMM_NT_HELD 1
#endif
#ifndef FMM_NT_STORE
#define FMM_NT_STORE 1
#endif
#ifndef FMM_NT_GATHER
#define FMM_NT_GATHER 0
#endif
constexpr bool kNtMeta = FMM_NT_META != 0;
constexpr bool kNtHeld = FMM_NT_HELD != 0;
constexpr bool kNtStore = FMM_NT_STORE != 0;
constexpr bool kNtGather = FMM_NT_GATHER != 0;

typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));

template <bool NT, class V> __device__ __forceinline__ V ld_hint(const V *p)
{
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class V> __device__ __forceinline__ void st_hint(V *p, V v)
{
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Load VW consecutive elements of T at p (16-byte vector loads where VW*sizeof(T)
// is a multiple of 16) and widen them to Acc; NT: with the streaming hint.
template <class T, int VW, class Acc> struct Ld;

template <> struct Ld<float, 1, float> {
    template <bool NT = false> static __device__ __forceinline__ void run(const float *p, float *o) {
        o[0] = ld_hint<NT>(p);
    }
};
template <> struct Ld<float, 4, float> {
    template <bool NT = false> static __device__ __forceinline__ void run(const float *p, float *o) {
        if constexpr (NT) {
            const f32x4_t v = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p));
            o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
        } else {
            float4 v = *reinterpret_cast<const float4 *>(p);
            o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
        }
    }
};
template <> struct Ld<float, 8, float> {
    template <bool NT = false> static __device__ __forceinline__ void run(const float *p, float *o) {
        if constexpr (NT) {
            const f32x4_t v = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p));
            const f32x4_t w = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p) + 1);
            o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
            o[4] = w.x; o[5] = w.y; o[6] = w.z; o[7] = w.w;
        } else {
            float4 v = reinterpret_cast<const float4 *>(p)[0];
            float4 w = reinterpret_cast<const float4 *>(p)[1];
            o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
            o[4] = w.x; o[5] = w.y; o[6] = w.z; o[7] = w.w;
        }
    }
};
template <> struct Ld<bf16_t, 8, float> {
    template <bool NT = false> static __device__ __forceinline__ void run(const bf16_t *p, float *o) {
        if constexpr (NT) {
            const u32x4_t v = ld_hint<true>(reinterpret_cast<const u32x4_t *>(p));
            o[0] = bf16_lo(v.x); o[1] = bf16_hi(v.x); o[2] = bf16_lo(v.y); o[3] = bf16_hi(v.y);
            o[4] = bf16_lo(v.z); o[5] = bf16_hi(v.z); o[6] = bf16_lo(v.w); o[7] = bf16_hi(v.w);
        } else {
            uint4 v = *reinterpret_cast<const uint4 *>(p);
            o[0] = bf16_lo(v.x); o[1] = bf16_hi(v.x); o[2] = bf16_lo(v.y); o[3] = bf16_hi(v.y);
            o[4] = bf16_lo(v.z); o[5] = bf16_hi(v.z); o[6] = bf16_lo(v.w); o[7] = bf16_hi(v.w);
        }
    }
};
template <> struct Ld<double, 1, double> {
    template <bool NT = false> static __device__ __forceinline__ void run(const double *p, double *o) {
        o[0] = ld_hint<NT>(p);
    }
};
template <> struct Ld<double, 2, double> {
    template <bool NT = false> static __device__ __forceinline__ void run(const double *p, double *o) {
        if constexpr (NT) {
            const f64x2_t v = ld_hint<true>(reinterpret_cast<const f64x2_t *>(p));
            o[0] = v.x; o[1] = v.y;
        } else {
            double2 v = *reinterpret_cast<const double2 *>(p);
            o[0] = v.x; o[1] = v.y;
        }
    }
};

// Fused multiply-add written out, so that every kernel that runs a line (the line kernel
// and the batched kernels, each compiled on its own) rounds each update the same way:
// the compiler's own contraction of an expression such as x += a*b + c*d may differ
// between instantiations.
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmadd(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class Acc, int VW> struct St;
template <> struct St<float, 1> {
    template <bool NT = false> static __device__ __forceinline__ void run(float *p, const float *v) {
        st_hint<NT>(p, v[0]);
    }
};
template <> struct St<float, 4> {
    template <bool NT = false> static __device__ __forceinline__ void run(float *p, const float *v) {
        if constexpr (NT) st_hint<true>(reinterpret_cast<f32x4_t *>(p), f32x4_t{v[0], v[1], v[2], v[3]});
        else *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};
template <> struct St<float, 8> {
    template <bool NT = false> static __device__ __forceinline__ void run(float *p, const float *v) {
        if constexpr (NT) {
            st_hint<true>(reinterpret_cast<f32x4_t *>(p), f32x4_t{v[0], v[1], v[2], v[3]});
            st_hint<true>(reinterpret_cast<f32x4_t *>(p) + 1, f32x4_t{v[4], v[5], v[6], v[7]});
        } else {
            reinterpret_cast<float4 *>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
            reinterpret_cast<float4 *>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
        }
    }
};
template <> struct St<double, 1> {
    template <bool NT = false> static __device__ __forceinline__ void run(double *p, const double *v) {
        st_hint<NT>(p, v[0]);
    }
};
template <> struct St<double, 2> {
    template <bool NT = false> static __device__ __forceinline__ void run(double *p, const double *v) {
        if constexpr (NT) st_hint<true>(reinterpret_cast<f64x2_t *>(p), f64x2_t{v[0], v[1]});
        else *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    }
};

// Raw vectors of a gathered row, kept in their storage type until each element is
// used (bfloat16 stays packed: 4 registers per 8 elements instead of 8).
template <class T, int VW> struct Raw;
template <> struct Raw<float, 1> {
    float x;
    __device__ __forceinline__ void pin() {}
    __device__ __forceinline__ void load(const float *p) { x = ld_hint<kNtGather>(p); }
    __device__ __forceinline__ void load_nt(const float *p) { x = ld_hint<true>(p); }
    __device__ __forceinline__ void zero() { x = 0.f; }
    __device__ __forceinline__ float get(int) const { return x; }
};
template <> struct Raw<float, 4> {
    float4 x;
    __device__ __forceinline__ void pin() {}
    __device__ __forceinline__ void load(const float *p) {
        if constexpr (kNtGather) {
            const f32x4_t v = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p));
            x = make_float4(v.x, v.y, v.z, v.w);
        } else {
            x = *reinterpret_cast<const float4 *>(p);
        }
    }
    __device__ __forceinline__ void load_nt(const float *p) {
        const f32x4_t v = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p));
        x = make_float4(v.x, v.y, v.z, v.w);
    }
    __device__ __forceinline__ void zero() { x = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ __forceinline__ float get(int e) const { return e == 0 ? x.x : e == 1 ? x.y : e == 2 ? x.z : x.w; }
};
template <> struct Raw<float, 8> {
    float4 x, y;
    __device__ __forceinline__ void pin() {}
    __device__ __forceinline__ void load(const float *p) {
        if constexpr (kNtGather) {
            const f32x4_t v = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p));
            const f32x4_t w = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p) + 1);
            x = make_float4(v.x, v.y, v.z, v.w);
            y = make_float4(w.x, w.y, w.z, w.w);
        } else {
            x = reinterpret_cast<const float4 *>(p)[0];
            y = reinterpret_cast<const float4 *>(p)[1];
        }
    }
    __device__ __forceinline__ void load_nt(const float *p) {
        const f32x4_t v = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p));
        const f32x4_t w = ld_hint<true>(reinterpret_cast<const f32x4_t *>(p) + 1);
        x = make_float4(v.x, v.y, v.z, v.w);
        y = make_float4(w.x, w.y, w.z, w.w);
    }
    __device__ __forceinline__ void zero() { x = y = make_float4(0.f, 0.f, 0.f, 0.f); }
    __device__ __forceinline__ float get(int e) const {
        const float4 &q = e < 4 ? x : y;
        const int f = e & 3;
        return f == 0 ? q.x : f == 1 ? q.y : f == 2 ? q.z : q.w;
    }
};
template <> struct Raw<bf16_t, 8> {
    uint4 x;
    __device__ __forceinline__ void load(const bf16_t *p) {
        if constexpr (kNtGather) {
            const u32x4_t v = ld_hint<true>(reinterpret_cast<const u32x4_t *>(p));
            x = make_uint4(v.x, v.y, v.z, v.w);
        } else {
            x = *reinterpret_cast<const uint4 *>(p);
        }
    }
    __device__ __forceinline__ void load_nt(const bf16_t *p) {
        const u32x4_t v = ld_hint<true>(reinterpret_cast<const u32x4_t *>(p));
        x = make_uint4(v.x, v.y, v.z, v.w);
    }
    __device__ __forceinline__ void zero() { x = make_uint4(0u, 0u, 0u, 0u); }
    // Make the packed words opaque to the optimiser, so elements widened for the dot
    // product are widened again for the update instead of staying live in between.
    __device__ __forceinline__ void pin() { asm volatile("" : "+v"(x.x), "+v"(x.y), "+v"(x.z), "+v"(x.w)); }
    __device__ __forceinline__ uint32_t word(int k) const { return k == 0 ? x.x : k == 1 ? x.y : k == 2 ? x.z : x.w; }
    __device__ __forceinline__ float get(int e) const {
        const uint32_t w = word(e >> 1);
        return (e & 1) ? bf16_hi(w) : bf16_lo(w);
    }
};
template <> struct Raw<double, 1> {
    double x;
    __device__ __forceinline__ void pin() {}
    __device__ __forceinline__ void load(const double *p) { x = p[0]; }
    __device__ __forceinline__ void load_nt(const double *p) { x = ld_hint<true>(p); }
    __device__ __forceinline__ void zero() { x = 0.0; }
    __device__ __forceinline__ double get(int) const { return x; }
};
template <> struct Raw<double, 2> {
    double2 x;
    __device__ __forceinline__ void pin() {}
    __device__ __forceinline__ void load(const double *p) { x = *reinterpret_cast<const double2 *>(p); }
    __device__ __forceinline__ void load_nt(const double *p) {
        const f64x2_t v = ld_hint<true>(reinterpret_cast<const f64x2_t *>(p));
        x = make_double2(v.x, v.y);
    }
    __device__ __forceinline__ void zero() { x = make_double2(0.0, 0.0); }
    __device__ __forceinline__ double get(int e) const { return e == 0 ? x.x : x.y; }
};

// ------------------------------------------------------------------ group all-reduce

template <int CTRL> __device__ __forceinline__ float dpp_f(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

__device__ __forceinline__ float swap16_sum(float x) {
    auto s = __builtin_amdgcn_permlane16_swap(__float_as_int(x), __float_as_int(x), false, false);
    return __int_as_float(s[0]) + __int_as_float(s[1]);
}
__device__ __forceinline__ float swap32_sum(float x) {
    auto s = __builtin_amdgcn_permlane32_swap(__float_as_int(x), __float_as_int(x), false, false);
    return __int_as_float(s[0]) + __int_as_float(s[1]);
}

// Sum over an aligned group of L lanes; every lane of the group gets the same value.
// Each step adds the value of a partner lane in the other half of the current
// span, and a + b == b + a exactly, so partners agree bit for bit.
template <int L> __device__ __forceinline__ float group_sum(float x) {
    if constexpr (L >= 2) x += dpp_f<0xB1>(x);   // quad_perm [1,0,3,2]
    if constexpr (L >= 4) x += dpp_f<0x4E>(x);   // quad_perm [2,3,0,1]
    if constexpr (L >= 8) x += dpp_f<0x141>(x);  // row_half_mirror
    if constexpr (L >= 16) x += dpp_f<0x140>(x); // row_mirror
    if constexpr (L >= 32) x = swap16_sum(x);
    if constexpr (L >= 64) x = swap32_sum(x);
    return x;
}

template <int CTRL> __device__ __forceinline__ double dpp_d(double x) {
    int2 v = *reinterpret_cast<int2 *>(&x);
    int2 o;
    o.x = __builtin_amdgcn_update_dpp(0, v.x, CTRL, 0xF, 0xF, false);
    o.y = __builtin_amdgcn_update_dpp(0, v.y, CTRL, 0xF, 0xF, false);
    return *reinterpret_cast<double *>(&o);
}
__device__ __forceinline__ double swap16_sum(double x) {
    int2 v = *reinterpret_cast<int2 *>(&x);
    auto a = __builtin_amdgcn_permlane16_swap(v.x, v.x, false, false);
    auto b = __builtin_amdgcn_permlane16_swap(v.y, v.y, false, false);
    int2 p0 = make_int2(a[0], b[0]), p1 = make_int2(a[1], b[1]);
    return *reinterpret_cast<double *>(&p0) + *reinterpret_cast<double *>(&p1);
}
__device__ __forceinline__ double swap32_sum(double x) {
    int2 v = *reinterpret_cast<int2 *>(&x);
    auto a = __builtin_amdgcn_permlane32_swap(v.x, v.x, false, false);
    auto b = __builtin_amdgcn_permlane32_swap(v.y, v.y, false, false);
    int2 p0 = make_int2(a[0], b[0]), p1 = make_int2(a[1], b[1]);
    return *reinterpret_cast<double *>(&p0) + *reinterpret_cast<double *>(&p1);
}
template <int L> __device__ __forceinline__ double group_sum(double x) {
    if constexpr (L >= 2) x += dpp_d<0xB1>(x);
    if constexpr (L >= 4) x += dpp_d<0x4E>(x);
    if constexpr (L >= 8) x += dpp_d<0x141>(x);
    if constexpr (L >= 16) x += dpp_d<0x140>(x);
    if constexpr (L >= 32) x = swap16_sum(x);
    if constexpr (L >= 64) x = swap32_sum(x);
    return x;
}

// ------------------------------------------------------------------ cross-group sum

// Sum over the GPL groups (of L lanes each) that share one wave when L * GPL == 64:
// rotations inside 16-lane rows (row_ror by L, 2L, ...), then the row-pair and
// half-wave swaps.  Every lane ends with a full sum; callers store group 0's copy.
template <int L, int GPL> __device__ __forceinline__ float cross_group_sum(float x) {
    static_assert(GPL == 1 || L * GPL == 64, "groups of a line must fill the wave");
    if constexpr (GPL > 1) {
        if constexpr (L < 16) {
#pragma unroll
            for (int s = L; s < 16; s <<= 1) {
                if (s == 1) x += dpp_f<0x121>(x);
                else if (s == 2) x += dpp_f<0x122>(x);
                else if (s == 4) x += dpp_f<0x124>(x);
                else x += dpp_f<0x128>(x);
            }
        }
        if constexpr (L < 32) x = swap16_sum(x);
        x = swap32_sum(x);
    }
    return x;
}
template <int L, int GPL> __device__ __forceinline__ double cross_group_sum(double x) {
    static_assert(GPL == 1 || L * GPL == 64, "groups of a line must fill the wave");
    if constexpr (GPL > 1) {
        if constexpr (L < 16) {
#pragma unroll
            for (int s = L; s < 16; s <<= 1) {
                if (s == 1) x += dpp_d<0x121>(x);
                else if (s == 2) x += dpp_d<0x122>(x);
                else if (s == 4) x += dpp_d<0x124>(x);
                else x += dpp_d<0x128>(x);
            }
        }
        if constexpr (L < 32) x = swap16_sum(x);
        x = swap32_sum(x);
    }
    return x;
}

// ------------------------------------------------------------------ one line

// Operands of a line pass (device pointers; types fixed by the template).
struct LineOperands {
    const int32_t *idx;
    const void *val;
    const void *wv1;
    const void *wv2;
    const int32_t *wperm;
    const int32_t *operm;
    const void *H;
    const void *G1;
    const void *G2;
    const void *H2;  // OP_FUSED1S second held matrix
    const uint8_t *hot;  // per-entry gather hint (NULL: every row with the default policy)
    void *R;         // per-entry output (nnz): OP_SDDMM, OP_FUSED1S
    float *cg_X, *cg_R, *cg_P, *cg_rr;  // OP_CG
    float cg_lambda;
    int32_t r;
    double beta;
};

// One conjugate-gradient step of one line, with q = M p (the line's sum, in registers)
// and p (the held row):  alpha = rr / <p, q + lambda p>;  x += alpha p;
// r -= alpha (q + lambda p);  beta = <r, r>_new / rr;  p = r + beta p;  rr = <r, r>_new.
// A line with zero residual or curvature keeps its iterate (alpha = beta = 0).
template <int L, int NV, int VW, class Acc>
__device__ __forceinline__ void cg_line_step(const LineOperands &o, int32_t line, int lane, const bool *act,
                                             const int *off, const Acc *h, const Acc *acc)
{
    constexpr int E = NV * VW;
    const size_t base = (size_t)line * o.r;
    const float lam = o.cg_lambda;
    float mq[E];
    float pq = 0.f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        mq[e] = float(acc[e]) + lam * float(h[e]);  // inactive lanes hold zeros
        pq += float(h[e]) * mq[e];
    }
    pq = group_sum<L>(pq);
    const float rr_old = o.cg_rr[line];
    const float alpha = (rr_old > 0.f && pq > 0.f) ? rr_old / pq : 0.f;
    float res[E];
    float rrn = 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (!act[v]) {
#pragma unroll
            for (int e = 0; e < VW; ++e) res[v * VW + e] = 0.f;
            continue;
        }
        float x[VW], rv[VW];
        Ld<float, VW, float>::run(o.cg_X + base + off[v], x);
        Ld<float, VW, float>::run(o.cg_R + base + off[v], rv);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            x[e] += alpha * float(h[v * VW + e]);
            res[v * VW + e] = rv[e] - alpha * mq[v * VW + e];
            rrn += res[v * VW + e] * res[v * VW + e];
        }
        St<float, VW>::run(o.cg_X + base + off[v], x);
        St<float, VW>::run(o.cg_R + base + off[v], res + v * VW);
    }
    rrn = group_sum<L>(rrn);
    const float beta = rr_old > 0.f ? rrn / rr_old : 0.f;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        if (!act[v]) continue;
        float np[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) np[e] = res[v * VW + e] + beta * float(h[v * VW + e]);
        St<float, VW>::run(o.cg_P + base + off[v], np);
    }
    if (lane == 0) o.cg_rr[line] = rrn;
}

// Process entries [begin, end) of one major line.  GPL groups of L lanes may share the
// line (GPL > 1: wavefront-per-line; group gidx takes every GPL-th batch of U entries
// and the partial sums are added across groups at the end).  dst receives the line's
// r-vector (beta applied when keep_beta); OP_SDDMM writes per-entry values instead.
template <int OP, class TH, class TG1, class TG2, class Acc, int L, int NV, int VW, int U, int GPL, bool PF = true>
__device__ __forceinline__ void process_line(const LineOperands &o, int lane, int gidx, int32_t line, int32_t begin,
                                             int32_t end, Acc *dst, bool keep_beta)
{
    constexpr int E = NV * VW;  // elements per lane
    const int r = o.r;

    // vector chunks this lane owns inside an r-vector
    const int C = r / VW;
    bool act[NV];
    int off[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const int cidx = v * L + lane;
        act[v] = cidx < C;
        off[v] = cidx * VW;
    }

    const int32_t *__restrict__ idx = o.idx;
    const Acc *__restrict__ val = static_cast<const Acc *>(o.val);
    const Acc *__restrict__ wv1 = static_cast<const Acc *>(o.wv1);
    const Acc *__restrict__ wv2 = static_cast<const Acc *>(o.wv2);
    const int32_t *__restrict__ wperm = o.wperm;
    const TG1 *__restrict__ G1 = static_cast<const TG1 *>(o.G1);
    const TG2 *__restrict__ G2 = static_cast<const TG2 *>(o.G2);

    constexpr bool kHeld = (OP == OP_SDDMM || OP == OP_FUSED1 || OP == OP_FUSED2 || OP == OP_FUSED1S || OP == OP_CG);
    constexpr bool kHeld2 = (OP == OP_FUSED1S);
    constexpr bool kTwo = (OP == OP_SPMM2 || OP == OP_FUSED2);

    // A line without entries needs no held row (its outputs are zeros), except a CG step,
    // whose update uses the direction itself; skipping the load saves a row read per empty
    // line (half the lines of an R-MAT pattern).
    const bool want_held = OP == OP_CG || begin < end;
    Acc h[E];
    if constexpr (kHeld) {
        const TH *__restrict__ Hrow = static_cast<const TH *>(o.H) + (size_t)line * r;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (act[v] && want_held) {
                Ld<TH, VW, Acc>::template run<kNtHeld>(Hrow + off[v], h + v * VW);
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e) h[v * VW + e] = Acc(0);
            }
        }
    }

    Acc h2[kHeld2 ? E : 1];
    if constexpr (kHeld2) {
        const TG2 *__restrict__ H2row = static_cast<const TG2 *>(o.H2) + (size_t)line * r;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (act[v] && want_held) {
                Ld<TG2, VW, Acc>::template run<kNtHeld>(H2row + off[v], h2 + v * VW);
            } else {
#pragma unroll
                for (int e = 0; e < VW; ++e) h2[v * VW + e] = Acc(0);
            }
        }
    }

    // A dot product of two bfloat16 vectors takes the bf16 dot instruction on packed words
    // (dot2_bf16), so the held rows it uses are kept packed as well; packing the widened
    // values back is exact.  Dot products with a float32 operand stay FMA chains.
    constexpr bool kF32 = std::is_same<Acc, float>::value && VW == 8;
    constexpr bool kDotH = kF32 && std::is_same<TH, bf16_t>::value && std::is_same<TG1, bf16_t>::value;  // <H, G1>
    constexpr bool kDotHG2 = kF32 && OP == OP_FUSED2 && std::is_same<TH, bf16_t>::value &&
                             std::is_same<TG2, bf16_t>::value;                                             // <H, G2>
    constexpr bool kDotH2 = kF32 && kHeld2 && std::is_same<TG2, bf16_t>::value &&
                            std::is_same<TG1, bf16_t>::value;                                              // <H2, G1>
    constexpr int PW = VW / 2;  // packed words per vector
    uint32_t hp[(kDotH || kDotHG2) ? NV * PW : 1];
    if constexpr (kDotH || kDotHG2) {
#pragma unroll
        for (int k = 0; k < NV * PW; ++k) hp[k] = bf16_pack_exact(h[2 * k], h[2 * k + 1]);
    }
    uint32_t h2p[kDotH2 ? NV * PW : 1];
    if constexpr (kDotH2) {
#pragma unroll
        for (int k = 0; k < NV * PW; ++k) h2p[k] = bf16_pack_exact(h2[2 * k], h2[2 * k + 1]);
    }

    Acc acc[E];
#pragma unroll
    for (int e = 0; e < E; ++e) acc[e] = Acc(0);

    // Branch-free operand access: a NULL weight array is read as a single 1 (stride 0)
    // and a NULL permutation as a single 0 plus the identity, so a full batch issues all
    // of its loads back to back, with no wait in between.
    const Acc *val_p = val ? val : unit_value<Acc>();
    const int32_t vs = val ? 1 : 0;
    const Acc *wv1_p = wv1 ? wv1 : unit_value<Acc>();
    const int32_t w1s = wv1 ? 1 : 0;
    const Acc *wv2_p = wv2 ? wv2 : unit_value<Acc>();
    const int32_t w2s = wv2 ? 1 : 0;
    const int32_t *perm_p = wperm ? wperm : zero_index();
    const int32_t ps = wperm ? 1 : 0;
    const uint8_t *hot_p = o.hot ? o.hot : kHotByte;
    const int32_t hs = o.hot ? 1 : 0;
    const bool partial = C < L * NV;  // some lanes own no vector of r (uniform)

    // Per-entry operands of one batch (column indices and weights).  Entries past `end`
    // read the last entry of the line, so every load is in bounds.
    auto load_meta = [&](int32_t p0, auto full_tag, int32_t *j, Acc *w1, Acc *w2, uint32_t *hv) {
        constexpr bool FULL = decltype(full_tag)::value;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int32_t p = p0 + u;
            const int32_t pc = (FULL || p < end) ? p : end - 1;
            j[u] = ld_hint<kNtMeta>(idx + pc);
            hv[u] = hot_p[pc * hs];
            const Acc base = ld_hint<kNtMeta>(val_p + pc * vs);
            if constexpr (OP == OP_SPMM1 || OP == OP_SPMM2) {
                const int32_t q = perm_p[pc * ps] + pc * (1 - ps);
                w1[u] = base * wv1_p[q * w1s];
                w2[u] = (OP == OP_SPMM2) ? base * wv2_p[q * w2s] : Acc(0);
            } else {
                w1[u] = base;
                w2[u] = Acc(0);
            }
        }
    };

    // One batch of U entries from p0 with operands (j, w1, w2): already loaded with PF,
    // else loaded here first.  FULL: all U entries lie in the line.  Otherwise the entries past `end` load no row
    // and are left out of every sum and store.  Their row registers are left as they are,
    // not zeroed: a zero write to a register that an in-flight load targets would force a
    // wait for that load, serialising the batch.  After the row loads are issued, the
    // operands of the batch at `pn` are loaded into (jn, w1n, w2n), so that they arrive
    // while this batch waits for its rows (PF; the batched persistent kernel, whose rows
    // are mostly L2 hits, runs faster without it).
    auto run_batch = [&](int32_t p0, auto full_tag, int32_t *j, Acc *w1, Acc *w2, uint32_t *hv, int32_t pn,
                         int32_t *jn, Acc *w1n, Acc *w2n, uint32_t *hvn) {
        constexpr bool FULL = decltype(full_tag)::value;
        if constexpr (!PF) load_meta(p0, full_tag, j, w1, w2, hv);
        bool okv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) okv[u] = FULL || p0 + u < end;
        Raw<TG1, VW> g1[U][NV];
        Raw<TG2, VW> g2[kTwo ? U : 1][kTwo ? NV : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const TG1 *row1 = G1 + (size_t)j[u] * r;
            const TG2 *row2 = G2 + (size_t)j[u] * r;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int o = act[v] ? off[v] : 0;  // idle lanes read a valid spot, zeroed below
                if (FULL || okv[u]) {
                    if (hv[u]) {
                        g1[u][v].load(row1 + o);
                        if constexpr (kTwo) g2[u][v].load(row2 + o);
                    } else {
                        g1[u][v].load_nt(row1 + o);
                        if constexpr (kTwo) g2[u][v].load_nt(row2 + o);
                    }
                }
            }
        }
        if constexpr (PF) {
            if (pn < end) load_meta(pn, std::false_type{}, jn, w1n, w2n, hvn);  // one clamped form: no divergence
        }
        if (partial) {
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    if (!act[v]) {
                        g1[u][v].zero();
                        if constexpr (kTwo) g2[u][v].zero();
                    }
        }

        if constexpr (OP == OP_SPMM1 || OP == OP_SPMM2) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!FULL && !okv[u]) continue;
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int e = 0; e < VW; ++e) {
                        if constexpr (OP == OP_SPMM2)
                            acc[v * VW + e] = fmadd(w2[u], Acc(g2[u][v].get(e)),
                                                    fmadd(w1[u], Acc(g1[u][v].get(e)), acc[v * VW + e]));
                        else
                            acc[v * VW + e] = fmadd(w1[u], Acc(g1[u][v].get(e)), acc[v * VW + e]);
                    }
            }
        } else if constexpr (OP == OP_FUSED2) {
            Acc d1[U], d2[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                Acc s1 = Acc(0), s2 = Acc(0);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if constexpr (kDotHG2) {
#pragma unroll
                        for (int k = 0; k < PW; ++k) s1 = dot2_bf16(hp[v * PW + k], g2[u][v].word(k), s1);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e) s1 = fmadd(h[v * VW + e], Acc(g2[u][v].get(e)), s1);
                    }
                    if constexpr (kDotH) {
#pragma unroll
                        for (int k = 0; k < PW; ++k) s2 = dot2_bf16(hp[v * PW + k], g1[u][v].word(k), s2);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e) s2 = fmadd(h[v * VW + e], Acc(g1[u][v].get(e)), s2);
                    }
                }
                d1[u] = s1;
                d2[u] = s2;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                d1[u] = group_sum<L>(d1[u]);
                d2[u] = group_sum<L>(d2[u]);
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    g1[u][v].pin();
                    g2[u][v].pin();
                }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!FULL && !okv[u]) continue;
                const Acc c1 = w1[u] * d1[u], c2 = w1[u] * d2[u];
#pragma unroll
                for (int v = 0; v < NV; ++v)
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        acc[v * VW + e] = fmadd(c2, Acc(g2[u][v].get(e)),
                                                fmadd(c1, Acc(g1[u][v].get(e)), acc[v * VW + e]));
            }
        } else {
            Acc d[U], dv[kHeld2 ? U : 1];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                Acc s = Acc(0), s2 = Acc(0);
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if constexpr (kDotH) {
#pragma unroll
                        for (int k = 0; k < PW; ++k) s = dot2_bf16(hp[v * PW + k], g1[u][v].word(k), s);
                    } else {
#pragma unroll
                        for (int e = 0; e < VW; ++e) s = fmadd(h[v * VW + e], Acc(g1[u][v].get(e)), s);
                    }
                    if constexpr (kDotH2) {
#pragma unroll
                        for (int k = 0; k < PW; ++k) s2 = dot2_bf16(h2p[v * PW + k], g1[u][v].word(k), s2);
                    } else if constexpr (kHeld2) {
#pragma unroll
                        for (int e = 0; e < VW; ++e) s2 = fmadd(h2[v * VW + e], Acc(g1[u][v].get(e)), s2);
                    }
                }
                d[u] = s;
                if constexpr (kHeld2) dv[u] = s2;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                d[u] = group_sum<L>(d[u]);
                if constexpr (kHeld2) dv[u] = group_sum<L>(dv[u]);
            }
            if constexpr (kHeld2) {  // V[p] = <H, G1_j> <H2, G1_j>
                Acc *V = static_cast<Acc *>(o.R);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t p = p0 + u;
                    if (lane == (u % L) && okv[u]) V[o.operm ? o.operm[p] : p] = d[u] * dv[u];
                }
            }
            if constexpr (OP == OP_SDDMM) {
                Acc *R = static_cast<Acc *>(o.R);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int32_t p = p0 + u;
                    if (lane == (u % L) && okv[u]) {
                        const Acc res = w1[u] * d[u];
                        const int64_t q = o.operm ? o.operm[p] : p;
                        R[q] = (o.beta == 0.0) ? res : Acc(o.beta) * R[q] + res;
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int v = 0; v < NV; ++v) g1[u][v].pin();
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (!FULL && !okv[u]) continue;
                    const Acc c = w1[u] * d[u];
#pragma unroll
                    for (int v = 0; v < NV; ++v)
#pragma unroll
                        for (int e = 0; e < VW; ++e) acc[v * VW + e] = fmadd(c, Acc(g1[u][v].get(e)), acc[v * VW + e]);
                }
            }
        }
    };

    {
        int32_t j[U], jn[U];
        Acc w1[U], w2[U], w1n[U], w2n[U];
        uint32_t hv[U], hvn[U];
        int32_t p0 = begin + gidx * U;
        if constexpr (PF) {
            if (p0 < end) load_meta(p0, std::false_type{}, j, w1, w2, hv);
        }
        for (; p0 < end; p0 += U * GPL) {
            const int32_t pn = p0 + U * GPL;
            if (p0 + U <= end) run_batch(p0, std::true_type{}, j, w1, w2, hv, pn, jn, w1n, w2n, hvn);
            else run_batch(p0, std::false_type{}, j, w1, w2, hv, pn, jn, w1n, w2n, hvn);
            if constexpr (PF) {
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    j[u] = jn[u];
                    w1[u] = w1n[u];
                    w2[u] = w2n[u];
                    hv[u] = hvn[u];
                }
            }
        }
    }

    if constexpr (OP == OP_CG) {
        static_assert(GPL == 1, "a CG step needs the whole line in one group");
        cg_line_step<L, NV, VW>(o, line, lane, act, off, h, acc);
        return;
    }
    if constexpr (OP != OP_SDDMM) {
        if (dst == nullptr) return;  // OP_FUSED1S without the row output
        if constexpr (GPL > 1) {
#pragma unroll
            for (int e = 0; e < E; ++e) acc[e] = cross_group_sum<L, GPL>(acc[e]);
            if (gidx != 0) return;
        }
        const Acc beta = Acc(o.beta);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (act[v]) {
                Acc outv[VW];
                if (keep_beta) {
                    Ld<Acc, VW, Acc>::run(dst + off[v], outv);
#pragma unroll
                    for (int e = 0; e < VW; ++e) outv[e] = beta * outv[e] + acc[v * VW + e];
                } else {
#pragma unroll
                    for (int e = 0; e < VW; ++e) outv[e] = acc[v * VW + e];
                }
                St<Acc, VW>::template run<kNtStore>(dst + off[v], outv);
            }
        }
    }
}

// ------------------------------------------------------------------ the line kernel

template <int OP, class TH, class TG1, class TG2, class Acc, int L, int NV, int VW, int U>
__global__ __launch_bounds__(kBlock) void line_kernel(LineArgs a, int32_t nb_chunk_blocks)
{
    constexpr int GPB = kBlock / L;  // groups per block
    const int lane = threadIdx.x % L;
    const int gib = threadIdx.x / L;
    const int r = a.r;

    int32_t line, begin, end;
    Acc *dst = nullptr;
    bool to_partial = false;
    if ((int32_t)blockIdx.x < nb_chunk_blocks) {
        const int32_t c = blockIdx.x * GPB + gib;
        if (c >= a.n_chunks) return;
        line = a.chunks[3 * c];
        begin = a.chunks[3 * c + 1];
        end = a.chunks[3 * c + 2];
        if (OP != OP_SDDMM && a.out) dst = static_cast<Acc *>(a.partial) + (size_t)c * r;
        to_partial = true;
    } else {
        const int32_t k = (blockIdx.x - nb_chunk_blocks) * GPB + gib;
        if (k >= a.nlines) return;
        line = a.order ? a.order[k] : k;
        begin = a.ptr[line];
        end = a.ptr[line + 1];
        if (a.n_chunks > 0 && end - begin > a.long_len) return;
        if (OP != OP_SDDMM && a.out) dst = static_cast<Acc *>(a.out) + (size_t)line * r;
    }
    LineOperands o;
    o.idx = a.idx;
    o.val = a.val;
    o.wv1 = a.wv1;
    o.wv2 = a.wv2;
    o.wperm = a.wperm;
    o.operm = a.operm;
    o.H = a.H;
    o.G1 = a.G1;
    o.G2 = a.G2;
    o.H2 = a.H2;
    o.hot = a.hot;
    o.R = OP == OP_FUSED1S ? a.values : a.out;
    o.cg_X = a.cg_X;
    o.cg_R = a.cg_R;
    o.cg_P = a.cg_P;
    o.cg_rr = a.cg_rr;
    o.cg_lambda = a.cg_lambda;
    o.r = r;
    o.beta = a.beta;
    process_line<OP, TH, TG1, TG2, Acc, L, NV, VW, U, 1>(o, lane, 0, line, begin, end, dst,
                                                         !to_partial && a.beta != 0.0);
}

// Sum the chunk partials of every split line, in chunk order, into its output row:
// out[line] = beta * out[line] + sum_c partial[first + c].
template <class Acc>
__global__ __launch_bounds__(kBlock) void merge_kernel(const int32_t *__restrict__ splits,
                                                       int32_t n_splits, int32_t r,
                                                       const Acc *__restrict__ partial,
                                                       Acc *__restrict__ out, double beta)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= (int64_t)n_splits * r) return;
    const int32_t s = (int32_t)(t / r);
    const int32_t k = (int32_t)(t % r);
    const int32_t line = splits[3 * s], first = splits[3 * s + 1], cnt = splits[3 * s + 2];
    const Acc *p = partial + (size_t)first * r + k;
    Acc sum = Acc(0);
    int32_t c = 0;
    // eight loads in flight, added in chunk order
    for (; c + 8 <= cnt; c += 8) {
        Acc v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = p[(size_t)(c + u) * r];
#pragma unroll
        for (int u = 0; u < 8; ++u) sum += v[u];
    }
    for (; c < cnt; ++c) sum += p[(size_t)c * r];
    Acc *o = out + (size_t)line * r + k;
    *o = (beta == 0.0) ? sum : Acc(beta) * *o + sum;
}

}  // namespace fmm
