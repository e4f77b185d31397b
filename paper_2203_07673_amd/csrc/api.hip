// C ABI of the local FusedMM library: argument checks, workspace rules and the
// mapping of every public call onto line-kernel launches.  See include/fmm.h for
// the contract of each entry point.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <vector>

#include "fmm.h"
#include "fmm_internal.hpp"

namespace fmm {

static thread_local int32_t g_last_hip_error = 0;
void set_last_hip_error(int32_t e) { g_last_hip_error = e; }

static Tuning g_tuning = {0, 0};
Tuning &tuning() { return g_tuning; }

static bool is_compiled_shape(int L, int NV)
{
    switch (NV) {
    case 1: return L == 1 || L == 2 || L == 4 || L == 8 || L == 16 || L == 32 || L == 64;
    case 2: return L == 16 || L == 32 || L == 64;
    case 4: return L == 64;
    default: return false;
    }
}

bool shape_supported(Shape s, int r, int vw)
{
    if (!is_compiled_shape(s.L, s.NV)) return false;
    const int C = r / vw;  // vectors per r-vector
    return s.L * s.NV >= C;  // the group's vectors cover r (surplus lanes are masked)
}

Shape default_shape(int r, int vw)
{
    const int C = r / vw;
    int L = 1;
    while (L < C && L < 64) L <<= 1;
    int NV = (C + L - 1) / L;
    if (NV == 3) NV = 4;
    return Shape{L, NV};
}

}  // namespace fmm

using namespace fmm;

namespace {

struct Kinds {
    int path;      // PATH_*
    size_t sbytes; // storage element size of A/B
    size_t obytes; // element size of S values, dC and outputs
};

fmm_status kinds_for(int32_t dtype, int32_t r, Kinds *k)
{
    switch (dtype) {
    case FMM_F32:
        *k = Kinds{PATH_F32, 4, 4};
        if (r < 1 || (r % 4 == 0 ? r > 1024 : r > 256)) return FMM_ERR_DTYPE;
        return FMM_OK;
    case FMM_BF16:
        *k = Kinds{PATH_BF16, 2, 4};
        if (r < 8 || r % 8 != 0 || r > 1024) return FMM_ERR_DTYPE;
        return FMM_OK;
    case FMM_F64:
        *k = Kinds{PATH_F64, 8, 8};
        if (r < 1 || (r % 2 == 0 ? r > 512 : r > 256)) return FMM_ERR_DTYPE;
        return FMM_OK;
    default:
        return FMM_ERR_DTYPE;
    }
}

fmm_status hip_status(hipError_t e)
{
    if (e == hipSuccess) return FMM_OK;
    g_last_hip_error = (int32_t)e;
    return FMM_ERR_HIP;
}

// Vector loads need 16-byte aligned rows; rows are r elements apart.
bool aligned_ok(const void *p, size_t elem, int32_t r)
{
    if (((size_t)r * elem) % 16 != 0) return true;  // scalar path
    return ((uintptr_t)p % 16) == 0;
}

fmm_status check_sparse(const fmm_sparse *S, int orient)
{
    if (!S) return FMM_ERR_NULL;
    if (S->orient != FMM_CSR && S->orient != FMM_CSC) return FMM_ERR_ORIENT;
    if (orient >= 0 && S->orient != orient) return FMM_ERR_ORIENT;
    if (S->rows < 0 || S->cols < 0 || S->nnz < 0) return FMM_ERR_DIM;
    if (!S->ptr) return FMM_ERR_NULL;
    if (S->nnz > 0 && !S->idx) return FMM_ERR_NULL;
    if (S->n_chunks < 0 || S->n_splits < 0) return FMM_ERR_DIM;
    if (S->variant < FMM_VARIANT_AUTO || S->variant > FMM_VARIANT_SHALLOW) return FMM_ERR_DIM;
    if (S->n_chunks > 0) {
        if (!S->chunks || !S->splits) return FMM_ERR_NULL;
        if (S->long_len < 1 || S->n_splits < 1) return FMM_ERR_DIM;
    }
    return FMM_OK;
}

inline int32_t nmajor(const fmm_sparse *S) { return S->orient == FMM_CSR ? S->rows : S->cols; }
inline int32_t nminor(const fmm_sparse *S) { return S->orient == FMM_CSR ? S->cols : S->rows; }

size_t partial_bytes(const fmm_sparse *S, int32_t r, size_t obytes)
{
    return (S && S->n_chunks > 0) ? (size_t)S->n_chunks * (size_t)r * obytes : 0;
}

fmm_status check_ws(const fmm_sparse *S, int32_t r, size_t obytes, void *ws, size_t ws_bytes)
{
    const size_t need = partial_bytes(S, r, obytes);
    if (need == 0) return FMM_OK;
    if (!ws || ws_bytes < need) return FMM_ERR_WORKSPACE;
    if ((uintptr_t)ws % 16 != 0) return FMM_ERR_WORKSPACE;
    return FMM_OK;
}

// Batch depth class of a descriptor: its explicit variant, else by mean line length.
int32_t unroll_class(const fmm_sparse *S)
{
    if (S->variant >= FMM_VARIANT_DEEP && S->variant <= FMM_VARIANT_SHALLOW) return S->variant;
    const int64_t lines = S->orient == FMM_CSR ? S->rows : S->cols;
    const double mean = lines > 0 ? (double)S->nnz / (double)lines : 0.0;
    return mean >= 24.0 ? FMM_VARIANT_DEEP : mean >= 6.0 ? FMM_VARIANT_MEDIUM : FMM_VARIANT_SHALLOW;
}

LineArgs base_args(const fmm_sparse *S, int32_t r, void *ws)
{
    LineArgs a;
    memset(&a, 0, sizeof(a));
    a.uclass = unroll_class(S);
    a.nlines = nmajor(S);
    a.r = r;
    a.ptr = S->ptr;
    a.idx = S->idx;
    a.val = S->val;
    a.long_len = S->long_len;
    a.n_chunks = S->n_chunks;
    a.chunks = S->chunks;
    a.order = S->order;
    a.hot = S->hot;
    a.partial = ws;
    a.beta = 0.0;
    return a;
}

Shape hint() { return Shape{tuning().lanes, tuning().nv}; }

// Operand kinds of the bfloat16 path: 'S' = storage (bfloat16), 'O' = float32.
template <int OP>
hipError_t run(int path, char hk, char g1k, char g2k, const LineArgs &a, const fmm_sparse *S, hipStream_t st)
{
    const int32_t ns = S->n_chunks > 0 ? S->n_splits : 0;
    const int32_t *sp = S->splits;
    if (path == PATH_F32) return launch_lines<OP, float, float, float, float>(a, ns, sp, hint(), st);
    if (path == PATH_F64) return launch_lines<OP, double, double, double, double>(a, ns, sp, hint(), st);
    typedef bf16_t Sb;
    typedef float Of;
    if constexpr (OP == OP_SDDMM) {
        if (hk == 'S' && g1k == 'S') return launch_lines<OP, Sb, Sb, Sb, float>(a, ns, sp, hint(), st);
        if (hk == 'O' && g1k == 'S') return launch_lines<OP, Of, Sb, Sb, float>(a, ns, sp, hint(), st);
        if (hk == 'S' && g1k == 'O') return launch_lines<OP, Sb, Of, Of, float>(a, ns, sp, hint(), st);
    } else if constexpr (OP == OP_SPMM1) {
        if (g1k == 'S') return launch_lines<OP, Sb, Sb, Sb, float>(a, ns, sp, hint(), st);
        if (g1k == 'O') return launch_lines<OP, Of, Of, Of, float>(a, ns, sp, hint(), st);
    } else if constexpr (OP == OP_SPMM2) {
        if (g1k == 'S' && g2k == 'O') return launch_lines<OP, Sb, Sb, Of, float>(a, ns, sp, hint(), st);
    } else if constexpr (OP == OP_FUSED1) {
        if (hk == 'S' && g1k == 'S') return launch_lines<OP, Sb, Sb, Sb, float>(a, ns, sp, hint(), st);
        if (hk == 'O' && g1k == 'S') return launch_lines<OP, Of, Sb, Sb, float>(a, ns, sp, hint(), st);
    } else if constexpr (OP == OP_FUSED2) {
        if (hk == 'S' && g1k == 'S' && g2k == 'O') return launch_lines<OP, Sb, Sb, Of, float>(a, ns, sp, hint(), st);
        if (hk == 'S' && g1k == 'S' && g2k == 'S') return launch_lines<OP, Sb, Sb, Sb, float>(a, ns, sp, hint(), st);
    } else if constexpr (OP == OP_FUSED1S) {  // g2k: kind of the second held row
        if (hk == 'O' && g1k == 'S' && g2k == 'S') return launch_lines<OP, Of, Sb, Sb, float>(a, ns, sp, hint(), st);
    }
    (void)g2k;
    return hipErrorInvalidValue;
}

#define FMM_TRY(x)                                                                               \
    do {                                                                                         \
        fmm_status _s = (x);                                                                     \
        if (_s != FMM_OK) return _s;                                                             \
    } while (0)

#define FMM_HIP(x)                                                                               \
    do {                                                                                         \
        hipError_t _e = (x);                                                                     \
        if (_e != hipSuccess) return hip_status(_e);                                             \
    } while (0)

fmm_status check_dense(const void *p, int64_t rows, size_t elem, int32_t r)
{
    if (rows > 0 && !p) return FMM_ERR_NULL;
    if (rows > 0 && !aligned_ok(p, elem, r)) return FMM_ERR_UNSUPPORTED;
    return FMM_OK;
}

fmm_status check_pair(const fmm_sparse *S_csr, const fmm_sparse *S_csc)
{
    FMM_TRY(check_sparse(S_csr, FMM_CSR));
    FMM_TRY(check_sparse(S_csc, FMM_CSC));
    if (S_csr->rows != S_csc->rows || S_csr->cols != S_csc->cols || S_csr->nnz != S_csc->nnz) return FMM_ERR_DIM;
    return FMM_OK;
}

size_t max_partial(const fmm_sparse *a, const fmm_sparse *b, int32_t r, size_t obytes)
{
    size_t x = partial_bytes(a, r, obytes), y = partial_bytes(b, r, obytes);
    return x > y ? x : y;
}

fmm_status check_ws2(const fmm_sparse *a, const fmm_sparse *b, int32_t r, size_t obytes, void *ws, size_t ws_bytes)
{
    const size_t need = max_partial(a, b, r, obytes);
    if (need == 0) return FMM_OK;
    if (!ws || ws_bytes < need || (uintptr_t)ws % 16 != 0) return FMM_ERR_WORKSPACE;
    return FMM_OK;
}

// dS = P * <X_i, Y_j> on S_csr in two SDDMM passes: P = <A_i, B_j> into dS, then
// dS[p] *= <X_i, Y_j> in place (each entry is read and written by the same lane group).
fmm_status values_unfused(const fmm_sparse *S_csr, const Kinds &k, const void *A, const void *B, char xk,
                                 const void *X, char yk, const void *Y, int32_t r, void *dS, hipStream_t stream)
{
    fmm_sparse Sx = *S_csr;
    Sx.n_splits = 0;
    LineArgs s = base_args(S_csr, r, nullptr);
    s.val = nullptr;
    s.H = A;
    s.G1 = B;
    s.out = dS;
    FMM_HIP(run<OP_SDDMM>(k.path, 'S', 'S', 'S', s, &Sx, stream));
    LineArgs t = base_args(S_csr, r, nullptr);
    t.val = dS;
    t.H = X;
    t.G1 = Y;
    t.out = dS;
    FMM_HIP(run<OP_SDDMM>(k.path, xk, yk, yk, t, &Sx, stream));
    return FMM_OK;
}

}  // namespace

// ---------------------------------------------------------------- internal helpers

namespace fmm {
// out_line = sum over the line's stored entries of <H_line, G_j> G_j, with S's values
// ignored (the pattern alone): the matrix-free product of the per-line Gram operator
// used by batched conjugate gradients.  H and out are float32; G has storage dtype.
fmm_status gram_apply(const fmm_sparse *S, const float *H, const void *G, int32_t r, int32_t dtype, float *out,
                      void *ws, size_t ws_bytes, hipStream_t st)
{
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    if (k.path == PATH_F64) return FMM_ERR_DTYPE;
    FMM_TRY(check_ws(S, r, k.obytes, ws, ws_bytes));
    LineArgs a = base_args(S, r, ws);
    a.val = nullptr;
    a.H = H;
    a.G1 = G;
    a.out = out;
    FMM_HIP(run<OP_FUSED1>(k.path, 'O', 'S', 'S', a, S, st));
    return FMM_OK;
}
// One batched CG step for every line of S fused with the Gram pass (OP_CG): the line's
// q = sum_j <P_line, G_j> G_j stays in registers and updates X, R, P and rr in place.
// S must carry no split schedule (a split line's q is only complete after its merge).
fmm_status gram_cg_step(const fmm_sparse *S, float *P, const void *G, int32_t r, int32_t dtype, float lambda,
                        float *X, float *R, float *rr, hipStream_t st)
{
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    if (S->n_chunks > 0) return FMM_ERR_UNSUPPORTED;
    LineArgs a = base_args(S, r, nullptr);
    a.val = nullptr;
    a.H = P;
    a.G1 = G;
    a.out = nullptr;
    a.cg_X = X;
    a.cg_R = R;
    a.cg_P = P;
    a.cg_rr = rr;
    a.cg_lambda = lambda;
    hipError_t e;
    if (dtype == FMM_F32) e = launch_lines<OP_CG, float, float, float, float>(a, 0, nullptr, hint(), st);
    else if (dtype == FMM_BF16) e = launch_lines<OP_CG, float, bf16_t, bf16_t, float>(a, 0, nullptr, hint(), st);
    else return FMM_ERR_DTYPE;
    FMM_HIP(e);
    return FMM_OK;
}
}  // namespace fmm

extern "C" {

int32_t fmm_abi_version(void) { return FMM_ABI_VERSION; }

const char *fmm_status_string(int32_t status)
{
    switch (status) {
    case FMM_OK: return "ok";
    case FMM_ERR_NULL: return "required pointer is NULL";
    case FMM_ERR_DIM: return "invalid or inconsistent size";
    case FMM_ERR_DTYPE: return "unsupported dtype or dtype/r combination";
    case FMM_ERR_ORIENT: return "sparse descriptor has the wrong orientation";
    case FMM_ERR_INDEX: return "index out of range or malformed pointer array";
    case FMM_ERR_NONCANONICAL: return "minor indices not strictly increasing within a line";
    case FMM_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case FMM_ERR_UNSUPPORTED: return "unsupported request (alignment or size limit)";
    case FMM_ERR_HIP: return "HIP runtime error";
    case FMM_ERR_STATE: return "batch plan has no current captured graph";
    default: return "unknown status";
    }
}

int32_t fmm_last_hip_error(void) { return g_last_hip_error; }

fmm_status fmm_device_info(int32_t *num_cu, char *arch, int32_t arch_len)
{
    int dev = 0;
    FMM_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FMM_HIP(hipGetDeviceProperties(&prop, dev));
    if (num_cu) *num_cu = prop.multiProcessorCount;
    if (arch && arch_len > 0) {
        strncpy(arch, prop.gcnArchName, (size_t)arch_len - 1);
        arch[arch_len - 1] = 0;
    }
    return FMM_OK;
}

fmm_status fmm_set_tuning(int32_t lanes, int32_t nv)
{
    if (lanes < 0 || nv < 0) return FMM_ERR_DIM;
    if ((lanes == 0) != (nv == 0)) return FMM_ERR_DIM;
    if (lanes != 0 && !is_compiled_shape(lanes, nv)) return FMM_ERR_UNSUPPORTED;
    tuning().lanes = lanes;
    tuning().nv = nv;
    return FMM_OK;
}

// ---------------------------------------------------------------- pattern prep

fmm_status fmm_validate(const fmm_sparse *S, hipStream_t stream)
{
    FMM_TRY(check_sparse(S, -1));
    int32_t *flag = nullptr;
    FMM_HIP(hipMalloc(&flag, 4));
    hipError_t e = hipMemsetAsync(flag, 0, 4, stream);
    if (e == hipSuccess) e = validate(nmajor(S), nminor(S), S->nnz, S->ptr, S->idx, flag, stream);
    int32_t f = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&f, flag, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    hipError_t e2 = hipFree(flag);
    if (e != hipSuccess) return hip_status(e);
    if (e2 != hipSuccess) return hip_status(e2);
    if (f & 1) return FMM_ERR_INDEX;
    if (f & 2) return FMM_ERR_NONCANONICAL;
    return FMM_OK;
}

fmm_status fmm_csr_to_csc_workspace(int32_t m, int32_t n, int32_t nnz, size_t *bytes)
{
    if (!bytes) return FMM_ERR_NULL;
    if (m < 0 || n < 0 || nnz < 0) return FMM_ERR_DIM;
    *bytes = transpose_workspace_bytes(m, n, nnz);
    return FMM_OK;
}

fmm_status fmm_csr_to_csc(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colidx,
                          const void *val, int32_t val_dtype, int32_t *colptr, int32_t *rowidx, void *valT,
                          int32_t *perm, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (m < 0 || n < 0 || nnz < 0) return FMM_ERR_DIM;
    if (!rowptr || !colptr) return FMM_ERR_NULL;
    if (nnz > 0 && (!colidx || !rowidx || !perm)) return FMM_ERR_NULL;
    if (val && val_dtype != FMM_F32 && val_dtype != FMM_F64) return FMM_ERR_DTYPE;
    if (nnz > 0 && m == 0) return FMM_ERR_DIM;
    if (!ws || ws_bytes < transpose_workspace_bytes(m, n, nnz)) return FMM_ERR_WORKSPACE;
    if ((uintptr_t)ws % 16 != 0) return FMM_ERR_WORKSPACE;
    FMM_HIP(csr_to_csc(m, n, nnz, rowptr, colidx, val, val_dtype == FMM_F64 ? 8 : 4, colptr, rowidx, valT, perm, ws,
                       stream));
    return FMM_OK;
}

fmm_status fmm_gather_values(const int32_t *perm, const void *src, int32_t val_dtype, void *dst, int32_t nnz,
                             hipStream_t stream)
{
    if (nnz < 0) return FMM_ERR_DIM;
    if (val_dtype != FMM_F32 && val_dtype != FMM_F64) return FMM_ERR_DTYPE;
    if (nnz == 0) return FMM_OK;
    if (!perm || !src || !dst) return FMM_ERR_NULL;
    FMM_HIP(gather_values(perm, src, dst, nnz, val_dtype == FMM_F64 ? 8 : 4, stream));
    return FMM_OK;
}

fmm_status fmm_line_order_workspace(int32_t nlines, size_t *bytes)
{
    if (!bytes) return FMM_ERR_NULL;
    if (nlines < 0) return FMM_ERR_DIM;
    *bytes = line_order_workspace_bytes(nlines);
    return FMM_OK;
}

fmm_status fmm_line_order(const int32_t *ptr, int32_t nlines, int32_t long_len, int32_t *order, void *ws,
                          size_t ws_bytes, hipStream_t stream)
{
    if (nlines < 0 || long_len < 1) return FMM_ERR_DIM;
    if (nlines == 0) return FMM_OK;
    if (!ptr || !order) return FMM_ERR_NULL;
    if (!ws || ws_bytes < line_order_workspace_bytes(nlines) || (uintptr_t)ws % 16 != 0) return FMM_ERR_WORKSPACE;
    FMM_HIP(line_order(ptr, nlines, long_len, order, ws, stream));
    return FMM_OK;
}

fmm_status fmm_gather_hints(const fmm_sparse *S, const int32_t *minor_ptr, int32_t n_minor, int32_t top,
                            uint8_t *hot, hipStream_t stream)
{
    FMM_TRY(check_sparse(S, -1));
    const int32_t minor = S->orient == FMM_CSR ? S->cols : S->rows;
    if (n_minor != minor) return FMM_ERR_DIM;
    if (S->nnz == 0) return FMM_OK;
    if (!minor_ptr || !hot) return FMM_ERR_NULL;
    // the length of the top-th longest minor line is the threshold (0: every line is hot)
    int32_t min_len = 0;
    if (top <= 0) {
        min_len = INT32_MAX;
    } else if (top < n_minor) {
        std::vector<int32_t> ptr((size_t)n_minor + 1);
        FMM_HIP(hipMemcpyAsync(ptr.data(), minor_ptr, ptr.size() * sizeof(int32_t), hipMemcpyDeviceToHost, stream));
        FMM_HIP(hipStreamSynchronize(stream));
        std::vector<int32_t> len((size_t)n_minor);
        for (int32_t j = 0; j < n_minor; ++j) len[j] = ptr[j + 1] - ptr[j];
        std::nth_element(len.begin(), len.begin() + (top - 1), len.end(), std::greater<int32_t>());
        min_len = std::max<int32_t>(1, len[top - 1]);
    }
    FMM_HIP(gather_hints(S->idx, minor_ptr, S->nnz, min_len, hot, stream));
    FMM_HIP(hipStreamSynchronize(stream));
    return FMM_OK;
}

fmm_status fmm_schedule_workspace(int32_t nmaj, size_t *bytes)
{
    if (!bytes) return FMM_ERR_NULL;
    if (nmaj < 0) return FMM_ERR_DIM;
    *bytes = schedule_workspace_bytes(nmaj);
    return FMM_OK;
}

fmm_status fmm_schedule_count(const int32_t *ptr, int32_t nmaj, int32_t long_len, int32_t chunk, int32_t *n_chunks,
                              int32_t *n_splits, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!ptr || !n_chunks || !n_splits) return FMM_ERR_NULL;
    if (nmaj < 0 || chunk < 1 || long_len < chunk) return FMM_ERR_DIM;
    if (!ws || ws_bytes < schedule_workspace_bytes(nmaj) || (uintptr_t)ws % 16 != 0) return FMM_ERR_WORKSPACE;
    int32_t totals[2] = {0, 0};
    FMM_HIP(schedule_count(ptr, nmaj, long_len, chunk, totals, ws, stream));
    *n_chunks = totals[0];
    *n_splits = totals[1];
    return FMM_OK;
}

fmm_status fmm_schedule_fill(const int32_t *ptr, int32_t nmaj, int32_t long_len, int32_t chunk, int32_t *chunks,
                             int32_t *splits, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!ptr || !chunks || !splits) return FMM_ERR_NULL;
    if (nmaj < 0 || chunk < 1 || long_len < chunk) return FMM_ERR_DIM;
    if (!ws || ws_bytes < schedule_workspace_bytes(nmaj) || (uintptr_t)ws % 16 != 0) return FMM_ERR_WORKSPACE;
    FMM_HIP(schedule_fill(ptr, nmaj, long_len, chunk, chunks, splits, ws, stream));
    return FMM_OK;
}

fmm_status fmm_f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t stream)
{
    if (n < 0) return FMM_ERR_DIM;
    if (n > 0 && (!x || !y)) return FMM_ERR_NULL;
    FMM_HIP(f32_to_bf16(x, y, n, stream));
    return FMM_OK;
}

fmm_status fmm_workspace_size(int32_t op, const fmm_sparse *S_csr, const fmm_sparse *S_csc, int32_t r, int32_t dtype,
                              size_t *bytes)
{
    if (!bytes) return FMM_ERR_NULL;
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    switch (op) {
    case FMM_OP_SDDMM: *bytes = 0; return FMM_OK;
    case FMM_OP_SPMM_A:
    case FMM_OP_FUSEDMM_A: *bytes = partial_bytes(S_csr, r, k.obytes); return FMM_OK;
    case FMM_OP_SPMM_B:
    case FMM_OP_FUSEDMM_B: *bytes = partial_bytes(S_csc, r, k.obytes); return FMM_OK;
    case FMM_OP_FUSEDMM_A_BWD:
    case FMM_OP_FUSEDMM_B_BWD:
    case FMM_OP_SDDMM_BWD:
    case FMM_OP_SPMM_A_BWD:
    case FMM_OP_SPMM_B_BWD: *bytes = max_partial(S_csr, S_csc, r, k.obytes); return FMM_OK;
    case FMM_OP_FUSEDMM_A_BWD_VALUES: *bytes = partial_bytes(S_csr, r, k.obytes); return FMM_OK;
    case FMM_OP_FUSEDMM_B_BWD_VALUES: *bytes = partial_bytes(S_csc, r, k.obytes); return FMM_OK;
    default: return FMM_ERR_DIM;
    }
}

// ---------------------------------------------------------------- forward

fmm_status fmm_sddmm(const fmm_sparse *S, const void *A, const void *B, int32_t r, int32_t dtype, void *R, double beta,
                     void *ws, size_t ws_bytes, hipStream_t stream)
{
    (void)ws;
    (void)ws_bytes;
    FMM_TRY(check_sparse(S, -1));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    FMM_TRY(check_dense(A, S->rows, k.sbytes, r));
    FMM_TRY(check_dense(B, S->cols, k.sbytes, r));
    if (S->nnz > 0 && !R) return FMM_ERR_NULL;
    LineArgs a = base_args(S, r, nullptr);
    a.n_chunks = S->n_chunks;  // chunks only rebalance; SDDMM has no partials
    const bool csr = S->orient == FMM_CSR;
    a.H = csr ? A : B;
    a.G1 = csr ? B : A;
    a.out = R;
    a.beta = beta;
    fmm_sparse Sx = *S;
    Sx.n_splits = 0;
    FMM_HIP(run<OP_SDDMM>(k.path, 'S', 'S', 'S', a, &Sx, stream));
    return FMM_OK;
}

fmm_status fmm_spmm_a(const fmm_sparse *S_csr, const void *w, const void *B, int32_t r, int32_t dtype, void *C,
                      double beta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_sparse(S_csr, FMM_CSR));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    FMM_TRY(check_dense(B, S_csr->cols, k.sbytes, r));
    FMM_TRY(check_dense(C, S_csr->rows, k.obytes, r));
    FMM_TRY(check_ws(S_csr, r, k.obytes, ws, ws_bytes));
    LineArgs a = base_args(S_csr, r, ws);
    if (w) { a.val = nullptr; a.wv1 = w; }
    a.G1 = B;
    a.out = C;
    a.beta = beta;
    FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csr, stream));
    return FMM_OK;
}

fmm_status fmm_spmm_b(const fmm_sparse *S_csc, const void *w, int32_t w_order, const void *A, int32_t r, int32_t dtype,
                      void *C, double beta, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_sparse(S_csc, FMM_CSC));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    if (w && w_order != FMM_CSR && w_order != FMM_CSC) return FMM_ERR_ORIENT;
    if (w && w_order == FMM_CSR && S_csc->nnz > 0 && !S_csc->perm) return FMM_ERR_NULL;
    FMM_TRY(check_dense(A, S_csc->rows, k.sbytes, r));
    FMM_TRY(check_dense(C, S_csc->cols, k.obytes, r));
    FMM_TRY(check_ws(S_csc, r, k.obytes, ws, ws_bytes));
    LineArgs a = base_args(S_csc, r, ws);
    if (w) {
        a.val = nullptr;
        a.wv1 = w;
        a.wperm = w_order == FMM_CSR ? S_csc->perm : nullptr;
    }
    a.G1 = A;
    a.out = C;
    a.beta = beta;
    FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csc, stream));
    return FMM_OK;
}

fmm_status fmm_fusedmm_a(const fmm_sparse *S_csr, const void *A, const void *B, int32_t r, int32_t dtype, void *C,
                         int32_t flags, void *R_ws, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_sparse(S_csr, FMM_CSR));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    FMM_TRY(check_dense(A, S_csr->rows, k.sbytes, r));
    FMM_TRY(check_dense(B, S_csr->cols, k.sbytes, r));
    FMM_TRY(check_dense(C, S_csr->rows, k.obytes, r));
    FMM_TRY(check_ws(S_csr, r, k.obytes, ws, ws_bytes));
    if (flags != FMM_FUSED && flags != FMM_UNFUSED) return FMM_ERR_DIM;
    if (flags == FMM_UNFUSED) {
        if (S_csr->nnz > 0 && !R_ws) return FMM_ERR_WORKSPACE;
        LineArgs s = base_args(S_csr, r, nullptr);
        s.H = A;
        s.G1 = B;
        s.out = R_ws;
        fmm_sparse Sx = *S_csr;
        Sx.n_splits = 0;
        FMM_HIP(run<OP_SDDMM>(k.path, 'S', 'S', 'S', s, &Sx, stream));
        LineArgs a = base_args(S_csr, r, ws);
        a.val = nullptr;
        a.wv1 = R_ws;
        a.G1 = B;
        a.out = C;
        FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csr, stream));
        return FMM_OK;
    }
    LineArgs a = base_args(S_csr, r, ws);
    a.H = A;
    a.G1 = B;
    a.out = C;
    FMM_HIP(run<OP_FUSED1>(k.path, 'S', 'S', 'S', a, S_csr, stream));
    return FMM_OK;
}

fmm_status fmm_fusedmm_b(const fmm_sparse *S_csc, const void *A, const void *B, int32_t r, int32_t dtype, void *C,
                         int32_t flags, void *R_ws, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_sparse(S_csc, FMM_CSC));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    FMM_TRY(check_dense(A, S_csc->rows, k.sbytes, r));
    FMM_TRY(check_dense(B, S_csc->cols, k.sbytes, r));
    FMM_TRY(check_dense(C, S_csc->cols, k.obytes, r));
    FMM_TRY(check_ws(S_csc, r, k.obytes, ws, ws_bytes));
    if (flags != FMM_FUSED && flags != FMM_UNFUSED) return FMM_ERR_DIM;
    if (flags == FMM_UNFUSED) {
        if (S_csc->nnz > 0 && (!R_ws || !S_csc->perm)) return FMM_ERR_WORKSPACE;
        // SDDMM on the transposed copy, written in CSR order (R keeps S's layout) ...
        LineArgs s = base_args(S_csc, r, nullptr);
        s.H = B;
        s.G1 = A;
        s.out = R_ws;
        s.operm = S_csc->perm;
        fmm_sparse Sx = *S_csc;
        Sx.n_splits = 0;
        FMM_HIP(run<OP_SDDMM>(k.path, 'S', 'S', 'S', s, &Sx, stream));
        // ... then SpMMB reads it back through perm
        LineArgs a = base_args(S_csc, r, ws);
        a.val = nullptr;
        a.wv1 = R_ws;
        a.wperm = S_csc->perm;
        a.G1 = A;
        a.out = C;
        FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csc, stream));
        return FMM_OK;
    }
    LineArgs a = base_args(S_csc, r, ws);
    a.H = B;
    a.G1 = A;
    a.out = C;
    FMM_HIP(run<OP_FUSED1>(k.path, 'S', 'S', 'S', a, S_csc, stream));
    return FMM_OK;
}

// ---------------------------------------------------------------- backward

fmm_status fmm_fusedmm_a_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A, const void *B,
                                  const void *dC, int32_t r, int32_t dtype, void *dA, void *dB, int32_t flags,
                                  const void *R_ws, void *dP_ws, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_pair(S_csr, S_csc));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    const bool dc16 = (flags & FMM_DC_BF16) != 0;
    flags &= ~FMM_DC_BF16;
    if (flags != FMM_FUSED && flags != FMM_UNFUSED) return FMM_ERR_DIM;
    if (dc16 && (dtype != FMM_BF16 || flags != FMM_FUSED)) return FMM_ERR_UNSUPPORTED;
    const char dck = dc16 ? 'S' : 'O';  // kind of dC: bfloat16 storage or float32
    FMM_TRY(check_dense(A, m, k.sbytes, r));
    FMM_TRY(check_dense(B, n, k.sbytes, r));
    FMM_TRY(check_dense(dC, m, dc16 ? k.sbytes : k.obytes, r));
    if (dA) FMM_TRY(check_dense(dA, m, k.obytes, r));
    if (dB) FMM_TRY(check_dense(dB, n, k.obytes, r));
    FMM_TRY(check_ws2(S_csr, S_csc, r, k.obytes, ws, ws_bytes));
    if (flags == FMM_UNFUSED) {
        if (S_csr->nnz > 0 && (!dP_ws || (dB && (!R_ws || !S_csc->perm)))) return FMM_ERR_WORKSPACE;
        LineArgs s = base_args(S_csr, r, nullptr);  // dP = S * (dC B^T)
        s.H = dC;
        s.G1 = B;
        s.out = dP_ws;
        fmm_sparse Sx = *S_csr;
        Sx.n_splits = 0;
        FMM_HIP(run<OP_SDDMM>(k.path, 'O', 'S', 'S', s, &Sx, stream));
        if (dA) {  // dA = dP B
            LineArgs a = base_args(S_csr, r, ws);
            a.val = nullptr;
            a.wv1 = dP_ws;
            a.G1 = B;
            a.out = dA;
            FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csr, stream));
        }
        if (dB) {  // dB = dP^T A + R^T dC, both read through perm
            LineArgs a = base_args(S_csc, r, ws);
            a.val = nullptr;
            a.wv1 = dP_ws;
            a.wv2 = R_ws;
            a.wperm = S_csc->perm;
            a.G1 = A;
            a.G2 = dC;
            a.out = dB;
            FMM_HIP(run<OP_SPMM2>(k.path, 'S', 'S', 'O', a, S_csc, stream));
        }
        return FMM_OK;
    }
    if (dA) {  // dA = FusedMMA(S, dC, B)
        LineArgs a = base_args(S_csr, r, ws);
        a.H = dC;
        a.G1 = B;
        a.out = dA;
        FMM_HIP(run<OP_FUSED1>(k.path, dck, 'S', 'S', a, S_csr, stream));
    }
    if (dB) {  // dB_j = sum_i S_ij (<B_j, dC_i> A_i + <B_j, A_i> dC_i)
        LineArgs a = base_args(S_csc, r, ws);
        a.H = B;
        a.G1 = A;
        a.G2 = dC;
        a.out = dB;
        FMM_HIP(run<OP_FUSED2>(k.path, 'S', 'S', dck, a, S_csc, stream));
    }
    return FMM_OK;
}

fmm_status fmm_fusedmm_b_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A, const void *B,
                                  const void *dC, int32_t r, int32_t dtype, void *dA, void *dB, int32_t flags,
                                  const void *R_ws, void *dP_ws, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_pair(S_csr, S_csc));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    const bool dc16 = (flags & FMM_DC_BF16) != 0;
    flags &= ~FMM_DC_BF16;
    if (flags != FMM_FUSED && flags != FMM_UNFUSED) return FMM_ERR_DIM;
    if (dc16 && (dtype != FMM_BF16 || flags != FMM_FUSED)) return FMM_ERR_UNSUPPORTED;
    const char dck = dc16 ? 'S' : 'O';
    FMM_TRY(check_dense(A, m, k.sbytes, r));
    FMM_TRY(check_dense(B, n, k.sbytes, r));
    FMM_TRY(check_dense(dC, n, dc16 ? k.sbytes : k.obytes, r));
    if (dA) FMM_TRY(check_dense(dA, m, k.obytes, r));
    if (dB) FMM_TRY(check_dense(dB, n, k.obytes, r));
    FMM_TRY(check_ws2(S_csr, S_csc, r, k.obytes, ws, ws_bytes));
    if (flags == FMM_UNFUSED) {
        if (S_csr->nnz > 0 && (!dP_ws || (dA && !R_ws) || (dB && !S_csc->perm))) return FMM_ERR_WORKSPACE;
        LineArgs s = base_args(S_csr, r, nullptr);  // dP = S * (A dC^T), CSR order
        s.H = A;
        s.G1 = dC;
        s.out = dP_ws;
        fmm_sparse Sx = *S_csr;
        Sx.n_splits = 0;
        FMM_HIP(run<OP_SDDMM>(k.path, 'S', 'O', 'O', s, &Sx, stream));
        if (dB) {  // dB = dP^T A through perm
            LineArgs a = base_args(S_csc, r, ws);
            a.val = nullptr;
            a.wv1 = dP_ws;
            a.wperm = S_csc->perm;
            a.G1 = A;
            a.out = dB;
            FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csc, stream));
        }
        if (dA) {  // dA = dP B + R dC
            LineArgs a = base_args(S_csr, r, ws);
            a.val = nullptr;
            a.wv1 = dP_ws;
            a.wv2 = R_ws;
            a.G1 = B;
            a.G2 = dC;
            a.out = dA;
            FMM_HIP(run<OP_SPMM2>(k.path, 'S', 'S', 'O', a, S_csr, stream));
        }
        return FMM_OK;
    }
    if (dB) {  // dB = FusedMMB(S, A, dC): on the transposed copy, held dC_j, gathered A_i
        LineArgs a = base_args(S_csc, r, ws);
        a.H = dC;
        a.G1 = A;
        a.out = dB;
        FMM_HIP(run<OP_FUSED1>(k.path, dck, 'S', 'S', a, S_csc, stream));
    }
    if (dA) {  // dA_i = sum_j S_ij (<A_i, dC_j> B_j + <A_i, B_j> dC_j)
        LineArgs a = base_args(S_csr, r, ws);
        a.H = A;
        a.G1 = B;
        a.G2 = dC;
        a.out = dA;
        FMM_HIP(run<OP_FUSED2>(k.path, 'S', 'S', dck, a, S_csr, stream));
    }
    return FMM_OK;
}

fmm_status fmm_fusedmm_a_backward_values(const fmm_sparse *S_csr, const void *A, const void *B, const void *dC,
                                         int32_t r, int32_t dtype, void *dS, void *dA, int32_t flags, void *ws,
                                         size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_sparse(S_csr, FMM_CSR));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    FMM_TRY(check_dense(A, m, k.sbytes, r));
    FMM_TRY(check_dense(B, n, k.sbytes, r));
    FMM_TRY(check_dense(dC, m, k.obytes, r));
    if (dA) FMM_TRY(check_dense(dA, m, k.obytes, r));
    if (S_csr->nnz > 0 && !dS) return FMM_ERR_NULL;
    if (flags != FMM_FUSED && flags != FMM_UNFUSED) return FMM_ERR_DIM;
    if (flags == FMM_UNFUSED) {
        if (dA) return FMM_ERR_UNSUPPORTED;
        return values_unfused(S_csr, k, A, B, 'O', dC, 'S', B, r, dS, stream);
    }
    if (dA) FMM_TRY(check_ws(S_csr, r, k.obytes, ws, ws_bytes));
    LineArgs a = base_args(S_csr, r, ws);  // held dC_i and A_i, gathered B_j
    a.H = dC;
    a.H2 = A;
    a.G1 = B;
    a.out = dA;
    a.values = dS;
    FMM_HIP(run<OP_FUSED1S>(k.path, 'O', 'S', 'S', a, S_csr, stream));
    return FMM_OK;
}

fmm_status fmm_fusedmm_b_backward_values(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A,
                                         const void *B, const void *dC, int32_t r, int32_t dtype, void *dS,
                                         void *dB, int32_t flags, void *ws, size_t ws_bytes, hipStream_t stream)
{
    FMM_TRY(check_pair(S_csr, S_csc));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    FMM_TRY(check_dense(A, m, k.sbytes, r));
    FMM_TRY(check_dense(B, n, k.sbytes, r));
    FMM_TRY(check_dense(dC, n, k.obytes, r));
    if (dB) FMM_TRY(check_dense(dB, n, k.obytes, r));
    if (S_csr->nnz > 0 && !dS) return FMM_ERR_NULL;
    if (flags != FMM_FUSED && flags != FMM_UNFUSED) return FMM_ERR_DIM;
    if (flags == FMM_UNFUSED) {
        if (dB) return FMM_ERR_UNSUPPORTED;
        return values_unfused(S_csr, k, A, B, 'S', A, 'O', dC, r, dS, stream);
    }
    if (S_csc->nnz > 0 && !S_csc->perm) return FMM_ERR_NULL;
    if (dB) FMM_TRY(check_ws(S_csc, r, k.obytes, ws, ws_bytes));
    LineArgs a = base_args(S_csc, r, ws);  // held dC_j and B_j, gathered A_i; dS through perm
    a.H = dC;
    a.H2 = B;
    a.G1 = A;
    a.out = dB;
    a.values = dS;
    a.operm = S_csc->perm;
    FMM_HIP(run<OP_FUSED1S>(k.path, 'O', 'S', 'S', a, S_csc, stream));
    return FMM_OK;
}

fmm_status fmm_sddmm_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A, const void *B,
                              const void *dR, int32_t r, int32_t dtype, void *dA, void *dB, void *ws, size_t ws_bytes,
                              hipStream_t stream)
{
    FMM_TRY(check_pair(S_csr, S_csc));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    FMM_TRY(check_dense(A, m, k.sbytes, r));
    FMM_TRY(check_dense(B, n, k.sbytes, r));
    if (dA) FMM_TRY(check_dense(dA, m, k.obytes, r));
    if (dB) FMM_TRY(check_dense(dB, n, k.obytes, r));
    if (S_csr->nnz > 0 && !dR) return FMM_ERR_NULL;
    if (dB && S_csr->nnz > 0 && !S_csc->perm) return FMM_ERR_NULL;
    FMM_TRY(check_ws2(S_csr, S_csc, r, k.obytes, ws, ws_bytes));
    if (dA) {  // dA = (S * dR) B
        LineArgs a = base_args(S_csr, r, ws);
        a.wv1 = dR;
        a.G1 = B;
        a.out = dA;
        FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csr, stream));
    }
    if (dB) {  // dB = (S * dR)^T A
        LineArgs a = base_args(S_csc, r, ws);
        a.wv1 = dR;
        a.wperm = S_csc->perm;
        a.G1 = A;
        a.out = dB;
        FMM_HIP(run<OP_SPMM1>(k.path, 'S', 'S', 'S', a, S_csc, stream));
    }
    return FMM_OK;
}

fmm_status fmm_spmm_a_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *w, const void *B,
                               const void *dC, int32_t r, int32_t dtype, void *dw, void *dB, void *ws, size_t ws_bytes,
                               hipStream_t stream)
{
    FMM_TRY(check_pair(S_csr, S_csc));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    FMM_TRY(check_dense(B, n, k.sbytes, r));
    FMM_TRY(check_dense(dC, m, k.obytes, r));
    if (dB) FMM_TRY(check_dense(dB, n, k.obytes, r));
    if (w && dB && S_csr->nnz > 0 && !S_csc->perm) return FMM_ERR_NULL;
    FMM_TRY(check_ws2(S_csr, S_csc, r, k.obytes, ws, ws_bytes));
    if (dw && S_csr->nnz > 0) {  // dw[p] = <dC_i, B_j>
        LineArgs s = base_args(S_csr, r, nullptr);
        s.val = nullptr;
        s.H = dC;
        s.G1 = B;
        s.out = dw;
        fmm_sparse Sx = *S_csr;
        Sx.n_splits = 0;
        FMM_HIP(run<OP_SDDMM>(k.path, 'O', 'S', 'S', s, &Sx, stream));
    }
    if (dB) {  // dB = W^T dC
        LineArgs a = base_args(S_csc, r, ws);
        if (w) {
            a.val = nullptr;
            a.wv1 = w;
            a.wperm = S_csc->perm;
        }
        a.G1 = dC;
        a.out = dB;
        FMM_HIP(run<OP_SPMM1>(k.path, 'O', 'O', 'O', a, S_csc, stream));
    }
    return FMM_OK;
}

fmm_status fmm_spmm_b_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *w, const void *A,
                               const void *dC, int32_t r, int32_t dtype, void *dw, void *dA, void *ws, size_t ws_bytes,
                               hipStream_t stream)
{
    FMM_TRY(check_pair(S_csr, S_csc));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    const int32_t m = S_csr->rows, n = S_csr->cols;
    FMM_TRY(check_dense(A, m, k.sbytes, r));
    FMM_TRY(check_dense(dC, n, k.obytes, r));
    if (dA) FMM_TRY(check_dense(dA, m, k.obytes, r));
    FMM_TRY(check_ws2(S_csr, S_csc, r, k.obytes, ws, ws_bytes));
    if (dw && S_csr->nnz > 0) {  // dw[p] = <A_i, dC_j>
        LineArgs s = base_args(S_csr, r, nullptr);
        s.val = nullptr;
        s.H = A;
        s.G1 = dC;
        s.out = dw;
        fmm_sparse Sx = *S_csr;
        Sx.n_splits = 0;
        FMM_HIP(run<OP_SDDMM>(k.path, 'S', 'O', 'O', s, &Sx, stream));
    }
    if (dA) {  // dA = W dC
        LineArgs a = base_args(S_csr, r, ws);
        if (w) {
            a.val = nullptr;
            a.wv1 = w;
        }
        a.G1 = dC;
        a.out = dA;
        FMM_HIP(run<OP_SPMM1>(k.path, 'O', 'O', 'O', a, S_csr, stream));
    }
    return FMM_OK;
}

// ---------------------------------------------------------------- launch introspection

fmm_status fmm_launch_shape(const fmm_sparse *S, int32_t two_row, int32_t r, int32_t dtype, int32_t *lanes, int32_t *nv,
                            int32_t *vw, int32_t *unroll)
{
    FMM_TRY(check_sparse(S, -1));
    Kinds k;
    FMM_TRY(kinds_for(dtype, r, &k));
    if (!lanes || !nv || !vw || !unroll) return FMM_ERR_NULL;
    // the vector width follows the narrowest operand: bfloat16 storage gives 8, else 16 / element
    const int vwv = k.path == PATH_BF16 ? 8 : k.path == PATH_F64 ? 2 : 4;
    const int w = (r % vwv) == 0 ? vwv : 1;
    const Shape hs{tuning().lanes, tuning().nv};
    const Shape sh = shape_supported(hs, r, w) ? hs : default_shape(r, w);
    const int cls = unroll_class(S);
    const int one = cls == 1 ? 8 : cls == 2 ? 4 : 2;
    int u = (two_row ? one / 2 : one) / sh.NV;
    *lanes = sh.L;
    *nv = sh.NV;
    *vw = w;
    *unroll = u < 1 ? 1 : u;
    return FMM_OK;
}

// ---------------------------------------------------------------- variant autotuning

fmm_status fmm_autotune(int32_t op, fmm_sparse *S_csr, fmm_sparse *S_csc, const void *A, const void *B, const void *dC,
                        int32_t r, int32_t dtype, void *C, void *dA, void *dB, void *ws, size_t ws_bytes,
                        hipStream_t stream)
{
    if (op != FMM_OP_FUSEDMM_A_BWD && op != FMM_OP_FUSEDMM_B_BWD) return FMM_ERR_DIM;
    FMM_TRY(check_pair(S_csr, S_csc));
    if (!C || !dA || !dB) return FMM_ERR_NULL;
    const bool form_a = op == FMM_OP_FUSEDMM_A_BWD;
    // the forward and its same-shaped adjoint pass run on `own`; the two-row pass on `other`
    fmm_sparse *own = form_a ? S_csr : S_csc;
    fmm_sparse *other = form_a ? S_csc : S_csr;
    hipEvent_t e0, e1;
    FMM_HIP(hipEventCreate(&e0));
    FMM_HIP(hipEventCreate(&e1));
    auto fwd = [&]() -> fmm_status {
        return form_a ? fmm_fusedmm_a(S_csr, A, B, r, dtype, C, FMM_FUSED, nullptr, ws, ws_bytes, stream)
                      : fmm_fusedmm_b(S_csc, A, B, r, dtype, C, FMM_FUSED, nullptr, ws, ws_bytes, stream);
    };
    auto two_row = [&]() -> fmm_status {
        return form_a ? fmm_fusedmm_a_backward(S_csr, S_csc, A, B, dC, r, dtype, nullptr, dB, FMM_FUSED, nullptr,
                                               nullptr, ws, ws_bytes, stream)
                      : fmm_fusedmm_b_backward(S_csr, S_csc, A, B, dC, r, dtype, dA, nullptr, FMM_FUSED, nullptr,
                                               nullptr, ws, ws_bytes, stream);
    };
    auto time_it = [&](const std::function<fmm_status()> &f, float *ms) -> fmm_status {
        FMM_TRY(f());  // warm-up
        FMM_HIP(hipEventRecord(e0, stream));
        for (int i = 0; i < 3; ++i) FMM_TRY(f());
        FMM_HIP(hipEventRecord(e1, stream));
        FMM_HIP(hipEventSynchronize(e1));
        FMM_HIP(hipEventElapsedTime(ms, e0, e1));
        return FMM_OK;
    };
    fmm_status st = FMM_OK;
    const int32_t keep_own = own->variant, keep_other = other->variant;
    float best_own = 1e30f, best_other = 1e30f;
    int32_t pick_own = keep_own, pick_other = keep_other;
    for (int32_t v = FMM_VARIANT_DEEP; v <= FMM_VARIANT_SHALLOW && st == FMM_OK; ++v) {
        float ms = 0.f;
        own->variant = v;
        st = time_it(fwd, &ms);
        if (st == FMM_OK && ms < best_own) {
            best_own = ms;
            pick_own = v;
        }
        if (st != FMM_OK) break;
        other->variant = v;
        st = time_it(two_row, &ms);
        if (st == FMM_OK && ms < best_other) {
            best_other = ms;
            pick_other = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    own->variant = st == FMM_OK ? pick_own : keep_own;
    other->variant = st == FMM_OK ? pick_other : keep_other;
    return st;
}

}  // extern "C"
