/*
 * fmm.h -- C ABI of the local FusedMM library for AMD Instinct MI355X (gfx950).
 *
 * Operations (Bharadwaj, Buluc, Demmel, "Distributed-Memory Sparse Kernels for
 * Machine Learning", Section II):
 *
 *   SDDMM(A, B, S)     = S * (A B^T)     Eq. (1): the sampled product, evaluated
 *                                          only at the stored entries of S
 *                                          (R_ij = S_ij <A_i:, B_j:>, Section IV-A)
 *   SpMMA(S, B)        = S B             m x r output
 *   SpMMB(S, A)        = S^T A           n x r output
 *   FusedMMA(S, A, B)  = SpMMA(SDDMM(A, B, S), B)
 *   FusedMMB(S, A, B)  = SpMMB(SDDMM(A, B, S), A)
 *
 * S is m x n sparse, A is m x r, B is n x r.  FusedMMB runs on a stored transposed
 * copy of S (Section IV-B).  The fused calls keep each sampled value R_ij in
 * registers between the two products instead of writing R to memory (the local
 * fused kernel the paper cites in Section IV-B).  Backward calls give the adjoints
 * with respect to A and B for a fixed S, and separate calls the gradient with
 * respect to S's stored values.  Beyond these: the graph-attention head and its
 * adjoint, batched CG for ALS (Section VI-E), batch plans over many graphs, and
 * streaming probes for measurement.
 *
 * Conventions that hold for every call unless its comment says otherwise:
 *   * Pointers named in a call are DEVICE pointers; sizes and descriptors are host
 *     values.  The caller owns every buffer.  Calls never allocate, except
 *     fmm_validate (a 4-byte flag) and the batch-plan calls (their own tables).
 *   * Dense matrices are row-major with r contiguous elements per row (row stride r).
 *     FMM_F32 and FMM_BF16 name the storage of A and B; S values, dC and every
 *     output are float32 for both (with FMM_BF16 the adjoints can also take dC as
 *     bfloat16: FMM_DC_BF16).  FMM_F64 makes everything float64.
 *     Limits on r: FMM_F32 r <= 1024 when r % 4 == 0, else r <= 256; FMM_BF16
 *     r % 8 == 0 and r <= 1024; FMM_F64 r <= 512 when r is even, else r <= 256.
 *     When r*sizeof(elem) is a multiple of 16 the dense bases must be 16-byte
 *     aligned (FMM_ERR_UNSUPPORTED otherwise).
 *   * Index arrays are int32 and canonical: ptr is non-decreasing with ptr[0] = 0,
 *     ptr[major] = nnz; idx holds minor indices strictly increasing inside each
 *     major line.  Hot calls trust this; fmm_validate checks it.
 *   * Calls enqueue work on `stream` and return without waiting, except where a
 *     comment says "synchronous".  An invalid argument returns a negative status
 *     before anything is enqueued.  A failed HIP launch returns FMM_ERR_HIP and
 *     fmm_last_hip_error() gives the hipError_t.
 *   * beta: outputs are overwritten when beta == 0 (prior contents are not read),
 *     otherwise out = beta * out + result (the "+=" form of the paper's local calls,
 *     Algorithm 1).
 *   * Results are deterministic: no floating-point atomics; every output element is
 *     summed in a fixed order for a fixed pattern, schedule and r.
 */
#ifndef FMM_H
#define FMM_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FMM_ABI_VERSION 4

typedef enum fmm_status {
    FMM_OK = 0,
    FMM_ERR_NULL = -1,          /* a required pointer is NULL                          */
    FMM_ERR_DIM = -2,           /* a size is negative, zero where it must not be, or
                                   inconsistent between arguments                       */
    FMM_ERR_DTYPE = -3,         /* unknown dtype, or dtype / r combination unsupported  */
    FMM_ERR_ORIENT = -4,        /* descriptor has the wrong orientation for the call    */
    FMM_ERR_INDEX = -5,         /* fmm_validate: index out of range, or ptr not
                                   monotone / not starting at 0 / not ending at nnz     */
    FMM_ERR_NONCANONICAL = -6,  /* fmm_validate: duplicate or unsorted minor indices    */
    FMM_ERR_WORKSPACE = -7,     /* workspace missing or smaller than required           */
    FMM_ERR_UNSUPPORTED = -8,   /* valid request this library does not implement        */
    FMM_ERR_HIP = -9,           /* a HIP runtime call failed                           */
    FMM_ERR_STATE = -10         /* batch plan not in the state the call needs (no graph
                                   captured, or captured before the latest autotune)   */
} fmm_status;

typedef enum fmm_dtype { FMM_F32 = 0, FMM_BF16 = 1, FMM_F64 = 2 } fmm_dtype;
typedef enum fmm_orient { FMM_CSR = 0, FMM_CSC = 1 } fmm_orient;

/* flags for the fused calls */
#define FMM_FUSED 0    /* one pass, sampled values kept in registers                    */
#define FMM_UNFUSED 1  /* SDDMM writes R (nnz values) to R_ws, then SpMM reads it back  */
#define FMM_DC_BF16 2  /* adjoints only, OR-ed with FMM_FUSED: dC is bfloat16 storage    */

/*
 * A sparse matrix S (rows x cols) in one orientation.
 *   orient == FMM_CSR: major lines are rows, ptr = rowptr[rows+1], idx = colidx.
 *   orient == FMM_CSC: major lines are columns, ptr = colptr[cols+1], idx = rowidx,
 *                      val = S's values in CSC order, perm[q] = CSR position of the
 *                      q-th CSC entry (needed only where a call says so).
 * val is float32 (float64 for FMM_F64); NULL means every stored value is 1.
 *
 * Optional split schedule (from fmm_schedule_count / fmm_schedule_fill): major lines
 * with more than long_len stored entries are cut into chunks that run in parallel and
 * are summed afterwards in chunk order.  n_chunks == 0 disables it.
 *
 * order: optional processing order of the major lines (from fmm_line_order), a
 * permutation of [0, major extent); NULL processes lines in index order.  It changes
 * only which lane group takes which line, never a line's arithmetic, so results are
 * bit-identical with and without it.  Grouping lines of similar length into the same
 * wavefront keeps a wavefront from idling behind its longest line.
 *
 * hot: optional gather hint per stored entry (orientation order, from fmm_gather_hints).
 * An entry with hot[p] == 0 gathers its dense row with the streaming (nontemporal) cache
 * policy, any other with the default policy; NULL gathers every row with the default
 * policy.  Rows of hub lines, which many entries gather, then keep their place in L2
 * and the MALL instead of being displaced by rows that are gathered once.  It changes
 * only the cache policy of loads, so results are bit-identical with and without it.
 *
 * variant: how many stored entries a lane group keeps in flight per batch (FMM_VARIANT_*).
 * Deep batches suit long, uniform lines; shallow ones use fewer registers, so more lines
 * are in flight at once, which suits many short lines.  FMM_VARIANT_AUTO picks from the
 * mean line length (>= 24: deep, >= 6: medium, else shallow); fmm_autotune picks by
 * timing.  Results differ only in summation order (all within the gate).
 */
#define FMM_VARIANT_AUTO 0
#define FMM_VARIANT_DEEP 1     /* 8 entries per batch (4 for the two-row passes) */
#define FMM_VARIANT_MEDIUM 2   /* 4 (2)                                          */
#define FMM_VARIANT_SHALLOW 3  /* 2 (1)                                          */
typedef struct fmm_sparse {
    int32_t orient;
    int32_t rows, cols;
    int32_t nnz;
    const int32_t *ptr;
    const int32_t *idx;
    const void *val;
    const int32_t *perm;
    int32_t long_len;          /* lines with more entries than this are split            */
    int32_t n_chunks;          /* number of chunk items                                  */
    int32_t n_splits;          /* number of split lines                                  */
    int32_t variant;           /* FMM_VARIANT_*                                            */
    const int32_t *chunks;     /* [3*n_chunks]: line, begin position, end position       */
    const int32_t *splits;     /* [3*n_splits]: line, first chunk, chunk count           */
    const int32_t *order;      /* [major extent] line processing order, or NULL          */
    const uint8_t *hot;        /* [nnz] gather hint per stored entry, or NULL            */
} fmm_sparse;

/* ---------------------------------------------------------------- diagnostics */

int32_t fmm_abi_version(void);
/* Static text for a status code. */
const char *fmm_status_string(int32_t status);
/* hipError_t of the last HIP failure seen by this thread (0 if none). */
int32_t fmm_last_hip_error(void);
/* Number of compute units and the GPU architecture name of the current device
   (arch: caller buffer of arch_len bytes, NUL-terminated). Synchronous. */
fmm_status fmm_device_info(int32_t *num_cu, char *arch, int32_t arch_len);

/*
 * Streaming probes for measurement (not part of the method): the HBM rate this GPU
 * reaches on contiguous traffic, the practical ceiling next to the 8 TB/s specification
 * against which the gather kernels' rates are read.
 *   fmm_stream_copy: dst[0, bytes) = src[0, bytes)  (reads and writes `bytes` each)
 *   fmm_stream_read: reads src[0, bytes) and folds it into one 32-bit value, which is
 *                    stored to *sink only if it equals key (so the pass writes nothing
 *                    in practice); sink: one device word.
 * bytes: a multiple of 16 (else FMM_ERR_DIM); pointers 16-byte aligned (else
 * FMM_ERR_UNSUPPORTED); the buffers must not overlap.  bytes = 0 does nothing.
 */
fmm_status fmm_stream_copy(const void *src, void *dst, size_t bytes, hipStream_t stream);
fmm_status fmm_stream_read(const void *src, size_t bytes, uint32_t key, uint32_t *sink, hipStream_t stream);
/*
 * Gather probe (measurement only): reads rows rows[0 .. n_rows-1] of src, each row_bytes
 * long (16 * 2^k bytes, k = 0..6, else FMM_ERR_DIM), one lane per 16 bytes with the
 * default cache policy, the way the line kernels gather rows; folds them into *sink as
 * fmm_stream_read does.  With rows a permutation of the rows of a buffer larger than the
 * caches, every row comes from memory once, so the pass moves a known number of bytes
 * (n_rows * row_bytes, plus 4 * n_rows of indices), to calibrate hardware counters on
 * gather-shaped traffic.  The caller keeps every rows[k] inside src.
 */
fmm_status fmm_stream_gather(const void *src, size_t row_bytes, const int32_t *rows, int64_t n_rows, uint32_t key,
                             uint32_t *sink, hipStream_t stream);

/*
 * Lane-group shape override for every later launch in this process (tuning and
 * benchmarking): `lanes` lanes own one major line and each lane holds `nv` 16-byte
 * vectors of an r-vector.  (0, 0) restores the automatic choice (the smallest power of
 * two lanes covering r).  Compiled shapes: nv = 1 with lanes 1..64 (powers of two),
 * nv = 2 with lanes 16, 32, 64, nv = 4 with lanes 64; a shape that does not fit r
 * falls back to the automatic one.  Not synchronised with launches on other threads.
 */
fmm_status fmm_set_tuning(int32_t lanes, int32_t nv);

/*
 * The line-kernel configuration a call on S would launch (for profiling and tests):
 * lanes per line, 16-byte vectors per lane, elements per vector and entries per batch,
 * for the one-row passes (two_row = 0: SDDMM, SpMM, fused forward, dA/dB of the same
 * orientation) or the two-row adjoint pass (two_row = 1).  Host-only; no device work.
 */
fmm_status fmm_launch_shape(const fmm_sparse *S, int32_t two_row, int32_t r, int32_t dtype, int32_t *lanes,
                            int32_t *nv, int32_t *vw, int32_t *unroll);

/* ---------------------------------------------------------------- pattern prep */

/*
 * Check that S is canonical (see conventions): ptr[0] == 0, ptr[major] == nnz, ptr
 * non-decreasing, 0 <= idx < minor extent, idx strictly increasing in each line.
 * The paper keeps its sparse blocks as coordinate lists and says nothing of order or
 * repeated coordinates (Section V); this library reads S as the set of its stored
 * entries, one per coordinate, so the CSR of S and its stored transposed copy (Section
 * IV-B) are unique, and the hot calls rely on that form.
 * Synchronous.  Returns FMM_OK, FMM_ERR_INDEX or FMM_ERR_NONCANONICAL.  Allocates
 * a 4-byte device flag for the duration of the call.
 */
fmm_status fmm_validate(const fmm_sparse *S, hipStream_t stream);

/*
 * Stored transposed copy of a CSR pattern (Section IV-B): from rowptr[m+1],
 * colidx[nnz] (and optional values val[nnz] of dtype val_dtype: FMM_F32 or FMM_F64)
 * build colptr[n+1], rowidx[nnz], perm[nnz] and, when val and valT are both
 * non-NULL, valT[q] = val[perm[q]].  Rows inside a column come out ascending, so
 * the result is the unique canonical CSC and equals any exact transpose bit for bit.
 * Needs a device workspace of fmm_csr_to_csc_workspace() bytes.  nnz < 2^31.
 */
fmm_status fmm_csr_to_csc_workspace(int32_t m, int32_t n, int32_t nnz, size_t *bytes);
fmm_status fmm_csr_to_csc(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr,
                          const int32_t *colidx, const void *val, int32_t val_dtype,
                          int32_t *colptr, int32_t *rowidx, void *valT, int32_t *perm,
                          void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Split schedule for skewed line lengths.  Lines (rows of a CSR, columns of a CSC)
 * with more than long_len entries are cut into chunks of at most `chunk` entries.
 *   fmm_schedule_count: synchronous; writes the number of chunks and of split lines
 *                       to the host ints *n_chunks, *n_splits.
 *   fmm_schedule_fill:  fills chunks[3*n_chunks] (line, begin, end) and
 *                       splits[3*n_splits] (line, first chunk, chunk count), lines
 *                       ascending.
 * Both take a workspace of fmm_schedule_workspace() bytes.  long_len >= chunk >= 1.
 */
fmm_status fmm_schedule_workspace(int32_t nmajor, size_t *bytes);
fmm_status fmm_schedule_count(const int32_t *ptr, int32_t nmajor, int32_t long_len, int32_t chunk,
                              int32_t *n_chunks, int32_t *n_splits, void *ws, size_t ws_bytes,
                              hipStream_t stream);
fmm_status fmm_schedule_fill(const int32_t *ptr, int32_t nmajor, int32_t long_len, int32_t chunk,
                             int32_t *chunks, int32_t *splits, void *ws, size_t ws_bytes,
                             hipStream_t stream);

/*
 * Values of S in another orientation: dst[q] = src[perm[q]] for q < nnz (float32 or
 * float64 per val_dtype).  With the perm of fmm_csr_to_csc it turns CSR-order values
 * (new or learned edge values) into the CSC order of the stored transposed copy.
 */
fmm_status fmm_gather_values(const int32_t *perm, const void *src, int32_t val_dtype, void *dst, int32_t nnz,
                             hipStream_t stream);

/*
 * Line processing order for a descriptor's `order` field (a schedule choice; the paper
 * balances load by permuting S at random, Section VI).  From ptr[nlines+1] it writes the
 * permutation order[nlines]: first the lines with at most long_len entries, by
 * decreasing length (lengths of 1023 and more count as equal), then the longer lines,
 * which the split schedule processes as chunks; ties keep index order.  A stable radix
 * sort on the GPU, so the result is unique.  Takes a device workspace of
 * fmm_line_order_workspace() bytes; asynchronous on `stream`.  long_len >= 1.
 */
fmm_status fmm_line_order_workspace(int32_t nlines, size_t *bytes);
fmm_status fmm_line_order(const int32_t *ptr, int32_t nlines, int32_t long_len, int32_t *order, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/*
 * Gather hints (see fmm_sparse.hot) for the descriptor S: hot[p] = 1 when the minor line
 * of stored entry p (its column for a CSR descriptor, its row for a CSC one) is among the
 * `top` longest minor lines, else 0.  minor_ptr is the other orientation's pointer array
 * (n_minor + 1 entries: colptr for a CSR S, rowptr for a CSC S), whose line lengths are
 * the minor lines' entry counts; every line as long as the top-th longest counts as one
 * of them.  top <= 0 marks no entry hot; top >= n_minor marks every entry hot.  hot:
 * S->nnz bytes, caller-owned.  Synchronous: the length threshold is found on the host
 * from a copy of minor_ptr.  The paper keeps reused rows in cache by blocking the loop
 * over stored entries (Section III-A); the hint keeps the most reused rows there by cache
 * policy instead, without reordering any work.  Pattern autotuning decides per
 * orientation whether to use it.
 */
fmm_status fmm_gather_hints(const fmm_sparse *S, const int32_t *minor_ptr, int32_t n_minor, int32_t top,
                            uint8_t *hot, hipStream_t stream);

/* Round float32 to bfloat16 storage (nearest, ties to even; NaN -> 0x7FC0). */
fmm_status fmm_f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t stream);

/*
 * Workspace bytes a call needs for the given descriptor(s), r and dtype: the split
 * partial sums (n_chunks * r output elements for each descriptor the call walks).
 * op: one of the FMM_OP_* values below.  Zero when no descriptor has a schedule.
 */
#define FMM_OP_SDDMM 0
#define FMM_OP_SPMM_A 1
#define FMM_OP_SPMM_B 2
#define FMM_OP_FUSEDMM_A 3
#define FMM_OP_FUSEDMM_B 4
#define FMM_OP_FUSEDMM_A_BWD 5
#define FMM_OP_FUSEDMM_B_BWD 6
#define FMM_OP_SDDMM_BWD 7
#define FMM_OP_SPMM_A_BWD 8
#define FMM_OP_SPMM_B_BWD 9
#define FMM_OP_FUSEDMM_A_BWD_VALUES 10
#define FMM_OP_FUSEDMM_B_BWD_VALUES 11
fmm_status fmm_workspace_size(int32_t op, const fmm_sparse *S_csr, const fmm_sparse *S_csc,
                              int32_t r, int32_t dtype, size_t *bytes);

/* ---------------------------------------------------------------- forward */

/*
 * SDDMM, Eq. (1): R[p] = beta*R[p] + val[p] * <A_i:, B_j:> for every stored entry
 * p = (i, j) of S, in S's orientation order (CSR positions for a CSR descriptor,
 * CSC positions for a CSC one).  A: rows x r, B: cols x r, R: nnz outputs.
 */
fmm_status fmm_sddmm(const fmm_sparse *S, const void *A, const void *B, int32_t r, int32_t dtype,
                     void *R, double beta, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * SpMMA (Section II): C = beta*C + W B, C: rows x r, B: cols x r, where W has S's
 * pattern and stored values w[p] (CSR order, output dtype), or S's own values when
 * w is NULL.  S_csr must be a CSR descriptor.
 */
fmm_status fmm_spmm_a(const fmm_sparse *S_csr, const void *w, const void *B, int32_t r,
                      int32_t dtype, void *C, double beta, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/*
 * SpMMB (Section II): C = beta*C + W^T A, C: cols x r, A: rows x r.  S_csc must be a
 * CSC descriptor.  W has S's pattern; its stored values are S's own (valT, CSC
 * order) when w is NULL, else w indexed by CSC position when w_order == FMM_CSC, or
 * by CSR position through perm when w_order == FMM_CSR (then S_csc->perm is required).
 */
fmm_status fmm_spmm_b(const fmm_sparse *S_csc, const void *w, int32_t w_order, const void *A,
                      int32_t r, int32_t dtype, void *C, double beta, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/*
 * FusedMMA(S, A, B) = SpMMA(SDDMM(A, B, S), B) (Section II; row form in Section IV-B):
 * C_i: = sum_j S_ij <A_i:, B_j:> B_j:, C: rows x r, overwritten (beta = 0).
 * flags FMM_FUSED: one pass.  FMM_UNFUSED: R_ws (nnz output elements) receives R,
 * then a second pass reads it back.  ws: split partials (see fmm_workspace_size).
 */
fmm_status fmm_fusedmm_a(const fmm_sparse *S_csr, const void *A, const void *B, int32_t r,
                         int32_t dtype, void *C, int32_t flags, void *R_ws, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/*
 * For callers that cannot allocate device memory: code under hipGraph / stream
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same result as
 * fmm_fusedmm_a(S_csr, A, B, r, dtype, C, FMM_FUSED, NULL, ws, ...), computed by the
 * same kernels, except that the partial sums of split lines go to a device array the
 * library owns: FMM_NOALLOC_SCRATCH_BYTES per GPU, held by each GPU the library runs
 * on until the process ends.  The call allocates nothing.  It returns
 * FMM_ERR_WORKSPACE when the split partials need more than that (fmm_workspace_size
 * with FMM_OP_FUSEDMM_A gives the need), and FMM_ERR_HIP if the array's device
 * address cannot be found on the current device.  Every call on one GPU shares that
 * GPU's array, which keeps the last call's contents: calls that overlap in time on one
 * GPU (on different streams, or from different threads) race and must not be issued.
 */
#define FMM_NOALLOC_SCRATCH_BYTES (64u << 20)
fmm_status fmm_fusedmm_a_noalloc(const fmm_sparse *S_csr, const void *A, const void *B, int32_t r,
                                 int32_t dtype, void *C, hipStream_t stream);

/*
 * FusedMMB(S, A, B) = SpMMB(SDDMM(A, B, S), A) (Section II):
 * C'_j: = sum_i S_ij <A_i:, B_j:> A_i:, C': cols x r, computed on the CSC descriptor
 * as FusedMMA(S^T, B, A) (Section IV-B's transposed copy).  UNFUSED: the SDDMM on the
 * transposed copy writes R into R_ws in S's own (CSR) order through S_csc->perm (the
 * layout of the paper's unfused sequence), and the SpMMB reads it back through perm;
 * S_csc->perm is required.
 */
fmm_status fmm_fusedmm_b(const fmm_sparse *S_csc, const void *A, const void *B, int32_t r,
                         int32_t dtype, void *C, int32_t flags, void *R_ws, void *ws,
                         size_t ws_bytes, hipStream_t stream);

/*
 * Choose the batch variant of S_csr and S_csc for the FusedMMA (op = FMM_OP_FUSEDMM_A_BWD)
 * or FusedMMB (op = FMM_OP_FUSEDMM_B_BWD) forward and adjoint, by timing each variant on
 * these operands with HIP events; writes S_csr->variant and S_csc->variant.  The pass that
 * decides each orientation is the one that runs on it: the forward (and its same-shaped
 * adjoint pass) for the operation's own orientation, the two-row adjoint pass for the
 * other.  C (forward output), dA and dB are overwritten; ws as for the adjoint call.
 * Synchronous.
 */
fmm_status fmm_autotune(int32_t op, fmm_sparse *S_csr, fmm_sparse *S_csc, const void *A, const void *B,
                        const void *dC, int32_t r, int32_t dtype, void *C, void *dA, void *dB, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- backward */

/*
 * The paper gives no adjoints.  Every call below is the chain rule through the forward
 * definitions it names (Section II; the sampled product per entry, Eq. (1) and Section
 * IV-A), with S's stored values held fixed unless the call says otherwise.  They match
 * central finite differences and dense autograd in the oracle's tests.
 *
 * Adjoint of C = FusedMMA(S, A, B) for fixed S, with upstream gradient dC (rows x r):
 *   dP = S * (dC B^T)          (the gradient reaching A B^T, an SDDMM)
 *   dA = dP B                  = FusedMMA(S, dC, B)            (row pass on S_csr)
 *   dB = dP^T A + R^T dC       with R = S * (A B^T)            (column pass on S_csc)
 * dA or dB may be NULL to skip that output.  FMM_FUSED recomputes the sampled values
 * in registers; FMM_UNFUSED writes dP to dP_ws (nnz, CSR order) and needs R from the
 * unfused forward in R_ws (CSR order) plus S_csc->perm.
 * FMM_FUSED | FMM_DC_BF16 (dtype FMM_BF16 only, else FMM_ERR_UNSUPPORTED): dC is
 * stored as bfloat16 like A and B, so the column pass gathers 2 bytes per element of
 * dC instead of 4 (accumulation and outputs stay float32).  The rounding of dC is the
 * caller's: results are those for the rounded dC.
 */
fmm_status fmm_fusedmm_a_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A,
                                  const void *B, const void *dC, int32_t r, int32_t dtype,
                                  void *dA, void *dB, int32_t flags, const void *R_ws, void *dP_ws,
                                  void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adjoint of C' = FusedMMB(S, A, B) (Section II; FusedMMA on the transposed copy,
 * Section IV-B) with upstream gradient dC (cols x r):
 *   dP = S * (A dC^T)
 *   dA = dP B + R dC           (row pass on S_csr)
 *   dB = dP^T A                = FusedMMB(S, A, dC)            (column pass on S_csc)
 * Same flag and workspace rules as fmm_fusedmm_a_backward, FMM_DC_BF16 included (R_ws,
 * from the unfused FusedMMB forward, and dP_ws are both in CSR order).
 */
fmm_status fmm_fusedmm_b_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A,
                                  const void *B, const void *dC, int32_t r, int32_t dtype,
                                  void *dA, void *dB, int32_t flags, const void *R_ws, void *dP_ws,
                                  void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Gradient with respect to S's stored values (learned edge values; the paper's attention
 * application, Section VI-E, trains such values), for C = FusedMMA(S, A, B) = R B with
 * R = S * P, P = A B^T and upstream gradient dC (rows x r):
 *   dS_ij = P_ij <dC_i, B_j>                      at every stored entry, CSR order.
 * dS: nnz values (float32; float64 for FMM_F64).  FMM_FUSED: one pass on S_csr holding
 * dC_i and A_i, gathering B_j, with both dot products in registers; when dA is non-NULL
 * the same pass also writes dA = FusedMMA(S, dC, B) (the row pass of
 * fmm_fusedmm_a_backward), so a training step with learned values costs no extra pass.
 * FMM_UNFUSED: two SDDMM passes (P into dS, then dS *= <dC_i, B_j> in place); dA must
 * be NULL.  ws: split partials of S_csr when dA is written (FMM_OP_FUSEDMM_A_BWD_VALUES).
 */
fmm_status fmm_fusedmm_a_backward_values(const fmm_sparse *S_csr, const void *A, const void *B, const void *dC,
                                         int32_t r, int32_t dtype, void *dS, void *dA, int32_t flags, void *ws,
                                         size_t ws_bytes, hipStream_t stream);

/*
 * The same for C' = FusedMMB(S, A, B) = R^T A, upstream gradient dC (cols x r):
 *   dS_ij = P_ij <A_i, dC_j>                      CSR order.
 * FMM_FUSED: one pass on the transposed copy S_csc holding dC_j and B_j, gathering A_i,
 * writing dS through S_csc->perm and, when dB is non-NULL, dB = FusedMMB(S, A, dC) (the
 * column pass of fmm_fusedmm_b_backward).  FMM_UNFUSED: two SDDMM passes on S_csr; dB
 * must be NULL.  ws: split partials of S_csc when dB is written.
 */
fmm_status fmm_fusedmm_b_backward_values(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A,
                                         const void *B, const void *dC, int32_t r, int32_t dtype, void *dS,
                                         void *dB, int32_t flags, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adjoint of R = SDDMM(A, B, S) (Eq. (1)) with upstream gradient dR (nnz, CSR order):
 *   dA = (S * dR) B on S_csr,  dB = (S * dR)^T A on S_csc (reads dR through perm).
 */
fmm_status fmm_sddmm_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *A,
                              const void *B, const void *dR, int32_t r, int32_t dtype, void *dA,
                              void *dB, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adjoint of C = SpMMA(W, B) (Section II) with stored values w (CSR order; NULL = S's values):
 *   dw[p] = <dC_i:, B_j:>        (nnz, CSR order; the gradient of the stored values)
 *   dB    = W^T dC               on S_csc (reads w through perm)
 */
fmm_status fmm_spmm_a_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *w,
                               const void *B, const void *dC, int32_t r, int32_t dtype, void *dw,
                               void *dB, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Adjoint of C' = SpMMB(W, A) (Section II) with stored values w (CSR order; NULL = S's
 * values), dC': cols x r:
 *   dw[p] = <A_i:, dC'_j:>       (nnz, CSR order)
 *   dA    = W dC'                on S_csr
 */
fmm_status fmm_spmm_b_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *w,
                               const void *A, const void *dC, int32_t r, int32_t dtype, void *dw,
                               void *dA, void *ws, size_t ws_bytes, hipStream_t stream);


/* ---------------------------------------------------------------- graph attention */

/*
 * Graph-attention variant of the sampled product (Section VI-E): one attention head on a
 * square graph S (n x n CSR, values S_ij or NULL for a 0/1 adjacency) with node features
 * H (n x r, H = A W computed by the caller) and attention vector a = (a1 || a2):
 *
 *   score_ij = a^T (H_i || H_j) = s_i + t_j,   s = H a1,  t = H a2      (fmm_gat_scores)
 *   e_ij     = LeakyReLU(S_ij * score_ij)  (negative_slope for x < 0)
 *   w_ij     = e_ij, or with FMM_GAT_SOFTMAX the softmax of e over the stored entries of
 *              row i (the softmax regularisation of learned edge weights)
 *   out_i    = sum_j w_ij H_j                                            (fmm_gat_forward)
 *
 * The forward is one pass per row: edge values never reach memory (with the softmax the
 * running maximum and normaliser are kept with the partial sum and rescaled as the
 * maximum grows).  Rows with no stored entry give 0.  dtype is H's storage (FMM_F32,
 * FMM_BF16, FMM_F64); a1, a2, s, t, out and S's values are float32 (float64 for
 * FMM_F64).  A split schedule on S is honoured; it then needs a workspace of
 * fmm_gat_workspace() bytes.  Multi-head attention is one call per head.  With the
 * softmax, lse (optional, n values; NULL skips it) receives each row's log-sum-exp
 * max_k e_ik + log sum_k exp(e_ik - max_k e_ik) (0 for an empty row), which the adjoint
 * uses to recompute the weights.
 */
#define FMM_GAT_SOFTMAX 1
fmm_status fmm_gat_scores(const void *H, int32_t n, int32_t r, int32_t dtype, const void *a1, const void *a2,
                          void *s, void *t, hipStream_t stream);
fmm_status fmm_gat_workspace(const fmm_sparse *S, int32_t r, int32_t dtype, size_t *bytes);
fmm_status fmm_gat_forward(const fmm_sparse *S, const void *s, const void *t, const void *H, int32_t r, int32_t dtype,
                           double negative_slope, int32_t flags, void *out, void *lse, void *ws, size_t ws_bytes,
                           hipStream_t stream);
/*
 * The edge values w_ij themselves, in CSR order (nnz values, float32; float64 for
 * FMM_F64): the unfused form, for a separate SpMM (fmm_spmm_a with w) or inspection.
 * The row softmax sums in a fixed order per row.  S's split schedule is not used.
 */
fmm_status fmm_gat_edge_values(const fmm_sparse *S, const void *s, const void *t, int32_t dtype,
                               double negative_slope, int32_t flags, void *w, hipStream_t stream);

/*
 * Adjoint of the attention head (the paper evaluates the forward only; this is the chain
 * rule through the definition above).  Given the forward's s, t (fmm_gat_scores), out
 * and, with the softmax, lse (fmm_gat_forward with the same flags and slope), and the
 * upstream gradient dO:
 *
 *   dw_ij = <dO_i, H_j>;  de = dw, or with the softmax w_ij (dw_ij - <dO_i, out_i>)
 *   dx_ij = de_ij * (1 if S_ij (s_i + t_j) > 0 else negative_slope)
 *   dS_ij = dx_ij (s_i + t_j)   (CSR order; skipped when dS is NULL)
 *   ds_i = sum_j dx_ij S_ij,  dt_j = sum_i dx_ij S_ij
 *   dH = W^T dO + ds a1^T + dt a2^T,  da1 = H^T ds,  da2 = H^T dt
 *
 * Two passes over the pattern (rows on S_csr, columns on S_csc), each recomputing the
 * edge weights and dw in registers; no atomics, fixed summation orders.  Both
 * descriptors' split schedules and orders are honoured.  dtype as for fmm_gat_forward
 * (dO, out, dH, da1, da2, s, t, a1, a2 float32; float64 for FMM_F64).  flags:
 * FMM_GAT_SOFTMAX as in the forward, OR-ed with FMM_DC_BF16 (FMM_BF16 only, else
 * FMM_ERR_UNSUPPORTED) when dO is stored as bfloat16: the row pass holds it and the
 * column pass gathers it at 2 bytes per element; every output stays float32.  ws: a
 * device workspace of fmm_gat_backward_workspace() bytes, 256-byte aligned.
 */
fmm_status fmm_gat_backward_workspace(const fmm_sparse *S_csr, const fmm_sparse *S_csc, int32_t r, int32_t dtype,
                                      size_t *bytes);
fmm_status fmm_gat_backward(const fmm_sparse *S_csr, const fmm_sparse *S_csc, const void *H, const void *a1,
                            const void *a2, const void *s, const void *t, const void *out, const void *lse,
                            const void *dO, int32_t r,
                            int32_t dtype, double negative_slope, int32_t flags, void *dH, void *da1, void *da2,
                            void *dS, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- alternating least squares */

/*
 * Batched conjugate gradients for the per-line least-squares problems of alternating
 * least squares on observed entries (Section VI-E).  For every major line x of S (a row
 * of A when S is the CSR and F = B; a row of B when S is the stored transpose and F = A):
 *
 *   (sum_{j in line} F_j F_j^T + lambda I) x = rhs_x,
 *
 * run `iters` CG steps from the start value in X (overwritten with the result).  Each
 * step computes the query vectors of all lines at once with one pass over S's pattern
 * (S's values are ignored: the pass is the FusedMM of the pattern, M p = sum_j <p, F_j> F_j
 * + lambda p), followed by one fused kernel that forms the step sizes per line and updates
 * X, the residual and the direction.  A line with zero residual or curvature keeps its
 * iterate.  rhs and X: nmajor x r float32; F: minor x r, dtype FMM_F32 or FMM_BF16;
 * work: fmm_cg_work_size() bytes (three nmajor x r float32 blocks and nmajor scalars);
 * ws: split partials of S as for the fused calls.  lambda >= 0.
 */
fmm_status fmm_cg_work_size(int32_t nmajor, int32_t r, size_t *bytes);
fmm_status fmm_cg_lines(const fmm_sparse *S, const void *F, int32_t r, int32_t dtype, const float *rhs,
                        float lambda, int32_t iters, float *X, float *work, size_t work_bytes, void *ws,
                        size_t ws_bytes, hipStream_t stream);

/*
 * Squared Frobenius residual of the factorisation on the observed entries (the ALS loss
 * of Section VI-E): *out = sum_p (val[p] - <A_i, B_j>)^2 over S's stored entries
 * (val = observed values; NULL means all ones), with the prediction an SDDMM on S's
 * pattern.  out is one device float64; the sum is accumulated in float64 in a fixed
 * order.  ws: fmm_residual_workspace() bytes.
 */
fmm_status fmm_residual_workspace(const fmm_sparse *S, size_t *bytes);
fmm_status fmm_sddmm_residual(const fmm_sparse *S_csr, const void *A, const void *B, int32_t r, int32_t dtype,
                              double *out, void *ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------- batched graphs */

/*
 * Many independent graphs in one persistent launch (fused forward and/or adjoint of
 * FusedMMA for every graph), optionally replayed from a captured hipGraph.  Each graph
 * g has its own S_g (CSR, and CSC for the adjoint), A_g, B_g, upstream gradient dC_g
 * and outputs; the operations are those of fmm_fusedmm_a / fmm_fusedmm_a_backward.
 *
 * The plan cuts every graph's lines into tiles of about tile_nnz stored entries,
 * assigns tiles to a fixed grid of workgroups (one resident wave set per CU) and keeps
 * the per-graph descriptor and tile tables in device memory it owns.  A workgroup copies
 * the column indices and weights of a tile of at most 2816 stored entries into LDS once,
 * so its batches read them there (same values, same results); larger tiles read them
 * from memory.  Schedules:
 *   - row-block: L lanes per line, several lines per wave;
 *   - wavefront-per-line: the 64 lanes of a wave share one line, each lane group
 *     taking every (64/L)-th batch of entries, partial sums added across groups;
 * Placements of the tiles on the grid (workgroup ids are dealt round-robin over the 8
 * XCDs of gfx950, each with its own L2):
 *   - FMM_BATCH_PLACE_GLOBAL: every tile to the least-loaded workgroup (LPT), fixed lists;
 *   - FMM_BATCH_PLACE_XCD: graphs go to XCDs by LPT and each graph's tiles to that XCD's
 *     workgroups, fixed lists;
 *   - FMM_BATCH_PLACE_QUEUES: graphs go to XCDs by LPT, and the workgroups of an XCD claim
 *     its tiles one at a time, in order, from a queue (a device counter), so the XCD
 *     works through one graph at a time while the graph's gathered rows sit in its L2
 *     (the cache blocking of Section III-A, at the level of the XCD's L2); a workgroup
 *     whose queue is drained claims from the next ones.  The forward and dA tiles of a
 *     line range are queued side by side, since both gather the same rows of B.  The
 *     last workgroup of a launch puts the counters back to zero, so launches of one plan
 *     (eager or replayed) must not overlap in time.
 * fmm_batch_autotune times candidate schedules with HIP events and keeps the fastest.
 * Results are deterministic for a fixed schedule (each line is computed by one tile, in a
 * fixed order, whichever workgroup claims it); with the row-block schedule they equal the
 * single-graph calls bit for bit under every placement.
 */
#define FMM_BATCH_FWD 1   /* compute C_g = FusedMMA(S_g, A_g, B_g)                        */
#define FMM_BATCH_BWD 2   /* compute dA_g, dB_g for upstream gradient dC_g                */
#define FMM_BATCH_DC_BF16 4 /* with FMM_BATCH_BWD and FMM_BF16: every dC_g is bfloat16     */
#define FMM_BATCH_PLACE_GLOBAL 0 /* placements (fmm_batch_set_schedule's xcd_aware)        */
#define FMM_BATCH_PLACE_XCD 1
#define FMM_BATCH_PLACE_QUEUES 2

typedef struct fmm_batch_graph {
    fmm_sparse csr;       /* rows x cols CSR descriptor of S_g (its split schedule is ignored) */
    fmm_sparse csc;       /* the stored transpose of S_g (required with FMM_BATCH_BWD)         */
    const void *A;        /* rows x r, storage dtype                                           */
    const void *B;        /* cols x r, storage dtype                                           */
    const void *dC;       /* rows x r upstream gradient (FMM_BATCH_BWD): float32, or bfloat16
                             with FMM_BATCH_DC_BF16                                            */
    void *C;              /* rows x r float32 output (FMM_BATCH_FWD)                           */
    void *dA;             /* rows x r float32 output (FMM_BATCH_BWD)                           */
    void *dB;             /* cols x r float32 output (FMM_BATCH_BWD)                           */
} fmm_batch_graph;

typedef struct fmm_batch_plan fmm_batch_plan;

typedef struct fmm_batch_info {
    int32_t tile_nnz;       /* target stored entries per tile                              */
    int32_t xcd_aware;      /* placement: FMM_BATCH_PLACE_GLOBAL, _XCD or _QUEUES           */
    int32_t lanes;          /* L                                                            */
    int32_t row_schedule;   /* 0 row-block, 1 wavefront-per-line (forward and dA passes)    */
    int32_t col_schedule;   /* same, for the dB column pass                                 */
    int32_t n_tiles;
    int32_t n_workgroups;
    int32_t n_candidates;   /* schedules the last autotune timed (0 = never tuned)          */
    float best_ms;          /* time of the chosen schedule in the last autotune             */
    int32_t graph_captured; /* 1 when a hipGraph of the current schedule is instantiated    */
} fmm_batch_info;

/*
 * Build a plan for nbatch graphs with common r and dtype (FMM_F32 or FMM_BF16 storage;
 * r % (16 / element size) == 0 and r <= 64 * 16 / element size).  flags: FMM_BATCH_FWD
 * and/or FMM_BATCH_BWD, plus FMM_BATCH_DC_BF16 (FMM_BF16 with FMM_BATCH_BWD only, else
 * FMM_ERR_UNSUPPORTED) when the upstream gradients are stored as bfloat16.  Synchronous: copies the pointer arrays of every graph to the
 * host to cut nnz-balanced tiles, then allocates and uploads the tables.  The default
 * schedule (before autotuning) is row-block, XCD-aware, tile_nnz 8192.  The graphs'
 * device buffers must stay valid for the life of the plan.  The plan also owns the
 * queue counters of FMM_BATCH_PLACE_QUEUES (zeroed here).
 */
fmm_status fmm_batch_plan_create(const fmm_batch_graph *graphs, int32_t nbatch, int32_t r, int32_t dtype,
                                 int32_t flags, fmm_batch_plan **plan);
/* Time every candidate schedule (each run overwrites the outputs with the same values)
   and keep the fastest.  Synchronous.  Invalidates a captured graph. */
fmm_status fmm_batch_autotune(fmm_batch_plan *plan, hipStream_t stream);
/* One persistent launch of the current schedule (eager). */
fmm_status fmm_batch_run(fmm_batch_plan *plan, hipStream_t stream);
/* Capture the current schedule's launch into a hipGraph and instantiate it.  stream must
   be a created (non-null) stream; nothing else may be enqueued on it meanwhile. */
fmm_status fmm_batch_capture(fmm_batch_plan *plan, hipStream_t stream);
/* Replay the captured graph on stream (FMM_ERR_STATE if none is current). */
fmm_status fmm_batch_launch(fmm_batch_plan *plan, hipStream_t stream);
fmm_status fmm_batch_plan_info(const fmm_batch_plan *plan, fmm_batch_info *info);
/* Force a schedule (as fmm_batch_autotune would pick it): tile_nnz >= 1, xcd_aware one of
   FMM_BATCH_PLACE_*, row/col schedule 0 (row-block) or 1 (wavefront-per-line);
   FMM_ERR_DIM otherwise.  Invalidates a captured graph. */
fmm_status fmm_batch_set_schedule(fmm_batch_plan *plan, int32_t tile_nnz, int32_t xcd_aware,
                                  int32_t row_schedule, int32_t col_schedule);
void fmm_batch_plan_destroy(fmm_batch_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* FMM_H */
