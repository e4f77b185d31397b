// Host-side declarations shared by the C-ABI layer and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fmm.h"
#include "fmm_lines.hpp"

namespace fmm {

// Storage-driven vector width: elements per 16-byte load of A/B (F32: 4, BF16: 8, F64: 2).
enum Path { PATH_F32 = 0, PATH_BF16 = 1, PATH_F64 = 2 };

// Lane-group shapes the line kernels are built for (L lanes per line, NV vectors per lane).
struct Shape {
    int L, NV;
};

// Chosen by the launcher from r (and the vector width vw) unless a valid hint is given.
// A shape is supported when it is one of the compiled ones and L * NV vectors of vw
// elements cover r.
Shape default_shape(int r, int vw);
bool shape_supported(Shape s, int r, int vw);
int max_r(int path, int r);  // 0 when r is not supported for the dtype path

// Tuning knobs (process-wide; set through fmm_set_tuning for experiments and the autotuner).
struct Tuning {
    int lanes;  // 0 = automatic
    int nv;     // 0 = automatic
};
Tuning &tuning();

// Record the hipError_t that fmm_last_hip_error() reports for this thread.
void set_last_hip_error(int32_t e);

// One launch of a line kernel (plus the merge of split lines for the accumulating ops).
// Instantiated in lines_<dtype>.hip for the type combinations the C ABI uses.
template <int OP, class TH, class TG1, class TG2, class Acc>
hipError_t launch_lines(const LineArgs &a, int32_t n_splits, const int32_t *splits, Shape hint,
                        hipStream_t stream);

// Gram operator of each major line of S on the pattern alone (api.hip):
// out_line = sum_j <H_line, G_j> G_j.
fmm_status gram_apply(const fmm_sparse *S, const float *H, const void *G, int32_t r, int32_t dtype, float *out,
                      void *ws, size_t ws_bytes, hipStream_t st);
fmm_status gram_cg_step(const fmm_sparse *S, float *P, const void *G, int32_t r, int32_t dtype, float lambda,
                        float *X, float *R, float *rr, hipStream_t st);

// Pattern preparation kernels (pattern.hip).
size_t scan_workspace_bytes(int64_t n);
hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s);
size_t transpose_workspace_bytes(int64_t m, int64_t n, int64_t nnz);
hipError_t csr_to_csc(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colidx,
                      const void *val, int val_bytes, int32_t *colptr, int32_t *rowidx, void *valT,
                      int32_t *perm, void *ws, hipStream_t s);
hipError_t validate(int32_t nmajor, int32_t nminor, int32_t nnz, const int32_t *ptr, const int32_t *idx,
                    int32_t *flag_dev, hipStream_t s);
hipError_t gather_values(const int32_t *perm, const void *src, void *dst, int32_t nnz, int val_bytes, hipStream_t s);
hipError_t gather_hints(const int32_t *idx, const int32_t *minor_ptr, int32_t nnz, int32_t min_len, uint8_t *hot,
                        hipStream_t s);
size_t line_order_workspace_bytes(int64_t nlines);
hipError_t line_order(const int32_t *ptr, int32_t nlines, int32_t long_len, int32_t *order, void *ws, hipStream_t s);
size_t schedule_workspace_bytes(int64_t nmajor);
hipError_t schedule_count(const int32_t *ptr, int32_t nmajor, int32_t long_len, int32_t chunk, int32_t *totals_host,
                          void *ws, hipStream_t s);
hipError_t schedule_fill(const int32_t *ptr, int32_t nmajor, int32_t long_len, int32_t chunk, int32_t *chunks,
                         int32_t *splits, void *ws, hipStream_t s);
hipError_t f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t s);

}  // namespace fmm
