// Persistent kernel over many graphs: each workgroup walks its own list of tiles
// (graph, pass, line range) and runs the same per-line code as the single-graph
// kernels (process_line), so a row-block schedule reproduces them bit for bit.
#pragma once

#include "fmm_internal.hpp"

namespace fmm {

enum { PASS_FWD = 0, PASS_BWD_ROW = 1, PASS_BWD_COL = 2 };

struct BatchGraphDev {
    const int32_t *rowptr, *colidx;
    const float *val;
    const int32_t *colptr, *rowidx;
    const float *valT;
    const void *A, *B;
    const void *dC;  // TD elements (float32, or bfloat16 with a bfloat16 upstream gradient)
    float *C, *dA, *dB;
    int32_t m, n;
};

struct BatchTile {
    int32_t graph, pass, l0, l1;
};

// TS: storage of A and B; TD: storage of dC.
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchGraphDev *__restrict__ graphs,
                                                       const BatchTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ wg_off, int32_t r)
{
    constexpr int UR = GPL_R > 1 ? 2 : 8;
    constexpr int UC = GPL_C > 1 ? 2 : 4;
    const int32_t t0 = wg_off[blockIdx.x], t1 = wg_off[blockIdx.x + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const BatchTile tl = tiles[t];
        const BatchGraphDev &g = graphs[tl.graph];
        LineOperands o;
        o.wv1 = o.wv2 = nullptr;
        o.wperm = o.operm = nullptr;
        o.R = nullptr;
        o.r = r;
        o.beta = 0.0;
        if (tl.pass != PASS_BWD_COL) {
            constexpr int LPB = kBlock / (L * GPL_R);  // lines in flight per block
            const int lane = threadIdx.x % L;
            const int gidx = (threadIdx.x / L) % GPL_R;
            const int slot = threadIdx.x / (L * GPL_R);
            o.idx = g.colidx;
            o.val = g.val;
            o.G1 = g.B;
            o.G2 = g.B;
            for (int32_t line = tl.l0 + slot; line < tl.l1; line += LPB) {
                const int32_t b = g.rowptr[line], e = g.rowptr[line + 1];
                if (tl.pass == PASS_FWD) {
                    o.H = g.A;
                    process_line<OP_FUSED1, TS, TS, TS, float, L, 1, VW, UR, GPL_R, false>(
                        o, lane, gidx, line, b, e, g.C + (size_t)line * r, false);
                } else {
                    o.H = g.dC;
                    process_line<OP_FUSED1, TD, TS, TS, float, L, 1, VW, UR, GPL_R, false>(
                        o, lane, gidx, line, b, e, g.dA + (size_t)line * r, false);
                }
            }
        } else {
            constexpr int LPB = kBlock / (L * GPL_C);
            const int lane = threadIdx.x % L;
            const int gidx = (threadIdx.x / L) % GPL_C;
            const int slot = threadIdx.x / (L * GPL_C);
            o.idx = g.rowidx;
            o.val = g.valT;
            o.H = g.B;
            o.G1 = g.A;
            o.G2 = g.dC;
            for (int32_t line = tl.l0 + slot; line < tl.l1; line += LPB) {
                const int32_t b = g.colptr[line], e = g.colptr[line + 1];
                process_line<OP_FUSED2, TS, TS, TD, float, L, 1, VW, UC, GPL_C, false>(
                    o, lane, gidx, line, b, e, g.dB + (size_t)line * r, false);
            }
        }
    }
}

// Host-side launcher table for one storage type: (L, row schedule, column schedule).
typedef void (*BatchKernelFn)(const BatchGraphDev *, const BatchTile *, const int32_t *, int32_t);

template <class TS, class TD> BatchKernelFn batch_kernel_for(int L, int row_wave, int col_wave);

}  // namespace fmm
