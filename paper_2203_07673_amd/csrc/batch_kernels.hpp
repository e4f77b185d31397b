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

// One tile (graph, pass, line range) by the whole workgroup: every line of the range
// goes to a lane group (row-block) or a wave (wavefront-per-line), as in the
// single-graph kernels.  TS: storage of A and B; TD: storage of dC.
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__device__ __forceinline__ void run_tile(const BatchGraphDev *__restrict__ graphs, const BatchTile &tl, int32_t r)
{
    constexpr int UR = GPL_R > 1 ? 2 : 8;
    constexpr int UC = GPL_C > 1 ? 2 : 4;
    const BatchGraphDev &g = graphs[tl.graph];
    LineOperands o;
    o.wv1 = o.wv2 = nullptr;
    o.wperm = o.operm = nullptr;
    o.hot = nullptr;
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

// Static placement: workgroup w runs tiles wg_off[w] .. wg_off[w + 1] - 1 in order.
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__global__ __launch_bounds__(kBlock) void batch_kernel(const BatchGraphDev *__restrict__ graphs,
                                                       const BatchTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ wg_off, int32_t r)
{
    const int32_t t0 = wg_off[blockIdx.x], t1 = wg_off[blockIdx.x + 1];
    for (int32_t t = t0; t < t1; ++t) run_tile<TS, TD, L, VW, GPL_R, GPL_C>(graphs, tiles[t], r);
}

// Queues per XCD: queue q holds tiles q_off[q] .. q_off[q + 1] - 1 (its graphs one after
// another), and the workgroups of XCD q (ids dealt round-robin over the n_q XCDs) claim
// them in order through the counter next[q], so an XCD works through one graph at a time
// while the graph's gathered rows sit in its L2.  A workgroup whose queue is drained
// moves on to the following queues (work stealing for the tail).  Every claim past a
// queue's end fails without effect, so each workgroup stops after at most one failed
// claim per queue; the last workgroup to finish (counted in next[n_q]) puts the counters
// back to zero for the next launch.  Launches of one plan must not overlap in time.
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__global__ __launch_bounds__(kBlock) void batch_queue_kernel(const BatchGraphDev *__restrict__ graphs,
                                                             const BatchTile *__restrict__ tiles,
                                                             const int32_t *__restrict__ q_off, int32_t *next,
                                                             int32_t n_q, int32_t r)
{
    __shared__ int32_t claimed;
    const int32_t home = (int32_t)(blockIdx.x % (uint32_t)n_q);
    for (int32_t k = 0; k < n_q; ++k) {
        const int32_t q = home + k < n_q ? home + k : home + k - n_q;
        const int32_t b = q_off[q], e = q_off[q + 1];
        for (;;) {
            if (threadIdx.x == 0) {
                const int32_t i = __hip_atomic_fetch_add(next + q, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                claimed = i < e - b ? b + i : -1;
            }
            __syncthreads();
            const int32_t t = claimed;
            __syncthreads();  // every wave has read the claim before the next one overwrites it
            if (t < 0) break;
            run_tile<TS, TD, L, VW, GPL_R, GPL_C>(graphs, tiles[t], r);
        }
    }
    if (threadIdx.x == 0) {
        const int32_t done = __hip_atomic_fetch_add(next + n_q, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (done == (int32_t)gridDim.x - 1) {
            for (int32_t q = 0; q <= n_q; ++q) __hip_atomic_store(next + q, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Host-side launcher tables for one storage type: (L, row schedule, column schedule).
typedef void (*BatchKernelFn)(const BatchGraphDev *, const BatchTile *, const int32_t *, int32_t);
typedef void (*BatchQueueKernelFn)(const BatchGraphDev *, const BatchTile *, const int32_t *, int32_t *, int32_t,
                                   int32_t);

template <class TS, class TD> BatchKernelFn batch_kernel_for(int L, int row_wave, int col_wave);
template <class TS, class TD> BatchQueueKernelFn batch_queue_kernel_for(int L, int row_wave, int col_wave);

}  // namespace fmm
