// Persistent kernel over many graphs: each workgroup walks its own list of tiles
// (graph, pass, line range) and runs the same per-line code as the single-graph
// kernels (process_line), so a row-block schedule reproduces them bit for bit (the
// operands it reads are the same, whether from LDS or from memory).
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

// Stored entries of a tile whose indices and weights are staged in LDS (24 KB per
// workgroup, so the 5 workgroups a CU holds fit its 160 KB).
constexpr int32_t kStageEntries = 3072;
// Workgroups per CU the persistent kernels are built for: 5 (5 waves per SIMD, at most 96
// registers), the occupancy their gathers need in flight, except with the row-block
// column pass, whose four two-row entries per batch need more registers than that.
constexpr int batch_blocks_per_cu(int gpl_c) { return gpl_c > 1 ? 5 : 4; }

// The lines of one tile, with the entry operands read through idx and val at positions
// relative to `base` (the tile's first entry when they are staged in LDS, else 0).
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__device__ __forceinline__ void run_lines(const BatchGraphDev &g, const BatchTile &tl, int32_t r,
                                          const int32_t *idx, const float *val, int32_t base)
{
    constexpr int UR = GPL_R > 1 ? 2 : 8;
    constexpr int UC = GPL_C > 1 ? 2 : 4;
    LineOperands o;
    o.idx = idx;
    o.val = val;
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
        o.G1 = g.B;
        o.G2 = g.B;
        for (int32_t line = tl.l0 + slot; line < tl.l1; line += LPB) {
            const int32_t b = g.rowptr[line] - base, e = g.rowptr[line + 1] - base;
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
        o.H = g.B;
        o.G1 = g.A;
        o.G2 = g.dC;
        for (int32_t line = tl.l0 + slot; line < tl.l1; line += LPB) {
            const int32_t b = g.colptr[line] - base, e = g.colptr[line + 1] - base;
            process_line<OP_FUSED2, TS, TS, TD, float, L, 1, VW, UC, GPL_C, false>(
                o, lane, gidx, line, b, e, g.dB + (size_t)line * r, false);
        }
    }
}

// One tile (graph, pass, line range) by the whole workgroup: every line of the range
// goes to a lane group (row-block) or a wave (wavefront-per-line), as in the
// single-graph kernels.  TS: storage of A and B; TD: storage of dC.
//
// A tile's entries are contiguous in the pass's orientation.  When they fit, the
// workgroup first copies their indices and weights to LDS (coalesced, once; weights of
// 1 for a pattern without values, the value an absent weight array stands for), so each
// batch of U entries reads its operands from LDS instead of waiting on a memory round
// trip before it can issue its row loads; the lines then run on entry positions
// relative to the tile.  The caller separates tiles with a barrier.
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__device__ __forceinline__ void run_tile(const BatchGraphDev *__restrict__ graphs, const BatchTile &tl, int32_t r,
                                         int32_t *s_idx, float *s_val)
{
    const BatchGraphDev &g = graphs[tl.graph];
    const bool rowp = tl.pass != PASS_BWD_COL;
    const int32_t *lptr = rowp ? g.rowptr : g.colptr;
    const int32_t *gidx = rowp ? g.colidx : g.rowidx;
    const float *gval = rowp ? g.val : g.valT;
    const int32_t first = lptr[tl.l0], count = lptr[tl.l1] - first;
    if (count <= kStageEntries) {  // the same for the whole workgroup
        for (int32_t k = threadIdx.x; k < count; k += kBlock) {
            s_idx[k] = gidx[first + k];
            s_val[k] = gval ? gval[first + k] : 1.0f;
        }
        __syncthreads();
        run_lines<TS, TD, L, VW, GPL_R, GPL_C>(g, tl, r, s_idx, s_val, first);
    } else {
        run_lines<TS, TD, L, VW, GPL_R, GPL_C>(g, tl, r, gidx, gval, 0);
    }
}

// Static placement: workgroup w runs tiles wg_off[w] .. wg_off[w + 1] - 1 in order.
template <class TS, class TD, int L, int VW, int GPL_R, int GPL_C>
__global__ __launch_bounds__(kBlock, batch_blocks_per_cu(GPL_C)) void batch_kernel(const BatchGraphDev *__restrict__ graphs,
                                                       const BatchTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ wg_off, int32_t r)
{
    __shared__ int32_t s_idx[kStageEntries];
    __shared__ float s_val[kStageEntries];
    const int32_t t0 = wg_off[blockIdx.x], t1 = wg_off[blockIdx.x + 1];
    for (int32_t t = t0; t < t1; ++t) {
        run_tile<TS, TD, L, VW, GPL_R, GPL_C>(graphs, tiles[t], r, s_idx, s_val);
        __syncthreads();  // the staged operands are overwritten by the next tile
    }
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
__global__ __launch_bounds__(kBlock, batch_blocks_per_cu(GPL_C)) void batch_queue_kernel(const BatchGraphDev *__restrict__ graphs,
                                                             const BatchTile *__restrict__ tiles,
                                                             const int32_t *__restrict__ q_off, int32_t *next,
                                                             int32_t n_q, int32_t r)
{
    __shared__ int32_t claimed;
    __shared__ int32_t s_idx[kStageEntries];
    __shared__ float s_val[kStageEntries];
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
            // the barriers above also keep a new tile's staging after the last tile's reads
            run_tile<TS, TD, L, VW, GPL_R, GPL_C>(graphs, tiles[t], r, s_idx, s_val);
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
