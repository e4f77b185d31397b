// Batched FusedMMA forward/adjoint over many graphs: plan construction (nnz-balanced
// tiles, XCD-aware or global LPT placement on a persistent grid), the autotuner,
// eager launch and hipGraph capture/replay.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <functional>
#include <queue>
#include <vector>

#include "batch_kernels.hpp"
#include "fmm.h"

using namespace fmm;

struct fmm_batch_plan {
    int32_t nbatch = 0, r = 0, dtype = 0, flags = 0;
    int32_t L = 0, vw = 0, ebytes = 0;
    int32_t num_cu = 0, n_xcd = 1;
    std::vector<BatchGraphDev> graphs;
    std::vector<std::vector<int32_t>> rowptr, colptr;
    BatchGraphDev *graphs_dev = nullptr;
    // current schedule
    int32_t tile_nnz = 8192, xcd = 1, rw = 0, cw = 0;
    BatchTile *tiles_dev = nullptr;
    int32_t *wgoff_dev = nullptr;  // per workgroup (static placement) or per queue (queues) tile offsets
    int32_t *qnext_dev = nullptr;  // queue counters plus the finished-workgroup count (zero between launches)
    int32_t n_tiles = 0, n_wg = 0;
    // tuning record
    int32_t n_candidates = 0;
    float best_ms = 0.f;
    // captured launch
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool captured = false;
};

namespace {

fmm_status hipfail(hipError_t e)
{
    set_last_hip_error((int32_t)e);
    return FMM_ERR_HIP;
}

#define BTRY(x)                                                                                  \
    do {                                                                                         \
        hipError_t _e = (x);                                                                     \
        if (_e != hipSuccess) return hipfail(_e);                                                \
    } while (0)

BatchKernelFn kernel_for(const fmm_batch_plan *p, int rw, int cw)
{
    if (p->dtype == FMM_BF16) {
        if (p->flags & FMM_BATCH_DC_BF16) return batch_kernel_for<bf16_t, bf16_t>(p->L, rw, cw);
        return batch_kernel_for<bf16_t, float>(p->L, rw, cw);
    }
    return batch_kernel_for<float, float>(p->L, rw, cw);
}

BatchQueueKernelFn queue_kernel_for(const fmm_batch_plan *p, int rw, int cw)
{
    if (p->dtype == FMM_BF16) {
        if (p->flags & FMM_BATCH_DC_BF16) return batch_queue_kernel_for<bf16_t, bf16_t>(p->L, rw, cw);
        return batch_queue_kernel_for<bf16_t, float>(p->L, rw, cw);
    }
    return batch_queue_kernel_for<float, float>(p->L, rw, cw);
}

// Kernel of a schedule, for occupancy queries.
const void *kernel_address(const fmm_batch_plan *p, int32_t placement, int rw, int cw)
{
    if (placement == FMM_BATCH_PLACE_QUEUES) return reinterpret_cast<const void *>(queue_kernel_for(p, rw, cw));
    return reinterpret_cast<const void *>(kernel_for(p, rw, cw));
}

struct TileCost {
    BatchTile t;
    double cost;
};

// Cut every pass of every graph into tiles of about tile_nnz entries; cost in bytes
// under the gather model (entries fetch rows; lines move their held row and output).
void cut_tiles(const fmm_batch_plan *p, int32_t tile_nnz, std::vector<std::vector<TileCost>> *per_graph)
{
    const double e = p->ebytes, r = p->r;
    const double ed = (p->flags & FMM_BATCH_DC_BF16) ? 2 : 4;  // bytes per element of dC
    per_graph->assign(p->nbatch, {});
    for (int32_t g = 0; g < p->nbatch; ++g) {
        for (int pass = 0; pass < 3; ++pass) {
            if (pass == PASS_FWD && !(p->flags & FMM_BATCH_FWD)) continue;
            if (pass != PASS_FWD && !(p->flags & FMM_BATCH_BWD)) continue;
            const std::vector<int32_t> &ptr = pass == PASS_BWD_COL ? p->colptr[g] : p->rowptr[g];
            const int32_t nl = (int32_t)ptr.size() - 1;
            const double per_entry = pass == PASS_BWD_COL ? (e + ed) * r + 8 : e * r + 8;
            const double per_line = pass == PASS_FWD ? (e + 4) * r : pass == PASS_BWD_ROW ? (ed + 4) * r : (e + 4) * r;
            int32_t l0 = 0;
            while (l0 < nl) {
                int32_t l1 = l0;
                int64_t ent = 0;
                while (l1 < nl && (ent < tile_nnz || l1 == l0)) {
                    ent += ptr[l1 + 1] - ptr[l1] + 1;
                    ++l1;
                }
                const int64_t stored = (int64_t)ptr[l1] - ptr[l0];
                TileCost tc;
                tc.t = BatchTile{g, pass, l0, l1};
                tc.cost = stored * per_entry + (l1 - l0) * per_line + 4096.0;
                (*per_graph)[g].push_back(tc);
                l0 = l1;
            }
        }
    }
}

// Graphs to XCDs by LPT on graph cost (largest first, each to the least-loaded XCD).
std::vector<std::vector<int32_t>> graphs_to_xcds(const fmm_batch_plan *p,
                                                 const std::vector<std::vector<TileCost>> &per_graph, int nx)
{
    std::vector<double> gcost(p->nbatch, 0.0);
    for (int32_t g = 0; g < p->nbatch; ++g)
        for (const TileCost &t : per_graph[g]) gcost[g] += t.cost;
    std::vector<int32_t> order(p->nbatch);
    for (int32_t g = 0; g < p->nbatch; ++g) order[g] = g;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return gcost[a] > gcost[b]; });
    std::vector<double> xload(nx, 0.0);
    std::vector<std::vector<int32_t>> xgraphs(nx);
    for (int32_t g : order) {
        const int x = (int)(std::min_element(xload.begin(), xload.end()) - xload.begin());
        xload[x] += gcost[g];
        xgraphs[x].push_back(g);
    }
    return xgraphs;
}

// Place tiles on n_wg workgroups.  XCD-aware: graphs go to XCDs by LPT on graph cost,
// then each graph's tiles go, in order, to the least-loaded workgroup of its XCD
// (workgroup w runs on XCD w % n_xcd), so the XCD works through its graphs one after
// another.  Otherwise: global LPT over all tiles.
void place_tiles(const fmm_batch_plan *p, const std::vector<std::vector<TileCost>> &per_graph, int32_t n_wg,
                 bool xcd, std::vector<BatchTile> *tiles, std::vector<int32_t> *wgoff)
{
    std::vector<std::vector<BatchTile>> lists(n_wg);
    typedef std::pair<double, int32_t> Load;  // (load, workgroup)
    if (xcd && p->n_xcd > 1 && n_wg % p->n_xcd == 0) {
        const int nx = p->n_xcd;
        const std::vector<std::vector<int32_t>> xgraphs = graphs_to_xcds(p, per_graph, nx);
        for (int x = 0; x < nx; ++x) {
            std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
            for (int32_t w = x; w < n_wg; w += nx) heap.push(Load(0.0, w));
            for (int32_t g : xgraphs[x]) {
                for (const TileCost &t : per_graph[g]) {
                    Load l = heap.top();
                    heap.pop();
                    lists[l.second].push_back(t.t);
                    l.first += t.cost;
                    heap.push(l);
                }
            }
        }
    } else {
        std::vector<TileCost> all;
        for (const auto &v : per_graph) all.insert(all.end(), v.begin(), v.end());
        std::stable_sort(all.begin(), all.end(), [](const TileCost &a, const TileCost &b) { return a.cost > b.cost; });
        std::priority_queue<Load, std::vector<Load>, std::greater<Load>> heap;
        for (int32_t w = 0; w < n_wg; ++w) heap.push(Load(0.0, w));
        for (const TileCost &t : all) {
            Load l = heap.top();
            heap.pop();
            lists[l.second].push_back(t.t);
            l.first += t.cost;
            heap.push(l);
        }
    }
    tiles->clear();
    wgoff->assign(n_wg + 1, 0);
    for (int32_t w = 0; w < n_wg; ++w) {
        (*wgoff)[w] = (int32_t)tiles->size();
        tiles->insert(tiles->end(), lists[w].begin(), lists[w].end());
    }
    (*wgoff)[n_wg] = (int32_t)tiles->size();
}

// Queues: one per XCD, holding its graphs (largest first) one after another.  Inside a
// graph the forward and dA tiles of the same line range sit side by side (both gather
// the same rows of B), then come the dB tiles.  qoff[q] .. qoff[q + 1] - 1 are queue q's.
void queue_tiles(const fmm_batch_plan *p, const std::vector<std::vector<TileCost>> &per_graph,
                 std::vector<BatchTile> *tiles, std::vector<int32_t> *qoff)
{
    const int nq = p->n_xcd;
    const std::vector<std::vector<int32_t>> xgraphs = graphs_to_xcds(p, per_graph, nq);
    tiles->clear();
    qoff->assign(nq + 1, 0);
    for (int q = 0; q < nq; ++q) {
        (*qoff)[q] = (int32_t)tiles->size();
        for (int32_t g : xgraphs[q]) {
            std::vector<BatchTile> rowp, colp;
            for (const TileCost &t : per_graph[g]) (t.t.pass == PASS_BWD_COL ? colp : rowp).push_back(t.t);
            std::stable_sort(rowp.begin(), rowp.end(), [](const BatchTile &a, const BatchTile &b) {
                return a.l0 != b.l0 ? a.l0 < b.l0 : a.pass < b.pass;
            });
            tiles->insert(tiles->end(), rowp.begin(), rowp.end());
            tiles->insert(tiles->end(), colp.begin(), colp.end());
        }
    }
    (*qoff)[nq] = (int32_t)tiles->size();
}

void release_graph(fmm_batch_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->captured = false;
}

// Build and upload the tables of a schedule; the grid is every CU times the resident
// workgroups of the schedule's kernel.
fmm_status apply_schedule(fmm_batch_plan *p, int32_t tile_nnz, int32_t placement, int32_t rw, int32_t cw)
{
    const void *fn = kernel_address(p, placement, rw, cw);
    if (!fn) return FMM_ERR_UNSUPPORTED;
    int per_cu = 0;
    BTRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0));
    if (per_cu < 1) per_cu = 1;
    const int32_t n_wg = p->num_cu * per_cu;
    std::vector<std::vector<TileCost>> per_graph;
    cut_tiles(p, tile_nnz, &per_graph);
    std::vector<BatchTile> tiles;
    std::vector<int32_t> off;
    if (placement == FMM_BATCH_PLACE_QUEUES) queue_tiles(p, per_graph, &tiles, &off);
    else place_tiles(p, per_graph, n_wg, placement == FMM_BATCH_PLACE_XCD, &tiles, &off);
    release_graph(p);
    // queue counters start from zero under every new schedule (each launch also leaves them
    // at zero; this also recovers from a launch that did not run to its end)
    BTRY(hipMemset(p->qnext_dev, 0, sizeof(int32_t) * (p->n_xcd + 1)));
    if (p->tiles_dev) BTRY(hipFree(p->tiles_dev));
    if (p->wgoff_dev) BTRY(hipFree(p->wgoff_dev));
    p->tiles_dev = nullptr;
    p->wgoff_dev = nullptr;
    BTRY(hipMalloc(&p->tiles_dev, std::max<size_t>(1, tiles.size()) * sizeof(BatchTile)));
    BTRY(hipMalloc(&p->wgoff_dev, off.size() * sizeof(int32_t)));
    if (!tiles.empty())
        BTRY(hipMemcpy(p->tiles_dev, tiles.data(), tiles.size() * sizeof(BatchTile), hipMemcpyHostToDevice));
    BTRY(hipMemcpy(p->wgoff_dev, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    p->tile_nnz = tile_nnz;
    p->xcd = placement;
    p->rw = rw;
    p->cw = cw;
    p->n_tiles = (int32_t)tiles.size();
    p->n_wg = n_wg;
    return FMM_OK;
}

hipError_t launch(fmm_batch_plan *p, hipStream_t s)
{
    const BatchGraphDev *g = p->graphs_dev;
    const BatchTile *t = p->tiles_dev;
    const int32_t *w = p->wgoff_dev;
    int32_t r = p->r;
    if (p->xcd == FMM_BATCH_PLACE_QUEUES) {
        BatchQueueKernelFn fn = queue_kernel_for(p, p->rw, p->cw);
        int32_t *next = p->qnext_dev;
        int32_t nq = p->n_xcd;
        void *args[] = {&g, &t, &w, &next, &nq, &r};
        return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(p->n_wg), dim3(kBlock), args, 0, s);
    }
    BatchKernelFn fn = kernel_for(p, p->rw, p->cw);
    void *args[] = {&g, &t, &w, &r};
    return hipLaunchKernel(reinterpret_cast<const void *>(fn), dim3(p->n_wg), dim3(kBlock), args, 0, s);
}

bool aligned16(const void *q) { return ((uintptr_t)q % 16) == 0; }

}  // namespace

extern "C" {

fmm_status fmm_batch_plan_create(const fmm_batch_graph *graphs, int32_t nbatch, int32_t r, int32_t dtype, int32_t flags,
                                 fmm_batch_plan **plan)
{
    if (!graphs || !plan) return FMM_ERR_NULL;
    *plan = nullptr;
    if (nbatch < 1) return FMM_ERR_DIM;
    if (!(flags & (FMM_BATCH_FWD | FMM_BATCH_BWD)) || (flags & ~(FMM_BATCH_FWD | FMM_BATCH_BWD | FMM_BATCH_DC_BF16)))
        return FMM_ERR_DIM;
    if ((flags & FMM_BATCH_DC_BF16) && (dtype != FMM_BF16 || !(flags & FMM_BATCH_BWD))) return FMM_ERR_UNSUPPORTED;
    int ebytes;
    if (dtype == FMM_F32) ebytes = 4;
    else if (dtype == FMM_BF16) ebytes = 2;
    else return FMM_ERR_DTYPE;
    const int vw = 16 / ebytes;
    if (r < vw || r % vw != 0 || r > 64 * vw) return FMM_ERR_DTYPE;
    int L = 4;
    while (L * vw < r) L <<= 1;
    const bool bwd = (flags & FMM_BATCH_BWD) != 0, fwd = (flags & FMM_BATCH_FWD) != 0;
    for (int32_t g = 0; g < nbatch; ++g) {
        const fmm_batch_graph &x = graphs[g];
        if (x.csr.orient != FMM_CSR) return FMM_ERR_ORIENT;
        if (x.csr.rows < 0 || x.csr.cols < 0 || x.csr.nnz < 0 || !x.csr.ptr) return FMM_ERR_DIM;
        if (x.csr.nnz > 0 && !x.csr.idx) return FMM_ERR_NULL;
        if (!x.A || !x.B) return FMM_ERR_NULL;
        if (!aligned16(x.A) || !aligned16(x.B)) return FMM_ERR_UNSUPPORTED;
        if (fwd && (!x.C || !aligned16(x.C))) return x.C ? FMM_ERR_UNSUPPORTED : FMM_ERR_NULL;
        if (bwd) {
            if (x.csc.orient != FMM_CSC) return FMM_ERR_ORIENT;
            if (x.csc.rows != x.csr.rows || x.csc.cols != x.csr.cols || x.csc.nnz != x.csr.nnz || !x.csc.ptr)
                return FMM_ERR_DIM;
            if (x.csc.nnz > 0 && !x.csc.idx) return FMM_ERR_NULL;
            if (!x.dC || !x.dA || !x.dB) return FMM_ERR_NULL;
            if (!aligned16(x.dC) || !aligned16(x.dA) || !aligned16(x.dB)) return FMM_ERR_UNSUPPORTED;
        }
    }
    fmm_batch_plan *p = new fmm_batch_plan();
    p->nbatch = nbatch;
    p->r = r;
    p->dtype = dtype;
    p->flags = flags;
    p->L = L;
    p->vw = vw;
    p->ebytes = ebytes;
    int dev = 0;
    hipDeviceProp_t prop;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) {
        delete p;
        return hipfail(e);
    }
    p->num_cu = prop.multiProcessorCount;
    // gfx950 deals workgroups round-robin over its 8 XCDs
    p->n_xcd = (strncmp(prop.gcnArchName, "gfx950", 6) == 0 && p->num_cu % 8 == 0) ? 8 : 1;
    p->graphs.resize(nbatch);
    p->rowptr.resize(nbatch);
    p->colptr.resize(nbatch);
    for (int32_t g = 0; g < nbatch; ++g) {
        const fmm_batch_graph &x = graphs[g];
        BatchGraphDev d;
        memset(&d, 0, sizeof(d));
        d.rowptr = x.csr.ptr;
        d.colidx = x.csr.idx;
        d.val = static_cast<const float *>(x.csr.val);
        d.A = x.A;
        d.B = x.B;
        d.C = static_cast<float *>(x.C);
        d.m = x.csr.rows;
        d.n = x.csr.cols;
        p->rowptr[g].resize((size_t)x.csr.rows + 1);
        e = hipMemcpy(p->rowptr[g].data(), x.csr.ptr, ((size_t)x.csr.rows + 1) * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && bwd) {
            d.colptr = x.csc.ptr;
            d.rowidx = x.csc.idx;
            d.valT = static_cast<const float *>(x.csc.val);
            d.dC = x.dC;
            d.dA = static_cast<float *>(x.dA);
            d.dB = static_cast<float *>(x.dB);
            p->colptr[g].resize((size_t)x.csc.cols + 1);
            e = hipMemcpy(p->colptr[g].data(), x.csc.ptr, ((size_t)x.csc.cols + 1) * 4, hipMemcpyDeviceToHost);
        }
        if (e != hipSuccess) {
            delete p;
            return hipfail(e);
        }
        p->graphs[g] = d;
    }
    e = hipMalloc(&p->graphs_dev, sizeof(BatchGraphDev) * nbatch);
    if (e == hipSuccess)
        e = hipMemcpy(p->graphs_dev, p->graphs.data(), sizeof(BatchGraphDev) * nbatch, hipMemcpyHostToDevice);
    // queue counters: zero here, and put back to zero by the last workgroup of every launch
    if (e == hipSuccess) e = hipMalloc(&p->qnext_dev, sizeof(int32_t) * (p->n_xcd + 1));
    if (e == hipSuccess) e = hipMemset(p->qnext_dev, 0, sizeof(int32_t) * (p->n_xcd + 1));
    if (e != hipSuccess) {
        fmm_batch_plan_destroy(p);
        return hipfail(e);
    }
    fmm_status st = apply_schedule(p, 8192, FMM_BATCH_PLACE_XCD, 0, 0);
    if (st != FMM_OK) {
        fmm_batch_plan_destroy(p);
        return st;
    }
    *plan = p;
    return FMM_OK;
}

fmm_status fmm_batch_set_schedule(fmm_batch_plan *p, int32_t tile_nnz, int32_t xcd_aware, int32_t row_schedule,
                                  int32_t col_schedule)
{
    if (!p) return FMM_ERR_NULL;
    if (tile_nnz < 1 || xcd_aware < FMM_BATCH_PLACE_GLOBAL || xcd_aware > FMM_BATCH_PLACE_QUEUES ||
        row_schedule < 0 || row_schedule > 1 || col_schedule < 0 || col_schedule > 1)
        return FMM_ERR_DIM;
    return apply_schedule(p, tile_nnz, xcd_aware, row_schedule, col_schedule);
}

fmm_status fmm_batch_run(fmm_batch_plan *p, hipStream_t stream)
{
    if (!p) return FMM_ERR_NULL;
    BTRY(launch(p, stream));
    return FMM_OK;
}

fmm_status fmm_batch_autotune(fmm_batch_plan *p, hipStream_t stream)
{
    if (!p) return FMM_ERR_NULL;
    // tiles up to 2560 entries keep their operands in LDS for lines of up to 256 entries
    const int32_t tiles_opts[4] = {1536, 2560, 8192, 32768};
    const int n_tiles_opts = 4;
    const bool row_pass = true;  // forward or dA pass is always present
    const bool col_pass = (p->flags & FMM_BATCH_BWD) != 0;
    const int wave_opts = p->L < 64 ? 2 : 1;  // at L = 64 both schedules coincide
    hipEvent_t e0, e1;
    BTRY(hipEventCreate(&e0));
    BTRY(hipEventCreate(&e1));
    float best = 1e30f;
    int32_t bt = p->tile_nnz, bx = p->xcd, brw = p->rw, bcw = p->cw;
    int32_t count = 0;
    fmm_status st = FMM_OK;
    for (int ti = 0; ti < n_tiles_opts && st == FMM_OK; ++ti) {
        for (int x = FMM_BATCH_PLACE_QUEUES; x >= FMM_BATCH_PLACE_GLOBAL && st == FMM_OK; --x) {
            for (int rw = 0; rw < (row_pass ? wave_opts : 1) && st == FMM_OK; ++rw) {
                for (int cw = 0; cw < (col_pass ? wave_opts : 1) && st == FMM_OK; ++cw) {
                    st = apply_schedule(p, tiles_opts[ti], x, rw, cw);
                    if (st != FMM_OK) break;
                    hipError_t e = launch(p, stream);  // warm-up
                    if (e == hipSuccess) e = hipEventRecord(e0, stream);
                    for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) e = launch(p, stream);
                    if (e == hipSuccess) e = hipEventRecord(e1, stream);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float ms = 0.f;
                    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                    if (e != hipSuccess) {
                        st = hipfail(e);
                        break;
                    }
                    ms /= 3.f;
                    ++count;
                    if (ms < best) {
                        best = ms;
                        bt = tiles_opts[ti];
                        bx = x;
                        brw = rw;
                        bcw = cw;
                    }
                }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != FMM_OK) return st;
    st = apply_schedule(p, bt, bx, brw, bcw);
    if (st != FMM_OK) return st;
    p->n_candidates = count;
    p->best_ms = best;
    return FMM_OK;
}

fmm_status fmm_batch_capture(fmm_batch_plan *p, hipStream_t stream)
{
    if (!p) return FMM_ERR_NULL;
    if (!stream) return FMM_ERR_UNSUPPORTED;  // the null stream cannot be captured
    release_graph(p);
    BTRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch(p, stream);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hipfail(e);
    }
    if (e2 != hipSuccess) return hipfail(e2);
    p->graph = g;
    BTRY(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    p->captured = true;
    return FMM_OK;
}

fmm_status fmm_batch_launch(fmm_batch_plan *p, hipStream_t stream)
{
    if (!p) return FMM_ERR_NULL;
    if (!p->captured) return FMM_ERR_STATE;
    BTRY(hipGraphLaunch(p->exec, stream));
    return FMM_OK;
}

fmm_status fmm_batch_plan_info(const fmm_batch_plan *p, fmm_batch_info *info)
{
    if (!p || !info) return FMM_ERR_NULL;
    info->tile_nnz = p->tile_nnz;
    info->xcd_aware = p->xcd;
    info->lanes = p->L;
    info->row_schedule = p->rw;
    info->col_schedule = p->cw;
    info->n_tiles = p->n_tiles;
    info->n_workgroups = p->n_wg;
    info->n_candidates = p->n_candidates;
    info->best_ms = p->best_ms;
    info->graph_captured = p->captured ? 1 : 0;
    return FMM_OK;
}

void fmm_batch_plan_destroy(fmm_batch_plan *p)
{
    if (!p) return;
    release_graph(p);
    if (p->tiles_dev) (void)hipFree(p->tiles_dev);
    if (p->wgoff_dev) (void)hipFree(p->wgoff_dev);
    if (p->graphs_dev) (void)hipFree(p->graphs_dev);
    if (p->qnext_dev) (void)hipFree(p->qnext_dev);
    delete p;
}

}  // extern "C"
