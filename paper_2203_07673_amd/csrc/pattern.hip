// Pattern preparation on the GPU: canonical-form check, the stored transposed copy
// of S (Section IV-B: FusedMMB and the column passes run on it), the split schedule
// for long lines, and float32 -> bfloat16 storage rounding.  All integer work is
// deterministic: the transpose is a stable LSD radix sort of (column, CSR position)
// pairs, so rows come out ascending inside each column without any atomics on the
// output order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fmm_internal.hpp"

namespace fmm {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;  // 2048

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 16;
constexpr int kSortTile = kSortThreads * kSortRounds;  // 4096 items per block

__device__ __forceinline__ int32_t wave_incl_scan(int32_t x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan of the block's thread totals; returns the thread's offset and the
// block total through *total.
__device__ int32_t block_excl_scan(int32_t x, int32_t *total)
{
    __shared__ int32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < kScanThreads / 64; ++i) {
        if (i < w) before += wsum[i];
        all += wsum[i];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

__global__ __launch_bounds__(kScanThreads) void scan_reduce_kernel(const int32_t *__restrict__ in, int64_t n,
                                                                   int32_t *__restrict__ sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    int32_t total;
    block_excl_scan(s, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void scan_apply_kernel(const int32_t *__restrict__ in, int64_t n,
                                                                  const int32_t *__restrict__ block_off,
                                                                  int32_t *__restrict__ out)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int32_t v[kScanItems];
    int32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0;
        s += v[i];
    }
    int32_t total;
    int32_t run = block_excl_scan(s, &total) + (block_off ? block_off[blockIdx.x] : 0);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
}

// ------------------------------------------------------------------ radix sort

__global__ __launch_bounds__(kSortThreads) void radix_hist_kernel(const int32_t *__restrict__ keys, int64_t n,
                                                                  int shift, int32_t *__restrict__ hist, int32_t nb)
{
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int rd = 0; rd < kSortRounds; ++rd) {
        const int64_t q = base + (int64_t)rd * kSortThreads + threadIdx.x;
        if (q < n) atomicAdd(&cnt[(keys[q] >> shift) & 0xFF], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one 8-bit digit.  Items of the tile are taken in order, 256 at
// a time; inside a wave the rank among equal digits comes from ballots, across the
// block's four waves from per-wave digit counts in LDS, across rounds from a running
// per-digit count, and across tiles from the digit-major exclusive scan `off`.
__global__ __launch_bounds__(kSortThreads) void radix_scatter_kernel(
    const int32_t *__restrict__ kin, const int32_t *__restrict__ vin, int32_t *__restrict__ kout,
    int32_t *__restrict__ vout, int64_t n, int shift, const int32_t *__restrict__ off, int32_t nb)
{
    __shared__ int32_t wcnt[kSortThreads / 64][256];
    __shared__ int32_t run[256];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    run[t] = off[(int64_t)t * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    for (int rd = 0; rd < kSortRounds; ++rd) {
        for (int i = t; i < (kSortThreads / 64) * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
        __syncthreads();
        const int64_t q = base + (int64_t)rd * kSortThreads + t;
        const bool valid = q < n;
        const int32_t key = valid ? kin[q] : 0;
        const int32_t v = valid ? (vin ? vin[q] : (int32_t)q) : 0;
        const int d = (key >> shift) & 0xFF;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int32_t pos = run[d] + rank;
            for (int w2 = 0; w2 < w; ++w2) pos += wcnt[w2][d];
            kout[pos] = key;
            vout[pos] = v;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int w2 = 0; w2 < kSortThreads / 64; ++w2) add += wcnt[w2][t];
        run[t] += add;
        __syncthreads();
    }
}

// After the sort: perm[q] = CSR position of the q-th CSC entry, rowidx[q] = its row
// (found by binary search in rowptr), valT[q] = val[perm[q]], and colptr from the
// boundaries of the sorted column keys (empty columns take the next boundary).
__global__ __launch_bounds__(256) void transpose_finish_kernel(
    const int32_t *__restrict__ skeys, const int32_t *__restrict__ svals, int32_t m, int32_t n, int32_t nnz,
    const int32_t *__restrict__ rowptr, const void *__restrict__ val, int val_bytes, int32_t *__restrict__ colptr,
    int32_t *__restrict__ rowidx, void *__restrict__ valT, int32_t *__restrict__ perm)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q > nnz) return;
    const int32_t k = q < nnz ? skeys[q] : n;
    const int32_t kp = q > 0 ? skeys[q - 1] : -1;
    for (int32_t c = kp + 1; c <= k; ++c) colptr[c] = (int32_t)q;
    if (q == nnz) return;
    const int32_t p = svals ? svals[q] : (int32_t)q;
    int32_t lo = 0, hi = m;  // largest i with rowptr[i] <= p
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (rowptr[mid] <= p) lo = mid; else hi = mid;
    }
    perm[q] = p;
    rowidx[q] = lo;
    if (val && valT) {
        if (val_bytes == 8)
            static_cast<double *>(valT)[q] = static_cast<const double *>(val)[p];
        else
            static_cast<float *>(valT)[q] = static_cast<const float *>(val)[p];
    }
}

// ------------------------------------------------------------------ validation

__global__ __launch_bounds__(256) void validate_ptr_kernel(int32_t nmajor, int32_t nnz, const int32_t *__restrict__ ptr,
                                                           int32_t *__restrict__ flag)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i > nmajor) return;
    bool bad = false;
    if (i == 0) bad |= ptr[0] != 0;
    if (i == nmajor) bad |= ptr[nmajor] != nnz;
    if (i < nmajor) bad |= ptr[i] > ptr[i + 1];
    if (bad) atomicOr(flag, 1);
}

__global__ __launch_bounds__(256) void validate_idx_kernel(int32_t nmajor, int32_t nminor, int32_t nnz,
                                                           const int32_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ idx, int32_t *__restrict__ flag)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nnz) return;
    int32_t lo = 0, hi = nmajor;  // line of p: largest i with ptr[i] <= p
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if (ptr[mid] <= p) lo = mid; else hi = mid;
    }
    const int32_t j = idx[p];
    if (j < 0 || j >= nminor) atomicOr(flag, 1);
    else if (p > ptr[lo] && idx[p - 1] >= j) atomicOr(flag, 2);
}

// ------------------------------------------------------------------ value permutation

template <class T>
__global__ __launch_bounds__(256) void gather_values_kernel(const int32_t *__restrict__ perm, const T *__restrict__ src,
                                                            T *__restrict__ dst, int32_t nnz)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q < nnz) dst[q] = src[perm[q]];
}

// ------------------------------------------------------------------ line order

constexpr int32_t kOrderCap = 1023;   // lengths at or above this sort as equal
constexpr int32_t kOrderLong = 1024;  // key of lines the split schedule processes as chunks
constexpr int kOrderBits = 11;        // keys lie in [0, kOrderLong]

// Sort key of each line: shorter lines get larger keys (so an ascending stable sort
// yields decreasing length), lines longer than long_len the largest.
__global__ __launch_bounds__(256) void line_key_kernel(const int32_t *__restrict__ ptr, int32_t nlines,
                                                       int32_t long_len, int32_t *__restrict__ key)
{
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= nlines) return;
    const int32_t len = ptr[l + 1] - ptr[l];
    key[l] = len > long_len ? kOrderLong : kOrderCap - (len < kOrderCap ? len : kOrderCap);
}

// ------------------------------------------------------------------ split schedule

__global__ __launch_bounds__(256) void sched_count_kernel(const int32_t *__restrict__ ptr, int32_t nmajor, int32_t long_len,
                                                          int32_t chunk, int32_t *__restrict__ nch,
                                                          int32_t *__restrict__ issplit)
{
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l > nmajor) return;
    int32_t c = 0;
    if (l < nmajor) {
        const int32_t len = ptr[l + 1] - ptr[l];
        c = len > long_len ? (len + chunk - 1) / chunk : 0;
    }
    nch[l] = c;
    issplit[l] = c > 0;
}

__global__ __launch_bounds__(256) void sched_fill_kernel(const int32_t *__restrict__ ptr, int32_t nmajor, int32_t chunk,
                                                         const int32_t *__restrict__ nch,
                                                         const int32_t *__restrict__ choff,
                                                         const int32_t *__restrict__ spoff,
                                                         int32_t *__restrict__ chunks, int32_t *__restrict__ splits)
{
    const int64_t l = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (l >= nmajor) return;
    const int32_t c = nch[l];
    if (c == 0) return;
    const int32_t s = spoff[l], first = choff[l];
    splits[3 * s] = (int32_t)l;
    splits[3 * s + 1] = first;
    splits[3 * s + 2] = c;
    const int32_t b = ptr[l], e = ptr[l + 1];
    for (int32_t k = 0; k < c; ++k) {
        const int32_t cb = b + k * chunk;
        chunks[3 * (first + k)] = (int32_t)l;
        chunks[3 * (first + k) + 1] = cb;
        chunks[3 * (first + k) + 2] = min(e, cb + chunk);
    }
}

// ------------------------------------------------------------------ bfloat16 storage

__device__ inline uint32_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7FC0u;  // canonical quiet NaN
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;                               // nearest, ties to even
}

// Elements [begin, n), one per thread.
__global__ __launch_bounds__(256) void f32_to_bf16_kernel(const float *__restrict__ x, uint16_t *__restrict__ y,
                                                          int64_t begin, int64_t n)
{
    const int64_t i = begin + (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    y[i] = (uint16_t)bf16_bits(x[i]);
}

// Groups of 8 elements (two 16-byte loads, one 16-byte store); x and y 16-byte aligned.
__global__ __launch_bounds__(256) void f32_to_bf16_x8_kernel(const float4 *__restrict__ x, uint4 *__restrict__ y,
                                                             int64_t groups)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (g >= groups) return;
    const float4 a = x[2 * g], b = x[2 * g + 1];
    uint4 o;
    o.x = bf16_bits(a.x) | (bf16_bits(a.y) << 16);
    o.y = bf16_bits(a.z) | (bf16_bits(a.w) << 16);
    o.z = bf16_bits(b.x) | (bf16_bits(b.y) << 16);
    o.w = bf16_bits(b.z) | (bf16_bits(b.w) << 16);
    y[g] = o;
}

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

// ------------------------------------------------------------------ host wrappers

size_t scan_workspace_bytes(int64_t n)
{
    size_t total = 0;
    while (n > kScanTile) {
        const int64_t nb = (n + kScanTile - 1) / kScanTile;
        total += 2 * align256((size_t)nb * sizeof(int32_t));  // block sums and their scan
        n = nb;
    }
    return total;
}

hipError_t exclusive_scan_i32(const int32_t *in, int32_t *out, int64_t n, void *ws, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    if (n <= kScanTile) {
        hipLaunchKernelGGL(scan_apply_kernel, dim3(1), dim3(kScanThreads), 0, s, in, n, (const int32_t *)nullptr, out);
        return hipGetLastError();
    }
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    int32_t *sums = static_cast<int32_t *>(ws);
    int32_t *sums_scan = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + align256((size_t)nb * 4));
    void *rest = static_cast<char *>(ws) + 2 * align256((size_t)nb * 4);
    hipLaunchKernelGGL(scan_reduce_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = exclusive_scan_i32(sums, sums_scan, nb, rest, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_apply_kernel, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n,
                       (const int32_t *)sums_scan, out);
    return hipGetLastError();
}

static int key_bits(int64_t n)
{
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
    return bits;  // keys lie in [0, n) and need this many bits
}

size_t transpose_workspace_bytes(int64_t m, int64_t n, int64_t nnz)
{
    (void)m;
    const int64_t nb = (nnz + kSortTile - 1) / kSortTile;
    size_t b = 4 * align256((size_t)nnz * 4);              // two key/value ping-pong pairs
    b += 2 * align256((size_t)(256 * nb) * 4);              // histogram and its scan
    b += scan_workspace_bytes(256 * nb);
    (void)n;
    return b + 256;
}

hipError_t csr_to_csc(int32_t m, int32_t n, int32_t nnz, const int32_t *rowptr, const int32_t *colidx,
                      const void *val, int val_bytes, int32_t *colptr, int32_t *rowidx, void *valT,
                      int32_t *perm, void *ws, hipStream_t s)
{
    const int64_t nb = (nnz + kSortTile - 1) / kSortTile;
    char *w = static_cast<char *>(ws);
    int32_t *ka = reinterpret_cast<int32_t *>(w); w += align256((size_t)nnz * 4);
    int32_t *va = reinterpret_cast<int32_t *>(w); w += align256((size_t)nnz * 4);
    int32_t *kb = reinterpret_cast<int32_t *>(w); w += align256((size_t)nnz * 4);
    int32_t *vb = reinterpret_cast<int32_t *>(w); w += align256((size_t)nnz * 4);
    int32_t *hist = reinterpret_cast<int32_t *>(w); w += align256((size_t)(256 * nb) * 4);
    int32_t *hoff = reinterpret_cast<int32_t *>(w); w += align256((size_t)(256 * nb) * 4);
    void *scan_ws = w;
    hipError_t e;

    const int bits = key_bits(n);
    const int passes = (bits + 7) / 8;
    const int32_t *kin = colidx;
    const int32_t *vin = nullptr;  // identity: CSR positions
    int32_t *kout = ka, *vout = va;
    for (int pass = 0; pass < passes && nnz > 0; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kin, (int64_t)nnz, shift,
                           hist, (int32_t)nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan_i32(hist, hoff, 256 * nb, scan_ws, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kin, vin, kout, vout,
                           (int64_t)nnz, shift, (const int32_t *)hoff, (int32_t)nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        vin = vout;
        kout = (kout == ka) ? kb : ka;
        vout = (vout == va) ? vb : va;
    }
    // with no pass (n <= 1, or nnz == 0) the keys are colidx itself and CSR order is
    // already column order, so the finish kernel reads the identity (svals == NULL)
    const int32_t *skeys = kin;
    const int32_t *svals = vin;
    const int64_t tb = ((int64_t)nnz + 1 + 255) / 256;
    hipLaunchKernelGGL(transpose_finish_kernel, dim3((unsigned)tb), dim3(256), 0, s, skeys, svals, m, n, nnz, rowptr,
                       val, val_bytes, colptr, rowidx, valT, perm);
    return hipGetLastError();
}

hipError_t validate(int32_t nmajor, int32_t nminor, int32_t nnz, const int32_t *ptr, const int32_t *idx,
                    int32_t *flag_dev, hipStream_t s)
{
    hipLaunchKernelGGL(validate_ptr_kernel, dim3((unsigned)((nmajor + 1 + 255) / 256)), dim3(256), 0, s, nmajor, nnz, ptr,
                       flag_dev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    int32_t f = 0;
    if ((e = hipMemcpyAsync(&f, flag_dev, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
    if (f != 0 || nnz == 0) return hipSuccess;  // bad ptr: idx pass would search a broken ptr
    hipLaunchKernelGGL(validate_idx_kernel, dim3((unsigned)(((int64_t)nnz + 255) / 256)), dim3(256), 0, s, nmajor, nminor,
                       nnz, ptr, idx, flag_dev);
    return hipGetLastError();
}

hipError_t gather_values(const int32_t *perm, const void *src, void *dst, int32_t nnz, int val_bytes, hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    const dim3 grid((unsigned)(((int64_t)nnz + 255) / 256));
    if (val_bytes == 8)
        hipLaunchKernelGGL(gather_values_kernel<double>, grid, dim3(256), 0, s, perm, static_cast<const double *>(src),
                           static_cast<double *>(dst), nnz);
    else
        hipLaunchKernelGGL(gather_values_kernel<float>, grid, dim3(256), 0, s, perm, static_cast<const float *>(src),
                           static_cast<float *>(dst), nnz);
    return hipGetLastError();
}

// hot[p] = 1 when minor line idx[p] has at least min_len entries (its length read from
// the other orientation's pointer array), else 0.
__global__ __launch_bounds__(256) void gather_hints_kernel(const int32_t *__restrict__ idx,
                                                           const int32_t *__restrict__ minor_ptr, int32_t nnz,
                                                           int32_t min_len, uint8_t *__restrict__ hot)
{
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= nnz) return;
    const int32_t j = idx[p];
    hot[p] = (minor_ptr[j + 1] - minor_ptr[j]) >= min_len ? 1 : 0;
}

hipError_t gather_hints(const int32_t *idx, const int32_t *minor_ptr, int32_t nnz, int32_t min_len, uint8_t *hot,
                        hipStream_t s)
{
    if (nnz <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_hints_kernel, dim3((unsigned)(((int64_t)nnz + 255) / 256)), dim3(256), 0, s, idx,
                       minor_ptr, nnz, min_len, hot);
    return hipGetLastError();
}

size_t line_order_workspace_bytes(int64_t nlines)
{
    const int64_t nb = (nlines + kSortTile - 1) / kSortTile;
    size_t b = 4 * align256((size_t)nlines * 4);             // keys, then one key/value pair and one key buffer
    b += 2 * align256((size_t)(256 * nb) * 4);               // histogram and its scan
    b += scan_workspace_bytes(256 * nb);
    return b + 256;
}

hipError_t line_order(const int32_t *ptr, int32_t nlines, int32_t long_len, int32_t *order, void *ws, hipStream_t s)
{
    if (nlines <= 0) return hipSuccess;
    const int64_t nb = (nlines + kSortTile - 1) / kSortTile;
    char *w = static_cast<char *>(ws);
    int32_t *key = reinterpret_cast<int32_t *>(w); w += align256((size_t)nlines * 4);
    int32_t *ka = reinterpret_cast<int32_t *>(w); w += align256((size_t)nlines * 4);
    int32_t *va = reinterpret_cast<int32_t *>(w); w += align256((size_t)nlines * 4);
    int32_t *kb = reinterpret_cast<int32_t *>(w); w += align256((size_t)nlines * 4);
    int32_t *hist = reinterpret_cast<int32_t *>(w); w += align256((size_t)(256 * nb) * 4);
    int32_t *hoff = reinterpret_cast<int32_t *>(w); w += align256((size_t)(256 * nb) * 4);
    void *scan_ws = w;
    hipLaunchKernelGGL(line_key_kernel, dim3((unsigned)(((int64_t)nlines + 255) / 256)), dim3(256), 0, s, ptr, nlines,
                       long_len, key);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // two stable 8-bit passes (keys have kOrderBits <= 16 bits); values start as the identity
    static_assert(kOrderBits <= 16, "two radix passes");
    const int32_t *kin = key;
    const int32_t *vin = nullptr;
    int32_t *kouts[2] = {ka, kb};
    int32_t *vouts[2] = {va, order};
    for (int pass = 0; pass < 2; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(radix_hist_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kin, (int64_t)nlines, shift,
                           hist, (int32_t)nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan_i32(hist, hoff, 256 * nb, scan_ws, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3((unsigned)nb), dim3(kSortThreads), 0, s, kin, vin, kouts[pass],
                           vouts[pass], (int64_t)nlines, shift, (const int32_t *)hoff, (int32_t)nb);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kouts[pass];
        vin = vouts[pass];
    }
    return hipSuccess;
}

size_t schedule_workspace_bytes(int64_t nmajor)
{
    return 4 * align256((size_t)(nmajor + 1) * 4) + scan_workspace_bytes(nmajor + 1) + 256;
}

static void sched_bufs(void *ws, int64_t nmajor, int32_t **nch, int32_t **choff, int32_t **iss, int32_t **spoff,
                       void **scan_ws)
{
    char *w = static_cast<char *>(ws);
    const size_t b = align256((size_t)(nmajor + 1) * 4);
    *nch = reinterpret_cast<int32_t *>(w);
    *choff = reinterpret_cast<int32_t *>(w + b);
    *iss = reinterpret_cast<int32_t *>(w + 2 * b);
    *spoff = reinterpret_cast<int32_t *>(w + 3 * b);
    *scan_ws = w + 4 * b;
}

hipError_t schedule_count(const int32_t *ptr, int32_t nmajor, int32_t long_len, int32_t chunk, int32_t *totals_host,
                          void *ws, hipStream_t s)
{
    int32_t *nch, *choff, *iss, *spoff;
    void *scan_ws;
    sched_bufs(ws, nmajor, &nch, &choff, &iss, &spoff, &scan_ws);
    hipLaunchKernelGGL(sched_count_kernel, dim3((unsigned)((nmajor + 1 + 255) / 256)), dim3(256), 0, s, ptr, nmajor,
                       long_len, chunk, nch, iss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = exclusive_scan_i32(nch, choff, nmajor + 1, scan_ws, s)) != hipSuccess) return e;
    if ((e = exclusive_scan_i32(iss, spoff, nmajor + 1, scan_ws, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&totals_host[0], choff + nmajor, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(&totals_host[1], spoff + nmajor, 4, hipMemcpyDeviceToHost, s)) != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

hipError_t schedule_fill(const int32_t *ptr, int32_t nmajor, int32_t long_len, int32_t chunk, int32_t *chunks,
                         int32_t *splits, void *ws, hipStream_t s)
{
    int32_t *nch, *choff, *iss, *spoff;
    void *scan_ws;
    sched_bufs(ws, nmajor, &nch, &choff, &iss, &spoff, &scan_ws);
    hipLaunchKernelGGL(sched_count_kernel, dim3((unsigned)((nmajor + 1 + 255) / 256)), dim3(256), 0, s, ptr, nmajor,
                       long_len, chunk, nch, iss);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = exclusive_scan_i32(nch, choff, nmajor + 1, scan_ws, s)) != hipSuccess) return e;
    if ((e = exclusive_scan_i32(iss, spoff, nmajor + 1, scan_ws, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(sched_fill_kernel, dim3((unsigned)((nmajor + 255) / 256)), dim3(256), 0, s, ptr, nmajor, chunk,
                       nch, choff, spoff, chunks, splits);
    return hipGetLastError();
}

hipError_t f32_to_bf16(const float *x, uint16_t *y, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t done = 0;
    if ((uintptr_t)x % 16 == 0 && (uintptr_t)y % 16 == 0) {
        const int64_t groups = n / 8;
        if (groups > 0) {
            const int64_t nb = (groups + 255) / 256;
            if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
            hipLaunchKernelGGL(f32_to_bf16_x8_kernel, dim3((unsigned)nb), dim3(256), 0, s,
                               reinterpret_cast<const float4 *>(x), reinterpret_cast<uint4 *>(y), groups);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        done = groups * 8;
    }
    if (done == n) return hipSuccess;
    const int64_t nb = (n - done + 255) / 256;
    if (nb > 0x7fffffffLL) return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3((unsigned)nb), dim3(256), 0, s, x, y, done, n);
    return hipGetLastError();
}

}  // namespace fmm
