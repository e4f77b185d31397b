// FusedMMA forward for callers that cannot allocate device memory (code under stream
// capture, serving loops, harnesses that forbid hipMalloc).  It runs the kernels of
// fmm_fusedmm_a (fused form); the partial sums of split lines, which that call keeps in
// a caller workspace, go to a library-owned device array instead.
//
// The array is a file-scope __device__ variable, so every GPU the library runs on holds
// its own copy until the process ends.  Host code never passes the variable's name to a
// kernel (on the host that name is a stand-in, not a device address): the device address
// is looked up once per device with hipGetSymbolAddress and kept.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "fmm.h"
#include "fmm_internal.hpp"

namespace {

__device__ __align__(256) unsigned char scratch[FMM_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the array (looked up on first use, with the
// device current, and cached per device).
hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" fmm_status fmm_fusedmm_a_noalloc(const fmm_sparse *S_csr, const void *A, const void *B, int32_t r,
                                            int32_t dtype, void *C, hipStream_t stream)
{
    if (!S_csr) return FMM_ERR_NULL;
    size_t need = 0;
    fmm_status st = fmm_workspace_size(FMM_OP_FUSEDMM_A, S_csr, nullptr, r, dtype, &need);
    if (st != FMM_OK) return st;
    if (need > (size_t)FMM_NOALLOC_SCRATCH_BYTES) return FMM_ERR_WORKSPACE;
    void *ws = nullptr;
    if (need > 0) {
        hipError_t e = scratch_address(&ws);
        if (e != hipSuccess) {
            fmm::set_last_hip_error((int32_t)e);
            return FMM_ERR_HIP;
        }
    }
    // every chunk writes its whole partial before the merge reads it, so the array
    // needs no clearing between calls
    return fmm_fusedmm_a(S_csr, A, B, r, dtype, C, FMM_FUSED, nullptr, ws, need, stream);
}
