// noalloc.hip -- pspfft_solve_noalloc: a solve that allocates nothing, for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops that forbid allocation).  Its workspace is a file-scope device
// array of kNoallocBytes, which every GPU the library runs on holds from the
// time the library's code is loaded there until the process ends.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "../../include/pspfft.h"

namespace pspfft {
pspfft_status solve_on(pspfft_plan_t plan, void *mem, size_t bytes, const void *S, void *Phi, hipStream_t stream);
pspfft_status report_failure(pspfft_status st, pspfft_plan_t plan, const char *what);
}

namespace {

constexpr size_t kNoallocBytes = PSPFFT_NOALLOC_MAX_BYTES;
constexpr int kMaxDevices = 64;

// The workspace of pspfft_solve_noalloc.  Host code never uses this name as an
// address (on the host it is only a stand-in for the symbol): the device
// address comes from hipGetSymbolAddress, per device.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch`, looked up once per device
// with that device current (it is, since the caller's current device is the
// one being asked for).
void *scratch_on(int dev) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace

extern "C" pspfft_status pspfft_solve_noalloc(pspfft_plan_t plan, const void *S, void *Phi, hipStream_t stream) {
    if (!plan || !S || !Phi)
        return pspfft::report_failure(PSPFFT_ERR_INVALID_ARGUMENT, plan, "pspfft_solve_noalloc: null argument");
    int dims[3];
    pspfft_precision prec;
    if (pspfft_plan_info(plan, dims, nullptr, &prec) != PSPFFT_OK)
        return pspfft::report_failure(PSPFFT_ERR_INVALID_ARGUMENT, plan, "pspfft_solve_noalloc: bad plan");
    const size_t need = pspfft_workspace_bytes(dims[0], dims[1], dims[2], prec);
    if (need == 0 || need > kNoallocBytes)
        return pspfft::report_failure(PSPFFT_ERR_UNSUPPORTED_SIZE, plan,
                                      "pspfft_solve_noalloc: the mesh's workspace exceeds the library's "
                                      "PSPFFT_NOALLOC_MAX_BYTES (128 MiB) array");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return pspfft::report_failure(PSPFFT_ERR_DEVICE, plan, "pspfft_solve_noalloc: hipGetDevice");
    void *mem = scratch_on(dev);
    if (!mem)
        return pspfft::report_failure(PSPFFT_ERR_DEVICE, plan, "pspfft_solve_noalloc: hipGetSymbolAddress");
    return pspfft::solve_on(plan, mem, kNoallocBytes, S, Phi, stream);
}
