// The entry point that allocates nothing: signtri_noalloc().
//
// For callers that cannot allocate memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation): sign(T) with the scratch
// memory the dataflow sweeps and the projector form need (signs, diagonal,
// completion flags, task lists, the projector's bases and flags) taken from a
// fixed array in device memory, and the host staging of the planner from a
// fixed host array, instead of a library-owned workspace that grows on demand.
//
// `scratch` is a file-scope device array: every GPU the library runs on holds
// its own copy until the process ends.  Its name is a host-side stand-in in host
// code, not a device address; the address of this device's copy comes from
// hipGetSymbolAddress, once per device (with that device current), and only
// that pointer is handed to kernels and copies.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "common.h"

namespace {

constexpr int64_t kNoAllocMaxN = 8192;             // largest order, real or complex
constexpr size_t kScratchBytes = 56ull << 20;      // device scratch: 56 MiB per GPU
constexpr size_t kHostBytes = 2ull << 20;          // host staging of the planner
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

alignas(256) char host_stage[kHostBytes];
std::mutex mu;                                     // one call at a time in this process
void *scratch_ptr[kMaxDevices];                    // per device: its copy of `scratch`

}  // namespace

extern "C" int signtri_noalloc(const void *T, int64_t ldt, void *U, int64_t ldu, int64_t n,
                               signtri_dtype dtype, void *stream, signtri_info *info)
{
    if (info) std::memset(info, 0, sizeof(*info));
    if (n > 0 && !T) return -1;
    if (ldt < std::max<int64_t>(1, n)) return -2;
    if (n > 0 && !U) return -3;
    if (ldu < std::max<int64_t>(1, n)) return -4;
    if (n < 0) return -5;
    if (dtype != SIGNTRI_R64 && dtype != SIGNTRI_C128) return -6;
    if (n == 0) return SIGNTRI_OK;
    // sizes beyond the fixed buffers are rejected before any device work
    if (n > kNoAllocMaxN || sgt::noalloc_device_bytes(n, dtype) > kScratchBytes ||
        sgt::noalloc_host_bytes(n, dtype) > kHostBytes)
        return SIGNTRI_ETOOBIG;

    std::lock_guard<std::mutex> g(mu);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SIGNTRI_EHIP;
    if (!scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SIGNTRI_EHIP;
        scratch_ptr[dev] = p;
    }
    const sgt::NoAllocBuffers na{scratch_ptr[dev], kScratchBytes, host_stage, kHostBytes};
    // with an info the call waits for its result (and reports a dependency wait
    // that gave up), so the scratch is free again when it returns
    signtri_info local;
    signtri_info *inf = info ? info : &local;
    const int rc = sgt::signtri_run(T, ldt, U, ldu, n, dtype, SIGNTRI_COL_MAJOR, SIGNTRI_FP64,
                                    SIGNTRI_AUTO, nullptr, 0, stream, nullptr, inf, &na);
    if (rc != SIGNTRI_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        return rc;
    }
    return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? SIGNTRI_OK : SIGNTRI_EHIP;
}
