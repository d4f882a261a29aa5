// Static device scratch of the allocation-free batched decode
// (ldpc_decode_batch_f32_noalloc), for callers that cannot allocate device
// memory during a call: code under HIP graph capture, tight serving loops.
//
// The array below lives in this library's code object, so every GPU that
// runs the library holds its own copy, at its own address, until the process
// ends. In host code the array's name is only a stand-in for that memory:
// its device address is looked up once per device with hipGetSymbolAddress
// (with that device current) and only the address is handed to kernels.
// All calls on one GPU share the array: calls that overlap on one GPU race.
#include <mutex>

#include "ldpc_internal.h"

namespace ldpc {

namespace {

// Work list of a batched decode: queue words, frame permutation, per-frame
// offsets and work items (see batch_work_bytes), for up to
// kBatchScratchFrames frames of a code set of up to 1024 codes.
static __device__ __align__(256) unsigned char scratch[kBatchScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

}  // namespace

int batch_scratch(int dev, void **out)
{
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LDPC_ERANGE, "device %d is beyond the %d devices the static scratch serves", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        int cur = 0;
        if (hipGetDevice(&cur) != hipSuccess || cur != dev)
            return fail(LDPC_EDEVICE, "device %d must be current to look up its scratch", dev);
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return fail(LDPC_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                        hipGetErrorString(hipGetLastError()));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return LDPC_OK;
}

}  // namespace ldpc
