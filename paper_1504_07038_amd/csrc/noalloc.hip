// Chunked decode without allocation, for callers that cannot allocate device
// memory (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): the chunked decode's workspace is a fixed device array of this
// file.  In host code the array's name is a host-side stand-in, not a device
// address: the address is taken once per device, with that device current,
// and kept; only that address reaches the kernels.
#include <map>
#include <mutex>

#include "mj_internal.h"

namespace {

static __device__ __align__(256) uint64_t scratch[MOJETTE_SCRATCH_WORDS];

// The device address of `scratch` on the current device (looked up on the
// first call per device), or null after a HIP error.
uint64_t *scratch_on_current_device() {
    static std::mutex mu;
    static std::map<int, uint64_t *> ptrs;
    int dev = 0;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) {
        mj::hip_status(ge);
        return nullptr;
    }
    std::lock_guard<std::mutex> g(mu);
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        mj::hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol);
        return nullptr;
    }
    return ptrs[dev] = static_cast<uint64_t *>(ptr);
}

}  // namespace

int mojette_decode_batch_chunked_noalloc(const mojette_chunk_plan *plan, const uint64_t *projs,
                                         const uint16_t *erased, int64_t nblocks, int32_t P,
                                         uint64_t *images, int32_t *status, void *stream) {
    const int64_t need = mojette_decode_chunked_workspace(plan, P, nblocks);
    if (need < 0) return MOJETTE_EINVAL;
    if (need > MOJETTE_SCRATCH_WORDS) return MOJETTE_ESCRATCH;
    uint64_t *ws = nullptr;
    if (need > 0) {
        (void)hipGetLastError();   // an earlier call's error is not this lookup's
        ws = scratch_on_current_device();
        if (!ws) return MOJETTE_EHIP;
    }
    // Every scratch word the decode reads was written earlier in the same
    // call (the chunks' end states, then the carries), so nothing is cleared.
    return mojette_decode_batch_chunked(plan, projs, erased, nblocks, P, images, status, ws,
                                        stream);
}
