// Systematic-code decode launches for 8 to 15 data lines (a unit of its own
// so that the kernels compile in parallel with those for fewer lines).
#include "decode_body.h"

namespace mj {

template <int Q, int NBT>
__global__ __launch_bounds__(kWave) void decode_sys_hi_kernel(DecodeArgs a) {
    const int64_t nbatches = (a.nblocks + a.nb - 1) / a.nb;
    for (int64_t batch = blockIdx.x; batch < nbatches; batch += gridDim.x)
        decode_batch<Q, kDecodeTile, true, kWhole, NBT, DecodeArgs, kStreamPolicy, true>(a, batch);
}

// The body compiled for half the slots (the full one spills: the known
// lines' loads add to the row windows' registers).
template <int Q>
static hipError_t launch_sys_hi_q(const DecodeArgs &a, int grid, hipStream_t s) {
    constexpr int half = half_slots<Q>();
    if (a.nb > half) return hipErrorInvalidValue;
    const size_t lds = decode_lds_bytes(Q, a.nb, a.ring_stride);
    hipLaunchKernelGGL((decode_sys_hi_kernel<Q, half>), dim3(grid), dim3(kWave), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_decode_sys_hi(int Q, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
        case 8: return launch_sys_hi_q<8>(a, grid, s);
        case 9: return launch_sys_hi_q<9>(a, grid, s);
        case 10: return launch_sys_hi_q<10>(a, grid, s);
        case 11: return launch_sys_hi_q<11>(a, grid, s);
        case 12: return launch_sys_hi_q<12>(a, grid, s);
        case 13: return launch_sys_hi_q<13>(a, grid, s);
        case 14: return launch_sys_hi_q<14>(a, grid, s);
        case 15: return launch_sys_hi_q<15>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mj
