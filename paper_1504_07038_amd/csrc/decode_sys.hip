// Systematic-code decode launches: the lost data lines of every block rebuilt
// from the parity bins and the surviving lines (the sweep of decode_body.h in
// its SYS form).
#include "decode_body.h"

namespace mj {

template <int Q, int NBT>
__global__ __launch_bounds__(kWave) void decode_sys_kernel(DecodeArgs a) {
    const int64_t nbatches = (a.nblocks + a.nb - 1) / a.nb;
    for (int64_t batch = blockIdx.x; batch < nbatches; batch += gridDim.x)
        decode_batch<Q, kDecodeTile, true, kWhole, NBT, DecodeArgs, kStreamPolicy, true>(a, batch);
}

// The body compiled for half the slots (the full one spills: the known
// lines' loads add to the row windows' registers).
template <int Q>
static hipError_t launch_sys_q(const DecodeArgs &a, int grid, hipStream_t s) {
    constexpr int half = half_slots<Q>();
    if (a.nb > half) return hipErrorInvalidValue;
    const size_t lds = decode_lds_bytes(Q, a.nb, a.ring_stride);
    hipLaunchKernelGGL((decode_sys_kernel<Q, half>), dim3(grid), dim3(kWave), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_decode_sys_hi(int Q, const DecodeArgs &a, int grid, hipStream_t s);

// Q: data lines per block, 1..15.
hipError_t launch_decode_sys(int Q, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
        case 1: return launch_sys_q<1>(a, grid, s);
        case 2: return launch_sys_q<2>(a, grid, s);
        case 3: return launch_sys_q<3>(a, grid, s);
        case 4: return launch_sys_q<4>(a, grid, s);
        case 5: return launch_sys_q<5>(a, grid, s);
        case 6: return launch_sys_q<6>(a, grid, s);
        case 7: return launch_sys_q<7>(a, grid, s);
        default: return launch_decode_sys_hi(Q, a, grid, s);
    }
}

}  // namespace mj
