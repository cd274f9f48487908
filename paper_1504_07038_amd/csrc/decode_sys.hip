// Systematic-code decode launches: the lost data lines of every block rebuilt
// from residual parity bins (the sweep of decode_body.h in its SYS form).
#include "decode_body.h"

namespace mj {

template <int Q, int NBT>
__global__ __launch_bounds__(kWave) void decode_sys_kernel(DecodeArgs a) {
    const int64_t nbatches = (a.nblocks + a.nb - 1) / a.nb;
    for (int64_t batch = blockIdx.x; batch < nbatches; batch += gridDim.x)
        decode_batch<Q, kDecodeTile, true, kWhole, NBT, DecodeArgs, kStreamPolicy, true>(a, batch);
}

template <int Q>
static hipError_t launch_sys_q(const DecodeArgs &a, int grid, hipStream_t s) {
    constexpr int full = full_slots<Q>();
    const size_t lds = decode_lds_bytes(Q, a.nb, a.ring_stride);
    if (full >= 2 && a.nb <= full / 2)
        hipLaunchKernelGGL((decode_sys_kernel<Q, (full >= 2 ? full / 2 : 1)>), dim3(grid),
                           dim3(kWave), lds, s, a);
    else
        hipLaunchKernelGGL((decode_sys_kernel<Q, full>), dim3(grid), dim3(kWave), lds, s, a);
    return hipGetLastError();
}

// Q: parity projections per block (the most lines that can be lost), 1..8.
hipError_t launch_decode_sys(int Q, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
        case 1: return launch_sys_q<1>(a, grid, s);
        case 2: return launch_sys_q<2>(a, grid, s);
        case 3: return launch_sys_q<3>(a, grid, s);
        case 4: return launch_sys_q<4>(a, grid, s);
        case 5: return launch_sys_q<5>(a, grid, s);
        case 6: return launch_sys_q<6>(a, grid, s);
        case 7: return launch_sys_q<7>(a, grid, s);
        case 8: return launch_sys_q<8>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mj
