// Single-geometry decode launches: whole blocks (a pool, or one block from
// projection pointers) and the three passes of the chunked decode.
#include "decode_body.h"

namespace mj {

int decode_tile(int) { return kDecodeTile; }

size_t decode_lds_bytes(int Q, int nb, int ring_stride) {
    return (size_t)nb * (Q * ring_stride + 1) * sizeof(uint64_t);
}

int decode_max_blocks_per_wave(int Q) { return kWave / ((Q + 1) / 2); }

int carry_waves(int state) {
    return std::min(kCarryWaves, std::max(1, (state + kWave - 1) / kWave));
}

size_t carry_lds_bytes(int state) {
    return ((size_t)state + 4 + kCarryTableWords) * sizeof(uint64_t);
}

bool carry_rows_in_registers(int state) {
    return state <= kWave * kCarryWaves && state <= 8 * 64;
}

hipError_t launch_decode_carry(const DecodeArgs &a, int Q, int grid, hipStream_t s) {
    const int state = Q * a.chunk.max_cols;
    if (state > kCarryMaxState) return hipErrorInvalidValue;
    const int threads = kWave * carry_waves(state);
    const size_t lds = carry_lds_bytes(state);
    // rows cached in registers while one thread per output word suffices
    if (carry_rows_in_registers(state))
        hipLaunchKernelGGL(decode_carry_kernel<8>, dim3(grid), dim3(threads), lds, s, a, Q);
    else
        hipLaunchKernelGGL(decode_carry_kernel<0>, dim3(grid), dim3(threads), lds, s, a, Q);
    return hipGetLastError();
}

// One step of the parallel carry over the chunks of every block.
__global__ __launch_bounds__(kWave * kCarryWaves) void decode_scan_kernel(DecodeArgs a, int Q,
                                                                          int step,
                                                                          const uint64_t *src,
                                                                          uint64_t *dst) {
    const int per = a.chunk.nchunks - 1;
    const int64_t total = a.nblocks * per;
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        const int64_t blk = item / per;
        scan_item(a, Q, blk, (int)(item - blk * per), step, src, dst);
    }
}

hipError_t launch_decode_scan(const DecodeArgs &a, int Q, int step, const uint64_t *src,
                              uint64_t *dst, hipStream_t s) {
    const int state = Q * a.chunk.max_cols;
    if (state > kScanMaxState) return hipErrorInvalidValue;
    const int threads = kWave * carry_waves(state);
    const size_t lds = ((size_t)state + 4 + (size_t)(state + 3) / 4 * 16) * sizeof(uint64_t);
    const int64_t items = a.nblocks * (a.chunk.nchunks - 1);
    const int grid = (int)std::min<int64_t>(items, 256 * 128);
    hipLaunchKernelGGL(decode_scan_kernel, dim3(grid), dim3(threads), lds, s, a, Q, step, src, dst);
    return hipGetLastError();
}

hipError_t launch_decode_hi(int Q, int mode, const DecodeArgs &a, int grid, hipStream_t s);

hipError_t launch_decode(int Q, int mode, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
        case 1: return launch_q<1>(mode, a, grid, s);
        case 2: return launch_q<2>(mode, a, grid, s);
        case 3: return launch_q<3>(mode, a, grid, s);
        case 4: return launch_q<4>(mode, a, grid, s);
        case 5: return launch_q<5>(mode, a, grid, s);
        case 6: return launch_q<6>(mode, a, grid, s);
        case 7: return launch_q<7>(mode, a, grid, s);
        case 8: return launch_q<8>(mode, a, grid, s);
        default: return launch_decode_hi(Q, mode, a, grid, s);
    }
}

}  // namespace mj
