// Merged chunked decode launches over several geometry classes.
#include "decode_body.h"

namespace mj {

// Merged chunked sweeps over the classes of a table (half-slot bodies).
template <unsigned QMASK, bool GATHER, int CHUNK>
__global__ __launch_bounds__(kWave) void decode_chunk_classes_kernel(DecodeChunkTable tab) {
    const int64_t total = tab.first_item[tab.nclasses];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int c = 0;
        while (item >= tab.first_item[c + 1]) ++c;
        const DecodeChunkClass &a = tab.cls[c];
        const int64_t batch = item - tab.first_item[c];
        switch (a.Q) {
#define MJ_CHUNK_CASE(QQ)                                                                  \
    case QQ:                                                                               \
        if constexpr ((QMASK >> QQ) & 1u)                                                  \
            decode_batch<QQ, kDecodeTile, !GATHER, CHUNK, half_slots<QQ>()>(a, batch);     \
        break;
            MJ_CHUNK_CASE(2) MJ_CHUNK_CASE(4) MJ_CHUNK_CASE(6) MJ_CHUNK_CASE(8) MJ_CHUNK_CASE(12)
#undef MJ_CHUNK_CASE
            default: break;
        }
    }
}

constexpr unsigned kQ4 = 1u << 4, kQ8 = 1u << 8;

// Row-count sets of the merged chunked launches: 2, 4, 6, 8, 12 alone and the
// {4, 8} mix, and (projection pools) the {4, 6, 8, 12} mix.
bool decode_chunk_classes_supported(unsigned qmask, bool gather) {
    switch (qmask) {
        case 1u << 2: case 1u << 4: case 1u << 6: case 1u << 8: case 1u << 12:
        case kQ4 | kQ8:
            return true;
        case kQ4 | (1u << 6) | kQ8 | (1u << 12):
            return !gather;
        default:
            return false;
    }
}

// One step of the parallel carry over the classes of a table.
__global__ __launch_bounds__(kWave * kCarryWaves) void decode_scan_classes_kernel(
    DecodeChunkTable tab, int step) {
    const int64_t total = tab.first_pair[tab.nclasses];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int c = 0;
        while (item >= tab.first_pair[c + 1]) ++c;
        const DecodeChunkClass &a = tab.cls[c];
        if (!a.chunk.ws_alt) continue;   // one chunk boundary: nothing to carry
        const int per = a.chunk.nchunks - 1;
        const int64_t local = item - tab.first_pair[c];
        const int64_t blk = local / per;
        const uint64_t *src = (step & 1) ? a.chunk.ws_alt : a.chunk.ws;
        uint64_t *dst = (step & 1) ? a.chunk.ws : a.chunk.ws_alt;
        scan_item(a, a.Q, blk, (int)(local - blk * per), step, src, dst);
    }
}

template <unsigned M, bool G>
static hipError_t launch_chunk_sweep(int mode, const DecodeChunkTable &tab, size_t lds, int grid,
                                     hipStream_t s) {
    if (mode == kLaunchChunkA)
        hipLaunchKernelGGL((decode_chunk_classes_kernel<M, G, kChunkA>), dim3(grid), dim3(kWave),
                           lds, s, tab);
    else
        hipLaunchKernelGGL((decode_chunk_classes_kernel<M, G, kChunkC>), dim3(grid), dim3(kWave),
                           lds, s, tab);
    return hipGetLastError();
}

hipError_t launch_decode_chunk_classes(int mode, unsigned qmask, bool gather,
                                       const DecodeChunkTable &tab, size_t lds, int grid,
                                       int threads, bool rows_in_registers, hipStream_t s) {
    if (mode >= kLaunchScan) {
        hipLaunchKernelGGL(decode_scan_classes_kernel, dim3(grid), dim3(threads), lds, s, tab,
                           mode - kLaunchScan);
        return hipGetLastError();
    }
    if (mode == kLaunchCarry) {
        if (rows_in_registers)
            hipLaunchKernelGGL(decode_carry_classes_kernel<8>, dim3(grid), dim3(threads), lds, s,
                               tab);
        else
            hipLaunchKernelGGL(decode_carry_classes_kernel<0>, dim3(grid), dim3(threads), lds, s,
                               tab);
        return hipGetLastError();
    }
    if (mode != kLaunchChunkA && mode != kLaunchChunkC) return hipErrorInvalidValue;
#define MJ_SWEEP(M)                                                               \
    return gather ? launch_chunk_sweep<M, true>(mode, tab, lds, grid, s)          \
                  : launch_chunk_sweep<M, false>(mode, tab, lds, grid, s)
    switch (qmask) {
        case 1u << 2: MJ_SWEEP(1u << 2);
        case 1u << 4: MJ_SWEEP(1u << 4);
        case 1u << 6: MJ_SWEEP(1u << 6);
        case 1u << 8: MJ_SWEEP(1u << 8);
        case 1u << 12: MJ_SWEEP(1u << 12);
        case kQ4 | kQ8: MJ_SWEEP(kQ4 | kQ8);
        case kQ4 | (1u << 6) | kQ8 | (1u << 12):
            if (gather) return hipErrorInvalidValue;
            return launch_chunk_sweep<kQ4 | (1u << 6) | kQ8 | (1u << 12), false>(mode, tab, lds,
                                                                                 grid, s);
        default: return hipErrorInvalidValue;
    }
#undef MJ_SWEEP
}

}  // namespace mj
