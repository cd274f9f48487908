// Mixed decode launches: several geometry classes in one launch.
#include "decode_body.h"

namespace mj {

// A mixed launch: batches of every class, in the order of the class table
// (heaviest first), one wavefront per workgroup.  QMASK has bit Q set for
// every row count the launch may meet; only those bodies are compiled in, so
// the kernel's registers are those of its largest body, not of all sixteen.
// The bodies are compiled for half the block slots, which leaves registers
// for more wavefronts per SIMD (measured: a mixed step of 16 classes ran
// 1.18x faster than with full-slot bodies).
template <unsigned QMASK, bool GATHER>
__global__ __launch_bounds__(kWave) void decode_classes_kernel(DecodeClassTable tab) {
    const int64_t total = tab.first_item[tab.nclasses];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int c = 0;
        while (item >= tab.first_item[c + 1]) ++c;
        const DecodeClass &a = tab.cls[c];
        const int64_t batch = item - tab.first_item[c];
        switch (a.Q) {
#define MJ_DEC_CASE(QQ)                                                                  \
    case QQ:                                                                             \
        if constexpr ((QMASK >> QQ) & 1u)                                               \
            decode_batch<QQ, kDecodeTile, !GATHER, kWhole, half_slots<QQ>(),              \
                         DecodeClass, 0>(a, batch);                                          \
        break;
            MJ_DEC_CASE(1) MJ_DEC_CASE(2) MJ_DEC_CASE(3) MJ_DEC_CASE(4)
            MJ_DEC_CASE(5) MJ_DEC_CASE(6) MJ_DEC_CASE(7) MJ_DEC_CASE(8)
            MJ_DEC_CASE(9) MJ_DEC_CASE(10) MJ_DEC_CASE(11) MJ_DEC_CASE(12)
            MJ_DEC_CASE(13) MJ_DEC_CASE(14) MJ_DEC_CASE(15) MJ_DEC_CASE(16)
#undef MJ_DEC_CASE
            default: break;
        }
    }
}

constexpr unsigned qbit(int q) { return 1u << q; }

// Row-count sets with a compiled mixed kernel: every single row count, and
// the mixes of the (4,2)+(8,4) and (4,2)+(6,3)+(8,4)+(12,4) code families.
// Gathering launches (blocks at arbitrary projection slots) exist for the
// even row counts up to 16 and the (4,2)+(8,4) mix.
bool decode_classes_supported(unsigned qmask, bool gather) {
    if (gather) {
        switch (qmask) {
            case qbit(2): case qbit(4): case qbit(6): case qbit(8): case qbit(10):
            case qbit(12): case qbit(14): case qbit(16): case qbit(4) | qbit(8): return true;
            default: return false;
        }
    }
    if (qmask && !(qmask & (qmask - 1))) return true;
    return qmask == (qbit(4) | qbit(8)) || qmask == (qbit(4) | qbit(6) | qbit(8) | qbit(12));
}

hipError_t launch_decode_classes(unsigned qmask, bool gather, const DecodeClassTable &tab,
                                 size_t lds, int grid, hipStream_t s) {
#define MJ_LAUNCH(M, G) \
    hipLaunchKernelGGL((decode_classes_kernel<M, G>), dim3(grid), dim3(kWave), lds, s, tab)
    if (gather) {
        switch (qmask) {
            case qbit(2): MJ_LAUNCH(qbit(2), true); break;
            case qbit(4): MJ_LAUNCH(qbit(4), true); break;
            case qbit(6): MJ_LAUNCH(qbit(6), true); break;
            case qbit(8): MJ_LAUNCH(qbit(8), true); break;
            case qbit(10): MJ_LAUNCH(qbit(10), true); break;
            case qbit(12): MJ_LAUNCH(qbit(12), true); break;
            case qbit(14): MJ_LAUNCH(qbit(14), true); break;
            case qbit(16): MJ_LAUNCH(qbit(16), true); break;
            case qbit(4) | qbit(8): MJ_LAUNCH(qbit(4) | qbit(8), true); break;
            default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    switch (qmask) {
        case qbit(1): MJ_LAUNCH(qbit(1), false); break;
        case qbit(2): MJ_LAUNCH(qbit(2), false); break;
        case qbit(3): MJ_LAUNCH(qbit(3), false); break;
        case qbit(4): MJ_LAUNCH(qbit(4), false); break;
        case qbit(5): MJ_LAUNCH(qbit(5), false); break;
        case qbit(6): MJ_LAUNCH(qbit(6), false); break;
        case qbit(7): MJ_LAUNCH(qbit(7), false); break;
        case qbit(8): MJ_LAUNCH(qbit(8), false); break;
        case qbit(9): MJ_LAUNCH(qbit(9), false); break;
        case qbit(10): MJ_LAUNCH(qbit(10), false); break;
        case qbit(11): MJ_LAUNCH(qbit(11), false); break;
        case qbit(12): MJ_LAUNCH(qbit(12), false); break;
        case qbit(13): MJ_LAUNCH(qbit(13), false); break;
        case qbit(14): MJ_LAUNCH(qbit(14), false); break;
        case qbit(15): MJ_LAUNCH(qbit(15), false); break;
        case qbit(16): MJ_LAUNCH(qbit(16), false); break;
        case qbit(4) | qbit(8): MJ_LAUNCH(qbit(4) | qbit(8), false); break;
        case qbit(4) | qbit(6) | qbit(8) | qbit(12):
            MJ_LAUNCH(qbit(4) | qbit(6) | qbit(8) | qbit(12), false);
            break;
        default: return hipErrorInvalidValue;
    }
#undef MJ_LAUNCH
    return hipGetLastError();
}

}  // namespace mj
