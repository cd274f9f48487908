// Whole-block decode of 128-bit pixels (Section 3.1): the sweep of
// decode_body.h with 16-byte rings, bins and pixels, in the geometry of the
// 16-byte image itself (P pixels per row, directions p).
#include "decode_body.h"

namespace mj {

hipError_t launch_decode_wide(int Q, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
        case 1: return launch_wide_q<1>(a, grid, s);
        case 2: return launch_wide_q<2>(a, grid, s);
        case 3: return launch_wide_q<3>(a, grid, s);
        case 4: return launch_wide_q<4>(a, grid, s);
        case 5: return launch_wide_q<5>(a, grid, s);
        case 6: return launch_wide_q<6>(a, grid, s);
        case 7: return launch_wide_q<7>(a, grid, s);
        case 8: return launch_wide_q<8>(a, grid, s);
        case 9: return launch_wide_q<9>(a, grid, s);
        case 10: return launch_wide_q<10>(a, grid, s);
        case 11: return launch_wide_q<11>(a, grid, s);
        case 12: return launch_wide_q<12>(a, grid, s);
        case 13: return launch_wide_q<13>(a, grid, s);
        case 14: return launch_wide_q<14>(a, grid, s);
        case 15: return launch_wide_q<15>(a, grid, s);
        case 16: return launch_wide_q<16>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mj
