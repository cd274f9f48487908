// Single-geometry decode launches for 9 to 16 rows (a unit of its own so that
// the kernels compile in parallel with those for fewer rows).
#include "decode_body.h"

namespace mj {

hipError_t launch_decode_hi(int Q, int mode, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
        case 9: return launch_q<9>(mode, a, grid, s);
        case 10: return launch_q<10>(mode, a, grid, s);
        case 11: return launch_q<11>(mode, a, grid, s);
        case 12: return launch_q<12>(mode, a, grid, s);
        case 13: return launch_q<13>(mode, a, grid, s);
        case 14: return launch_q<14>(mode, a, grid, s);
        case 15: return launch_q<15>(mode, a, grid, s);
        case 16: return launch_q<16>(mode, a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mj
