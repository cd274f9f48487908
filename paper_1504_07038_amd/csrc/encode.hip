// Forward Mojette transform on gfx950 (Section 2.1, Eq. 1, XOR addition).
//
// Bin b of direction (p, 1) is the XOR of pixel (l*p - b, l) over the rows l
// whose column l*p - b lies inside the image.  One wavefront owns one
// (block, column tile) work item: it stages the tile's rows plus a halo into
// LDS with coalesced loads, zero-filled outside the image so that no bin
// needs a bounds check, then each lane produces consecutive bins of one
// projection at a time, so every store instruction writes 64 contiguous
// words of a projection.
#include "mj_internal.h"

namespace mj {

template <int Q>
__global__ __launch_bounds__(kWave *kEncodeWaves) void encode_kernel(EncodeArgs a) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x >> 6;
    uint64_t *tile = lds + (size_t)wv * Q * a.S;
    const int64_t nitems = a.nblocks * a.ntiles;
    const int64_t nwaves = (int64_t)gridDim.x * a.waves;
    for (int64_t item = (int64_t)blockIdx.x * a.waves + wv; item < nitems; item += nwaves) {
        int64_t blk;
        int t;
        if (a.ntiles == 1) {
            blk = item;
            t = 0;
        } else {
            blk = item / a.ntiles;
            t = (int)(item - blk * a.ntiles);
        }
        const int x0 = t * a.W;
        const uint64_t *img = a.images + blk * a.img_stride;

        // Stage image columns [x0 - H, x0 + W + H) of every row, zeros outside.
#pragma unroll
        for (int l = 0; l < Q; ++l) {
            const uint64_t *row = img + (int64_t)l * a.P;
            for (int c = lane; c < a.S; c += kWave) {
                const int col = x0 - a.H + c;
                uint64_t v = 0;
                if ((unsigned)col < (unsigned)a.P) v = row[col];
                tile[l * a.S + c] = v;
            }
        }
        wave_sync();

        // The bins whose row-0 crossing -b falls in [x0, x0 + W); the first
        // tile also takes the edge bins with -b < 0, the last those with
        // -b >= P.
        const bool first = (t == 0), last = (t == a.ntiles - 1);
        const int base = a.H - x0;
        for (int i = 0; i < a.n; ++i) {
            const int p = a.p[i];
            const int bmin = a.bmin[i];
            const int bmax = bmin + a.nbins[i] - 1;
            const int bh = first ? bmax : min(bmax, -x0);
            const int bl = last ? bmin : max(bmin, -x0 - a.W + 1);
            uint64_t *dst = a.out[i] + blk * a.proj_stride;
            const int rstride = a.S + p;
            for (int b = bl + lane; b <= bh; b += kWave) {
                uint64_t v = 0;
#pragma unroll
                for (int l = 0; l < Q; ++l) v ^= tile[l * rstride + base - b];
                dst[b - bmin] = v;
            }
        }
        wave_sync();  // the next item restages this wave's tile
    }
}

size_t encode_lds_bytes(int Q, int S, int waves) { return (size_t)waves * Q * S * sizeof(uint64_t); }

template <int Q>
static hipError_t launch_q(const EncodeArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(encode_kernel<Q>, dim3(grid), dim3(kWave * a.waves),
                       encode_lds_bytes(Q, a.S, a.waves), s, a);
    return hipGetLastError();
}

hipError_t launch_encode(const EncodeArgs &a, int grid, hipStream_t s) {
    switch (a.Q) {
        case 1: return launch_q<1>(a, grid, s);
        case 2: return launch_q<2>(a, grid, s);
        case 3: return launch_q<3>(a, grid, s);
        case 4: return launch_q<4>(a, grid, s);
        case 5: return launch_q<5>(a, grid, s);
        case 6: return launch_q<6>(a, grid, s);
        case 7: return launch_q<7>(a, grid, s);
        case 8: return launch_q<8>(a, grid, s);
        case 9: return launch_q<9>(a, grid, s);
        case 10: return launch_q<10>(a, grid, s);
        case 11: return launch_q<11>(a, grid, s);
        case 12: return launch_q<12>(a, grid, s);
        case 13: return launch_q<13>(a, grid, s);
        case 14: return launch_q<14>(a, grid, s);
        case 15: return launch_q<15>(a, grid, s);
        case 16: return launch_q<16>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace mj
