// Inverse Mojette transform on gfx950 (Section 2.2), XOR addition.
//
// Reconstruction path.  Of the surviving projections, the Q with the smallest
// p are used; sorted by p, the r-th (p_r) is dedicated to image row r, as the
// fixed path of Section 2.2 dedicates one projection to one line.  Bin
// b = r*p_r - k of that projection crosses pixel (k, r) and, in every other
// row l, pixel (k + (l-r)*p_r, l).  So
//
//     f(k, r) = bin_r[r*p_r - k] XOR  XOR_{l != r} f(k + (l-r)*p_r, l),
//
// with pixels outside the image counting as zero.  With
// A_r = 2*(p_0 + ... + p_{r-1}) + r, pixel (k, r) is reconstructed at
// half-step h = 2k - A_r (+ a constant): every pixel it needs has a strictly
// smaller h, because for l > r, A_l - A_r - 2(l-r)p_r = 2*sum_{r<=j<l}(p_j - p_r)
// + (l - r) > 0, and for l < r the distinct sorted p give p_r - p_j >= r - j,
// so the gap is at least (r - l)^2 > 0.  Rows therefore sweep their columns
// left to right in lockstep (the left-to-right reconstruction of Section
// 3.1), row r active on half-steps of parity A_r.
//
// Mapping.  One lane per (block, row); a wavefront holds up to 64/Q blocks and one
// workgroup is one wavefront, so no barrier is ever needed.  A row keeps only
// its last R pixels, in an LDS ring (slot = column mod R): a pixel is read at
// most D columns behind its row's newest pixel, D fixed by the survivor set,
// and R > D is chosen by the host over every survivor set.  Columns outside
// the image are written as zero, and rings start zeroed, so dependency reads
// are never bounds checked.  Each lane streams its own row's P used bins
// from HBM one tile of TW columns ahead; after each tile the wave stores the
// tile's pixels of all its rows, eight lanes per 128-byte row segment.
#include <climits>

#include "mj_internal.h"

namespace mj {

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}

// Loads the bins of columns k0 .. k0+TW-1 of one row.  Every load is issued
// unconditionally from an in-range address (columns clamped to [0, P)), so the
// results stay in flight until the next tile uses them; values loaded for
// columns outside the image, or by lanes without a block, are never used.
template <int TW>
__device__ __forceinline__ void load_bins(uint64_t (&dst)[TW], const uint64_t *bins, int jbase,
                                          int k0, int P) {
#pragma unroll
    for (int i = 0; i < TW; ++i) {
        int k = k0 + i;
        k = k < 0 ? 0 : (k >= P ? P - 1 : k);
        dst[i] = bins[jbase - k];
    }
}

template <int Q>
__global__ __launch_bounds__(kWave) void decode_kernel(DecodeArgs a) {
    constexpr int NBMAX = kWave / Q;  // blocks per wavefront at most
    constexpr int TW = kDecodeTile;
    constexpr int LPS = TW / 2;     // lanes per stored row segment (two words each)
    constexpr int SPI = kWave / LPS;

    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x;
    const int slot = lane / Q;
    const int r = lane - slot * Q;
    const int NB = a.nb;
    const int NSEG = NB * Q;          // ring rows in use
    const bool lane_used = slot < NB;
    const int RS = a.ring_stride;
    const int Rmask = a.R - 1;
    uint64_t *zero_row = lds + (size_t)NSEG * RS;
    for (int c = lane; c < a.R; c += kWave) zero_row[c] = 0;

    const int64_t nbatches = (a.nblocks + NB - 1) / NB;
    for (int64_t batch = blockIdx.x; batch < nbatches; batch += gridDim.x) {
        const int64_t blk = batch * NB + slot;
        bool valid = lane_used && blk < a.nblocks;
        uint32_t mask = a.mask_uniform;
        if (valid && a.masks) mask = a.masks[blk];

        // Survivors in ascending p; row r takes the r-th.
        int my_p = 0, my_id = 0, A_r = 0, A_max = INT_MIN, A_min = INT_MAX, cnt = 0, psum = 0;
        for (int s = 0; s < a.n; ++s) {
            const int id = a.id_sorted[s];
            const int p = a.p_sorted[s];
            if (!((mask >> id) & 1u) && cnt < Q) {
                const int A = 2 * psum + cnt;
                if (cnt == r) {
                    my_p = p;
                    my_id = id;
                    A_r = A;
                }
                A_max = max(A_max, A);
                A_min = min(A_min, A);
                psum += p;
                ++cnt;
            }
        }
        if (cnt < Q) {
            if (valid && r == 0 && a.status) a.status[0] = MOJETTE_ENOTRECON;
            valid = false;
        }
        // Tile t of row r covers columns [t*TW + d, t*TW + d + TW); column
        // t*TW + d + i is handled at sub-step 2i + e.
        const int d = valid ? -((A_max - A_r) >> 1) : 0;
        const int e = valid ? 2 * d - (A_r - A_max) : 0;
        const int dmin = valid ? -((A_max - A_min) >> 1) : 0;
        const int ntiles = valid ? (a.P - dmin + TW - 1) / TW : 0;
        const int ntiles_wave = wave_max(ntiles);

        uint64_t *ring = lds + (size_t)(lane_used ? lane : 0) * RS;
        uint64_t *dep[Q];
        int delta[Q];
#pragma unroll
        for (int l = 0; l < Q; ++l) {
            dep[l] = (l == r || !lane_used) ? zero_row : lds + (size_t)(slot * Q + l) * RS;
            delta[l] = (l - r) * my_p;
        }
        if (lane_used)
            for (int c = 0; c < a.R; ++c) ring[c] = 0;

        // Lanes without a block read column bins of a projection that always
        // exists (p = 0 gives jbase = P - 1, so indices stay in [0, P)).
        const uint64_t *bins = valid ? a.in[my_id] + blk * a.proj_stride : a.fallback;
        const int jbase = valid ? r * my_p - bin_offset(my_p, a.P, Q) : a.P - 1;
        uint64_t cb[TW], nb[TW];
        load_bins<TW>(cb, bins, jbase, d, a.P);
        wave_sync();

        for (int t = 0; t < ntiles_wave; ++t) {
            const int k0 = t * TW + d;
            load_bins<TW>(nb, bins, jbase, k0 + TW, a.P);
            int o[Q];
#pragma unroll
            for (int l = 0; l < Q; ++l) o[l] = k0 + delta[l];
#pragma unroll
            for (int u = 0; u < 2 * TW; ++u) {
                const int i = u >> 1;
                if (valid && e == (u & 1)) {
                    uint64_t v = cb[i];
#pragma unroll
                    for (int l = 0; l < Q; ++l) v ^= dep[l][(o[l] + i) & Rmask];
                    const int k = k0 + i;
                    if ((unsigned)k >= (unsigned)a.P) v = 0;
                    ring[k & Rmask] = v;
                }
                wave_sync();
            }
            // Store this tile's columns of every row of the wave.
#pragma unroll
            for (int it = 0; it < (NBMAX * Q + SPI - 1) / SPI; ++it) {
                const int seg = it * SPI + lane / LPS;
                const int pair = lane % LPS;
                const int od = __shfl(valid ? d : INT_MIN, seg < kWave ? seg : 0);
                if (seg < NSEG && od != INT_MIN) {
                    const int sslot = seg / Q;
                    const int srow = seg - sslot * Q;
                    const int k = t * TW + od + 2 * pair;
                    const uint64_t *sring = lds + (size_t)seg * RS;
                    uint64_t *dst = a.images + (batch * NB + sslot) * a.img_stride +
                                    (int64_t)srow * a.P;
                    if ((unsigned)k < (unsigned)a.P) dst[k] = sring[k & Rmask];
                    if ((unsigned)(k + 1) < (unsigned)a.P) dst[k + 1] = sring[(k + 1) & Rmask];
                }
            }
            wave_sync();
#pragma unroll
            for (int i = 0; i < TW; ++i) cb[i] = nb[i];
        }
        wave_sync();
    }
}

size_t decode_lds_bytes(int Q, int nb, int ring_stride) {
    return (size_t)(nb * Q + 1) * ring_stride * sizeof(uint64_t);
}

template <int Q>
static hipError_t launch_q(const DecodeArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(decode_kernel<Q>, dim3(grid), dim3(kWave), decode_lds_bytes(Q, a.nb, a.ring_stride),
                       s, a);
    return hipGetLastError();
}

hipError_t launch_decode(int Q, const DecodeArgs &a, int grid, hipStream_t s) {
    switch (Q) {
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
