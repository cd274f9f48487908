// Forward Mojette transform on gfx950 (Section 2.1, Eq. 1, XOR addition).
//
// Bin b of direction (p, 1) is the XOR of pixel (l*p - b, l) over the rows l
// whose column l*p - b lies inside the image.  One wavefront owns one
// (block, column tile) work item: it stages the tile's rows plus a halo into
// LDS with coalesced loads, zero-filled outside the image so that no bin
// needs a bounds check, then each lane produces consecutive bins of one
// projection at a time, so every store instruction writes 64 contiguous
// words of a projection.  (Non-temporal loads or stores made it slower on the
// MI355X: 1.73 and 1.77 against 1.93 TB/s of user data for 4 KB blocks.)
//
// 128-bit pixels (Section 3.1) use the same kernel.  XOR acts on every bit
// alone, so a P x Q image of 16-byte pixels is a 2P x Q image of 8-byte
// words, half h of pixel k at word column 2k + h, and its projection along
// (p, 1) is that word image's projection along (2p, 1): half h of pixel k
// lands on word bin 2b - h.  Word bins 2j+1 and 2j thus hold the two halves
// of bin j in reverse order; with bin_swap = 1 word bin j is stored at word
// j ^ 1, which keeps every 16-byte bin in a pixel's half order.
#include "mj_internal.h"

namespace mj {

// One work item: the bins of block `blk` whose row-0 crossing falls in
// column tile t, computed by one wavefront from its LDS tile.  `A` supplies
// the geometry (EncodeArgs for one pool, EncodeClass for one class of a mixed
// launch).
template <int Q, class A, bool VERIFY = false>
__device__ __forceinline__ void encode_bins(const A &a, int64_t blk, int t, const uint64_t *tile,
                                            int lane, uint32_t use, int64_t slice_in = -1);

// VERIFY (A = VerifyArgs): the bins of every surviving projection are
// compared with the stored ones instead of being written.
template <int Q, class A, bool VERIFY = false>
__device__ __forceinline__ void encode_item(const A &a, int64_t blk, int t, uint64_t *tile,
                                            int lane) {
    const int P = a.P, W = a.W, H = a.H, S = a.S;
    const int x0 = t * W;
    const uint64_t *img = a.image_of(blk);

    uint32_t use = 0;                       // VERIFY: the projections checked
    if constexpr (VERIFY) {
        const uint32_t mask = a.masks ? a.masks[blk] : a.mask_uniform;
        use = ~mask & ((1u << a.n) - 1u);
    }

    // Stage image columns [x0 - H, x0 + W + H) of every row, zeros outside.
#pragma unroll
    for (int l = 0; l < Q; ++l) {
        const uint64_t *row = img + (int64_t)l * P;
        for (int c = lane; c < S; c += kWave) {
            const int col = x0 - H + c;
            uint64_t v = 0;
            if ((unsigned)col < (unsigned)P) v = row[col];
            tile[l * S + c] = v;
        }
    }
    wave_sync();
    encode_bins<Q, A, VERIFY>(a, blk, t, tile, lane, use);
}

// The bins of work item (blk, t) from the wave's staged LDS tile; ends with
// the wave done reading the tile.
// `slice`: the block's projection slice when the caller has it (else -1).
template <int Q, class A, bool VERIFY>
__device__ __forceinline__ void encode_bins(const A &a, int64_t blk, int t, const uint64_t *tile,
                                            int lane, uint32_t use, int64_t slice_in) {
    const int P = a.P, W = a.W, H = a.H, S = a.S;
    const int x0 = t * W;
    // The bins whose row-0 crossing -b falls in [x0, x0 + W); the first tile
    // also takes the edge bins with -b < 0, the last those with -b >= P.
    const bool first = (t == 0), last = (t == a.ntiles - 1);
    const int base = H - x0;
    // read once: the stores below cannot alias it
    const int64_t slice = slice_in >= 0 ? slice_in : a.slice(blk);
    for (int i = 0; i < a.n; ++i) {
        const int p = a.dir(i);
        // the stored bins: all of Eq. 2's, or the kept ones (Section 2.3)
        const int bmin = bin_offset(p, P, Q) + a.kept_first(i);
        const int bmax = bmin + a.kept_count(i, proj_bins(p, P, Q)) - 1;
        int bh = first ? bmax : min(bmax, -x0);
        int bl = last ? bmin : max(bmin, -x0 - W + 1);
        const uint64_t *src = nullptr;
        if constexpr (VERIFY) {
            if (!((use >> i) & 1u)) continue;
            src = a.par[i] + blk * a.proj_stride;
        }
        uint64_t *dst = a.proj_in(i, slice);
        const int rstride = S + p;
        for (int b = bl + lane; b <= bh; b += kWave) {
            uint64_t v = 0;
#pragma unroll
            for (int l = 0; l < Q; ++l) v ^= tile[l * rstride + base - b];
            if constexpr (VERIFY) {
                if (v != src[(b - bmin) ^ a.bin_swap]) *a.status = MOJETTE_EINCONSISTENT;
                continue;
            }
            dst[(b - bmin) ^ a.bin_swap] = v;
        }
    }
    wave_sync();  // the next item restages this wave's tile
}

// encode_bins for a tile staged in row windows (the descriptor encode of
// codes of 9 to 12 rows): row l holds columns [x0 + l*plo, x0 + W +
// l*(plo + pspan)), which contain every column that a bin crossing row 0 in
// [x0, x0 + W) meets in row l, and every column inside the image that an
// edge bin of the first or last tile meets there (plo <= 0 <= plo + pspan).
// Edge bins read with a bounds check, the others without.
template <int Q>
__device__ __forceinline__ void encode_bins_rw(const EncodeDesc &a, int t, const uint64_t *tile,
                                               int lane, int64_t slice) {
    const int P = a.P, W = a.W;
    const int x0 = t * W;
    const bool first = (t == 0), last = (t == a.ntiles - 1);
    for (int i = 0; i < a.n; ++i) {
        const int p = a.dir(i);
        const int bmin = bin_offset(p, P, Q) + a.kept_first(i);
        const int bmax = bmin + a.kept_count(i, proj_bins(p, P, Q)) - 1;
        // pixel (l*p - b, l) sits at word base[l] - b of the tile
        int base[Q];
#pragma unroll
        for (int l = 0; l < Q; ++l) base[l] = row_window_off(l, W, a.pspan) + l * (p - a.plo) - x0;
        uint64_t *dst = a.proj_in(i, slice);
        // the bins crossing row 0 in [x0, x0 + W).  Every row's word is
        // read before the first XOR waits for one: left to itself the
        // compiler issued one read per LDS round trip here (8 KB (12,4)
        // tiles of 1 MB blocks: 48.8 against 29.5 ms for the tile-and-halo
        // layout at equal occupancy)
        const int bh = min(bmax, -x0), bl = max(bmin, -x0 - W + 1);
        for (int b = bl + lane; b <= bh; b += kWave) {
            uint64_t w[Q];
#pragma unroll
            for (int l = 0; l < Q; ++l) w[l] = tile[base[l] - b];
            __builtin_amdgcn_sched_barrier(0);
            uint64_t v = 0;
#pragma unroll
            for (int l = 0; l < Q; ++l) v ^= w[l];
            dst[(b - bmin) ^ a.bin_swap] = v;
        }
        // edge bins: crossing row 0 left of column 0 (first tile) or right of
        // the last tile; their columns outside the image count as zero
        auto edge = [&](int lo, int hi) {
            for (int b = lo + lane; b <= hi; b += kWave) {
                uint64_t v = 0;
#pragma unroll
                for (int l = 0; l < Q; ++l)
                    if ((unsigned)(l * p - b) < (unsigned)P) v ^= tile[base[l] - b];
                dst[(b - bmin) ^ a.bin_swap] = v;
            }
        };
        if (first) edge(max(bh + 1, bmin), bmax);
        if (last) edge(bmin, min(bl - 1, bmax));
    }
    wave_sync();  // the next item restages this wave's tile
}

// Tiles of at most PF*64 columns (halo included): each lane keeps its words
// of the next work item's tile in registers, loaded while the current item's
// bins are made and stored, so a wavefront always has loads in flight.  It
// pays where the tiles' LDS leaves few wavefronts per compute unit (5 to 8
// rows: 8 KB (8,4) blocks encode 2.2x faster; 9 to 12 rows, tiles up to 320
// columns: 1 MB (12,4) blocks 2.4x faster); with up to 4 rows 32 wavefronts
// share a unit and the extra registers cost more than they hide (8 KB (4,2)
// blocks 7% slower), and above 12 rows the registers run out.
template <int Q>
constexpr int encode_prefetch_chunks() { return Q >= 5 && Q <= 8 ? 4 : Q >= 9 && Q <= 12 ? 5 : 0; }

template <int Q, int PF>
__device__ __forceinline__ void encode_pipelined(const EncodeArgs &a, uint64_t *tile, int lane,
                                                 int64_t item, int64_t nwaves, int64_t nitems) {
    const int P = a.P, W = a.W, H = a.H, S = a.S;
    uint64_t reg[Q][PF];
    auto fetch = [&](int64_t it) {
        const int64_t blk = it / a.ntiles;
        const int t = (int)(it - blk * a.ntiles);
        const uint64_t *img = a.images + blk * (int64_t)P * Q;
        const int x0 = t * W;
#pragma unroll
        for (int l = 0; l < Q; ++l)
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int c = lane + j * kWave;
                const int col = x0 - H + c;
                reg[l][j] = (c < S && (unsigned)col < (unsigned)P) ? img[(int64_t)l * P + col] : 0;
            }
    };
    if (item >= nitems) return;
    fetch(item);
    for (; item < nitems; item += nwaves) {
#pragma unroll
        for (int l = 0; l < Q; ++l)
#pragma unroll
            for (int j = 0; j < PF; ++j) {
                const int c = lane + j * kWave;
                if (c < S) tile[l * S + c] = reg[l][j];
            }
        wave_sync();
        const int64_t blk = item / a.ntiles;
        const int t = (int)(item - blk * a.ntiles);
        if (item + nwaves < nitems) fetch(item + nwaves);
        encode_bins<Q, EncodeArgs, false>(a, blk, t, tile, lane, 0);
    }
}

template <int Q>
__global__ __launch_bounds__(kWave *kEncodeWaves) void encode_kernel(EncodeArgs a) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x >> 6;
    uint64_t *tile = lds + (size_t)wv * Q * a.S;
    const int64_t nitems = a.nblocks * a.ntiles;
    const int64_t nwaves = (int64_t)gridDim.x * a.waves;
    constexpr int PF = encode_prefetch_chunks<Q>();
    if constexpr (PF > 0) {
        if (a.S <= PF * kWave) {
            encode_pipelined<Q, PF>(a, tile, lane, (int64_t)blockIdx.x * a.waves + wv, nwaves,
                                    nitems);
            return;
        }
    }
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
        encode_item<Q>(a, blk, t, tile, lane);
    }
}

// The consistency check: every work item of every block, as the encode.
template <int Q>
__global__ __launch_bounds__(kWave *kEncodeWaves) void verify_kernel(VerifyArgs a) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x >> 6;
    uint64_t *tile = lds + (size_t)wv * Q * a.S;
    const int64_t nitems = a.nblocks * a.ntiles;
    const int64_t nwaves = (int64_t)gridDim.x * a.waves;
    for (int64_t item = (int64_t)blockIdx.x * a.waves + wv; item < nitems; item += nwaves) {
        const int64_t blk = item / a.ntiles;
        const int t = (int)(item - blk * a.ntiles);
        encode_item<Q, VerifyArgs, true>(a, blk, t, tile, lane);
    }
}

// A mixed launch: items of every class, in the order of the class table
// (heaviest items first), one wavefront per workgroup.
template <int QMAX>
__global__ __launch_bounds__(kWave) void encode_classes_kernel(EncodeClassTable tab) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x;
    const int64_t total = tab.first_item[tab.nclasses];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int c = 0;
        while (item >= tab.first_item[c + 1]) ++c;
        const EncodeClass &a = tab.cls[c];
        const int64_t local = item - tab.first_item[c];
        const int64_t blk = local / a.ntiles;
        const int t = (int)(local - blk * a.ntiles);
        switch (a.Q) {
#define MJ_ENC_CASE(QQ)                                      \
    case QQ:                                                 \
        if constexpr (QQ <= QMAX) encode_item<QQ>(a, blk, t, lds, lane); \
        break;
            MJ_ENC_CASE(1) MJ_ENC_CASE(2) MJ_ENC_CASE(3) MJ_ENC_CASE(4)
            MJ_ENC_CASE(5) MJ_ENC_CASE(6) MJ_ENC_CASE(7) MJ_ENC_CASE(8)
            MJ_ENC_CASE(9) MJ_ENC_CASE(10) MJ_ENC_CASE(11) MJ_ENC_CASE(12)
            MJ_ENC_CASE(13) MJ_ENC_CASE(14) MJ_ENC_CASE(15) MJ_ENC_CASE(16)
#undef MJ_ENC_CASE
            default: break;
        }
    }
}

// A descriptor-driven launch over the items of launch group g (the classes
// of one row count Q), read from the call's workspace.  The items are taken
// grid-stride (below); the class of a wavefront's next item is found by
// stepping forward from the current one; `waves` wavefronts per workgroup,
// each with its own LDS tile of tile_words words.  With PF > 0 (every
// class's tile and halo within PF*64 columns) each lane holds its words of
// the next item's tile in registers, loaded while the current item's bins
// are made: an item's loads are dependent otherwise (class, block index,
// descriptor, image), which left the encode of 1 MB blocks at a third of
// the single-geometry rate.
template <int Q, int PF>
__global__ __launch_bounds__(kWave *kEncodeWaves) void encode_desc_kernel(const uint8_t *__restrict__ ws,
                                                                          int g, int waves,
                                                                          int tile_words) {
    extern __shared__ uint64_t lds[];
    const int lane = threadIdx.x & (kWave - 1);
    // the wavefront's index, uniform across it: the item, its class and the
    // class's fields then live in scalar registers (scalar loads), not in
    // vector loads that share the vector memory counter with the image loads
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const DescHeader &hd = *reinterpret_cast<const DescHeader *>(ws + DescWorkspace::kHeader);
    const int64_t *first = reinterpret_cast<const int64_t *>(ws + DescWorkspace::kFirstItem);
    const EncodeDesc *cls = reinterpret_cast<const EncodeDesc *>(ws + DescWorkspace::kClasses);
    const int64_t lo = hd.range[2 * g], hi = hd.range[2 * g + 1];
    const int64_t nw = (int64_t)gridDim.x * waves;
    // Grid-stride: wave w takes items lo + w, lo + w + nw, ..., so the
    // wavefronts resident at one time work on neighbouring items (the tiles
    // of a long block, consecutive blocks) and their loads and stores stay
    // in a narrow band of the pool.  Measured against contiguous runs per
    // wavefront: 10,000 1 MB (4,2) blocks 6.82 -> 5.04 ms, (6,3) 6.97 ->
    // 5.84, 64 KB (4,2) 0.43 -> 0.36.
    int64_t item = lo + (int64_t)blockIdx.x * waves + wv;
    const int64_t end = hi;
    const int64_t step = nw;
    if (item >= end) return;
    uint64_t *tile = lds + (size_t)wv * tile_words;
    // the class holding the first item: the last c with first[c] <= item
    int c = 0, c1 = hd.nclasses;
    while (c1 - c > 1) {
        const int m = (c + c1) >> 1;
        if (first[m] <= item) c = m; else c1 = m;
    }
    int64_t next = first[c + 1];
    if constexpr (PF == 0) {
        for (; item < end; item += step) {
            while (item >= next) next = first[++c + 1];
            const EncodeDesc &a = cls[c];
            const int64_t local = item - first[c];
            const int64_t blk = local / a.ntiles;
            const int t = (int)(local - blk * a.ntiles);
            encode_item<Q>(a, blk, t, tile, lane);
        }
    } else {
        // RW: row windows (codes of 9 to 12 rows): row l stages its
        // W + l*pspan columns from x0 + l*plo; else every row the tile and
        // both halos, S columns from x0 - H
        constexpr bool RW = encode_row_windows(Q);
        uint64_t reg[Q][PF];
        // the projection slice of the item being fetched, read with its
        // image offset from the one descriptor read of the item
        int64_t f_slice = 0;
        auto fetch = [&](const EncodeDesc &a, int64_t local) {
            const int64_t blk = local / a.ntiles;
            const int t = (int)(local - blk * a.ntiles);
            const mojette_block &b = a.block(blk);
            const uint64_t *img = (const uint64_t *)(a.pool + b.image_off);
            f_slice = (int64_t)b.proj_off;
            const int x0 = t * a.W;
#pragma unroll
            for (int l = 0; l < Q; ++l)
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int cc = lane + j * kWave;
                    const int col = RW ? x0 + l * a.plo + cc : x0 - a.H + cc;
                    const int width = RW ? a.W + l * a.pspan : a.S;
                    reg[l][j] = (cc < width && (unsigned)col < (unsigned)a.P)
                                    ? img[(int64_t)l * a.P + col] : 0;
                }
        };
        fetch(cls[c], item - first[c]);
        while (item < end) {
            const EncodeDesc &a = cls[c];
            const int64_t slice = f_slice;   // the item's block, fetched with its words
#pragma unroll
            for (int l = 0; l < Q; ++l)
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int cc = lane + j * kWave;
                    if constexpr (RW) {
                        if (cc < a.W + l * a.pspan)
                            tile[row_window_off(l, a.W, a.pspan) + cc] = reg[l][j];
                    } else {
                        if (cc < a.S) tile[l * a.S + cc] = reg[l][j];
                    }
                }
            wave_sync();
            const int64_t local = item - first[c];
            const int64_t blk = local / a.ntiles;
            const int t = (int)(local - blk * a.ntiles);
            // the next item and its class; its words load during this one
            const int64_t nit = item + step;
            int c2 = c;
            int64_t next2 = next;
            while (nit >= next2 && nit < end) next2 = first[++c2 + 1];
            if (nit < end) fetch(cls[c2], nit - first[c2]);
            if constexpr (RW)
                encode_bins_rw<Q>(a, t, tile, lane, slice);
            else
                encode_bins<Q, EncodeDesc, false>(a, blk, t, tile, lane, 0, slice);
            item = nit;
            c = c2;
            next = next2;
        }
    }
}

// Register prefetch chunks of a descriptor encode launch of Q rows whose
// tiles and halos span at most max_s columns (0: none fits).
int encode_desc_prefetch(int Q, int max_s) {
    const int pf = Q <= 4 ? 3 : Q <= 8 ? 4 : Q <= 12 ? 5 : 0;
    return pf && max_s <= pf * kWave ? pf : 0;
}

hipError_t launch_encode_desc(int Q, const DescCall &c, int g, int waves, int tile_words,
                              int max_row, int grid, hipStream_t s) {
    const uint8_t *ws = c.ws;
    const size_t lds = (size_t)waves * tile_words * sizeof(uint64_t);
    const int pf = encode_desc_prefetch(Q, max_row);
#define MJ_ENC_LAUNCH2(QQ, PP)                                                                 \
    hipLaunchKernelGGL((encode_desc_kernel<QQ, PP>), dim3(grid), dim3(kWave * waves), lds, s, \
                       ws, g, waves, tile_words)
#define MJ_ENC_LAUNCH(QQ, PPF)                                                                 \
    case QQ:                                                                                   \
        if (pf) MJ_ENC_LAUNCH2(QQ, PPF); else MJ_ENC_LAUNCH2(QQ, 0);                           \
        break;
    switch (Q) {
        MJ_ENC_LAUNCH(1, 3) MJ_ENC_LAUNCH(2, 3) MJ_ENC_LAUNCH(3, 3) MJ_ENC_LAUNCH(4, 3)
        MJ_ENC_LAUNCH(5, 4) MJ_ENC_LAUNCH(6, 4) MJ_ENC_LAUNCH(7, 4) MJ_ENC_LAUNCH(8, 4)
        MJ_ENC_LAUNCH(9, 5) MJ_ENC_LAUNCH(10, 5) MJ_ENC_LAUNCH(11, 5) MJ_ENC_LAUNCH(12, 5)
        case 13: MJ_ENC_LAUNCH2(13, 0); break;
        case 14: MJ_ENC_LAUNCH2(14, 0); break;
        case 15: MJ_ENC_LAUNCH2(15, 0); break;
        case 16: MJ_ENC_LAUNCH2(16, 0); break;
        default: return hipErrorInvalidValue;
    }
#undef MJ_ENC_LAUNCH
#undef MJ_ENC_LAUNCH2
    return hipGetLastError();
}

hipError_t launch_encode_classes(int qmax, const EncodeClassTable &tab, size_t lds, int grid,
                                 hipStream_t s) {
    if (qmax <= 4)
        hipLaunchKernelGGL(encode_classes_kernel<4>, dim3(grid), dim3(kWave), lds, s, tab);
    else if (qmax <= 8)
        hipLaunchKernelGGL(encode_classes_kernel<8>, dim3(grid), dim3(kWave), lds, s, tab);
    else if (qmax <= 12)
        hipLaunchKernelGGL(encode_classes_kernel<12>, dim3(grid), dim3(kWave), lds, s, tab);
    else
        hipLaunchKernelGGL(encode_classes_kernel<16>, dim3(grid), dim3(kWave), lds, s, tab);
    return hipGetLastError();
}

size_t encode_lds_bytes(int Q, int S, int waves) { return (size_t)waves * Q * S * sizeof(uint64_t); }

template <int Q>
static hipError_t launch_q(const EncodeArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(encode_kernel<Q>, dim3(grid), dim3(kWave * a.waves),
                       encode_lds_bytes(Q, a.S, a.waves), s, a);
    return hipGetLastError();
}

template <int Q>
static hipError_t launch_verify_q(const VerifyArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(verify_kernel<Q>, dim3(grid), dim3(kWave * a.waves),
                       encode_lds_bytes(Q, a.S, a.waves), s, a);
    return hipGetLastError();
}

hipError_t launch_verify(const VerifyArgs &a, int grid, hipStream_t s) {
    switch (a.Q) {
        case 1: return launch_verify_q<1>(a, grid, s);
        case 2: return launch_verify_q<2>(a, grid, s);
        case 3: return launch_verify_q<3>(a, grid, s);
        case 4: return launch_verify_q<4>(a, grid, s);
        case 5: return launch_verify_q<5>(a, grid, s);
        case 6: return launch_verify_q<6>(a, grid, s);
        case 7: return launch_verify_q<7>(a, grid, s);
        case 8: return launch_verify_q<8>(a, grid, s);
        case 9: return launch_verify_q<9>(a, grid, s);
        case 10: return launch_verify_q<10>(a, grid, s);
        case 11: return launch_verify_q<11>(a, grid, s);
        case 12: return launch_verify_q<12>(a, grid, s);
        case 13: return launch_verify_q<13>(a, grid, s);
        case 14: return launch_verify_q<14>(a, grid, s);
        case 15: return launch_verify_q<15>(a, grid, s);
        case 16: return launch_verify_q<16>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
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
