// Inverse Mojette transform on gfx950 (Section 2.2), XOR addition: the device
// code shared by the decode translation units (decode_*.hip).
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
// 3.1).  Row r is active on half-steps of the parity of A_r, which is the
// parity of r, so rows 2j and 2j+1 are never active together.
//
// Mapping.  One lane owns the row pair (2j, 2j+1) of one block and works on
// every half-step, alternately on each row; a wavefront holds up to
// 64 / ceil(Q/2) blocks and one workgroup is one wavefront, so no barrier is
// ever needed.  Every row lives in an LDS ring of R words (slot = column mod
// R).  A slot first receives the bin of its column, staged one tile ahead;
// the sweep replaces it by the pixel.  A pixel is read at most D columns
// behind its row's newest pixel (D fixed by the survivor set), and the host
// picks R >= max(2 TW, TW + D + 1) over every survivor set, so a staged bin
// never lands on a pixel that is still needed or not yet stored.  Columns
// outside the image are written as zero and rings start zeroed, so
// dependency reads are never bounds checked.  Equal columns of different
// rows and blocks fall on different LDS banks: for codes of 5 to 8 rows the
// rings are aligned to their length (a slot's address is then the ring's
// address OR'ed with the masked column offset) and the ring of row l in
// block slot s is rotated by s*(Q+1) + l slots; for the others rings are
// R + 1 words apart and block slots an odd number of words apart.
//
// Memory traffic.  A tile is TW columns per row.  After sweeping tile t the
// wave (1) stores, for every row, the TW-aligned window of TW pixels that has
// just been completed (lagging the sweep by less than one tile), (2) writes
// the bins of tile t+1, loaded one tile earlier, into the rings, and (3)
// issues the loads for tile t+2 (t+3 in the body with whole-line loads,
// which has the registers for two tiles in flight).  Only bins of columns
// inside the image are loaded.  Loads and stores are cooperative: TW/2
// consecutive lanes move one row window as 16-byte pieces, so every
// instruction touches whole cache lines (bins are loaded one 8-byte word per
// instruction so that every word is bounds checked on its own).  In pool mode
// (batches) they are raw buffer instructions on the wave's slice of the pool:
// a disabled lane uses an offset past the slice, which the hardware drops
// (stores) or answers with zero (loads).  Every memory instruction is therefore issued
// unconditionally, the compiler knows exactly how many are in flight, and
// waiting for a tile's bins never waits for the stores issued after them.
#pragma once

#include <algorithm>
#include <climits>
#include <type_traits>

#include "mj_internal.h"

namespace mj {

__device__ __forceinline__ int ceil_half(int x) { return x >= 0 ? (x + 1) / 2 : -((-x) / 2); }

template <class T>
constexpr bool kIsDecodeArgs = std::is_same<T, DecodeArgs>::value;

// Descriptor-driven classes (DecodeDesc) find a block's mask, bins and image
// through its descriptor; the other argument types through their pools.
template <class T, class = void>
struct IsDesc : std::false_type {};
template <class T>
struct IsDesc<T, std::void_t<decltype(T::kDesc)>> : std::bool_constant<T::kDesc> {};
template <class T>
constexpr bool kIsDesc = IsDesc<T>::value;

__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o));
    return __builtin_amdgcn_readfirstlane(v);
}

// gfx9 buffer descriptor word 3: 32-bit data format, raw (stride 0) access.
constexpr int kBufferWord3 = 0x00020000;
constexpr uint32_t kOffNone = 0x80000000u;   // past any slice: dropped / reads zero
// Cache policy of the image stores: non-temporal (the decoded image is
// written once and not read again by the decode).  Measured: 4 KB blocks
// decode 1.07x faster; mixed launches of 16 classes 1.07x slower, so those
// keep the default policy.
constexpr int kStreamPolicy = 2;

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint64_t lo64(u32x4 v) { return ((uint64_t)v.y << 32) | v.x; }
__device__ __forceinline__ uint64_t hi64(u32x4 v) { return ((uint64_t)v.w << 32) | v.z; }

// Two consecutive words with one 16-byte store.  The address is only 8-byte
// aligned; gfx950 global stores accept that (unaligned buffer access).
struct __attribute__((aligned(8))) WordPair {
    uint64_t lo, hi;
};
__device__ __forceinline__ void store_pair(uint64_t *dst, uint64_t lo, uint64_t hi) {
    *reinterpret_cast<WordPair *>(dst) = WordPair{lo, hi};
}
typedef uint64_t u64x2_a8 __attribute__((ext_vector_type(2), aligned(8)));
__device__ __forceinline__ void store_pair(global_u64 *dst, uint64_t lo, uint64_t hi) {
    *reinterpret_cast<__attribute__((address_space(1))) u64x2_a8 *>(dst) = u64x2_a8{lo, hi};
}

// A 16-byte pixel or bin (Section 3.1's 128-bit pixels): word 0 is the low
// half.  XOR acts on each word.
struct __attribute__((aligned(16))) Pix128 {
    uint64_t lo, hi;
};
__device__ __forceinline__ Pix128 operator^(Pix128 a, Pix128 b) { return {a.lo ^ b.lo, a.hi ^ b.hi}; }
__device__ __forceinline__ Pix128 &operator^=(Pix128 &a, Pix128 b) { return a = a ^ b; }

// Pixel of W words: uint64_t (W = 1) or Pix128 (W = 2).
template <int W>
using PixT = typename std::conditional<W == 1, uint64_t, Pix128>::type;

template <class T>
__device__ __forceinline__ T pix_zero() { return T{}; }

// Sweep state of one row of one lane (pixels of type T).  Rings are aligned
// to their length (R pixels), so the LDS byte address of a column's slot is
// the ring's offset OR'ed with the masked byte offset of the column: one add
// and one and-or per access.
template <int Q, class T = uint64_t>
struct RowState {
    static constexpr int QM = Q > 1 ? Q - 1 : 1;
    uint32_t ring;           // LDS address of this row's ring
    uint32_t dep[QM];        // LDS addresses of the other rows' rings
    int rot;                 // this ring's rotation (slot of column c: c + rot mod R)
    int delta[QM];           // column offset (l - r) * p_r of each other row, plus its ring's rotation
    int d;                   // first column of tile 0
    bool on;                 // a real row of a decodable block
};

// Reconstructs column k0 + i of one row: the bin staged in the row's slot
// XOR the other rows' pixels on the same line, zero outside the image.
// own / o[m]: byte offsets (before masking) of the row's and the other rows'
// slots for i = 0; M = (R - 1) * sizeof(T).
// EDGE: the column may lie outside the image (else the whole tile of every
// row of the wavefront is inside it and nothing needs zeroing).
template <class T>
using LdsPtr = __attribute__((address_space(3))) T *;

// The LDS address of a ring slot: the ring's address plus the masked byte
// offset of the column; with aligned rings (a ring's address a multiple of
// its byte length) the add is an OR, folded with the mask into one and-or.
template <class T, bool ALN>
__device__ __forceinline__ T *ring_slot(uint32_t ring, uint32_t off, uint32_t M) {
    return (T *)(LdsPtr<T>)(uintptr_t)(ALN ? ring | (off & M) : ring + (off & M));
}

template <int Q, bool EDGE, class T>
__device__ __forceinline__ void sweep_pixel(const RowState<Q, T> &s, uint32_t own,
                                            const uint32_t (&o)[RowState<Q, T>::QM], int k0,
                                            int i, uint32_t M, int P) {
    if (!s.on) return;
    constexpr uint32_t E = sizeof(T);
    constexpr bool ALN = ring_aligned(Q);
    const int k = k0 + i;
    T dv[RowState<Q, T>::QM];
    T *const slot = ring_slot<T, ALN>(s.ring, own + i * E, M);
    const T own_v = *slot;
#pragma unroll
    for (int m = 0; m < Q - 1; ++m) dv[m] = *ring_slot<T, ALN>(s.dep[m], o[m] + i * E, M);
    // Tall codes: every read is issued before the first XOR waits for one
    // (the scheduler splits eight reads into two round trips to LDS
    // otherwise).  Measured: 8 KB (12,8) decode 902 -> 964 GB/s, 1 MB
    // (12,4) 25.0 -> 21.7 ms; 4-row codes 2-5% slower with it, so not there.
    if constexpr (Q > 4) __builtin_amdgcn_sched_barrier(0);
    T v = own_v;
#pragma unroll
    for (int m = 0; m < Q - 1; ++m) v ^= dv[m];
    if (EDGE && (unsigned)k >= (unsigned)P) v = pix_zero<T>();
    *slot = v;
}

// Row window owned by one lane in store/load iteration `it`: segment
// it*SPI + lane/LPS, words 2q, 2q+1 of the window (16-byte pixels: pixels q
// and q + TW/2), q = lane % LPS.  Offsets count pixels (words when W = 1).
struct SegParam {
    int ring;      // LDS index of the segment's ring row (valid slots only)
    int rot;       // its ring's rotation (column c at slot c + rot mod R)
    int gbin;      // pool: offset (in the wave's pool slice) of column 0's bin;
                   // systematic code, known line: of its column 0 in the image slice
                   // pointer mode: bin index of column 0 (jbase)
    int col0;      // column of the lane's first word (pixel) of tile 0's load window
    int scol0;     // first column stored by this lane at tile 0 (window lag applied)
    int mis;       // aligned loads: the row window's offset past a 128-byte line
    int img;       // offset (in the wave's image slice) of the segment's row
    const global_u64 *bins; // pointer mode: the row's projection
    global_u64 *dst;        // descriptor classes: the segment's image row
    int last;      // two-corner sweeps: the last column computed in the row
    bool mir;      // two-corner sweeps: the row belongs to a mirrored sweep
    bool on;       // segment belongs to a block slot in use
    bool known;    // systematic code: a surviving line (staged from the image, not stored)
};

// One batch of up to nb blocks of one geometry, swept by one wavefront.  `A`
// supplies the geometry and buffers (`Args`: DecodeArgs for one pool or one block,
// DecodeClass for one class of a mixed launch).
//
// CHUNK selects what a slot of the wave sweeps (the chunked decode of long
// rows; the tiles of a block are cut into chunks of a.chunk.tiles tiles):
//   kWhole   the whole block (every tile), from zeroed rings;
//   kChunkA  chunk c of the first nchunks-1 chunks of a block, from zeroed
//            rings; chunk 0 stores its image windows (its start state is the
//            true one); every chunk saves its end state (the last E pixels
//            of every row) to the workspace;
//   kChunkC  chunk c >= 1, from its exact start state read from the
//            workspace; stores its image windows.
//   kTwoCorner  (pool mode, whole blocks) two slots per block: side 0
//            sweeps from column 0, side 1 from column P-1.  The image read
//            from its right end is the column-mirror of the image, whose
//            projections are those along (-p, 1) with their bins in reverse
//            order (bin j of direction p is bin B-1-j of direction -p of the
//            mirror), so side 1 is the same sweep on the mirrored block: its
//            rows take the survivors in ascending -p, it loads its bins in
//            ascending order and stores its pixels at mirrored columns.  A
//            sweep stopped after any number of tiles has computed a set of
//            pixels that holds every pixel each of them depends on (all are
//            earlier in the sweep), and both are exact.  Each side sweeps
//            until every row has reached the middle column from its end,
//            about half the tiles of a whole sweep, then stores the pixels
//            it has computed; columns both reach are stored twice with the
//            same words.  The dependency chain of a block is about halved.
//
// NBT is the most block slots the body is compiled for (a.nb <= NBT): the
// full 64 / ceil(Q/2), or half of it when long rings leave LDS for no more,
// which saves the registers of the unused row windows.
//
// STPOL is the cache policy of the image stores in pool mode (kStreamPolicy:
// non-temporal; 0: default).
//
// SYS: the systematic code (DecodeArgs only, whole blocks, pool mode).  A
// block is Q data lines stored as they are (the image) plus a.n parity
// projections in the pool (mask bits 0..Q-1 lines, then projections).  The
// rows are the Q lines.  The lost ones, in ascending order, are swept: the
// r-th lost line m_r takes the r-th surviving projection in ascending p, and
// A_{r+1} = A_r + 2 (m_{r+1} - m_r) p_r + 1, which keeps every dependency on
// another lost line strictly earlier: for l > r the gap is
// sum 2 (m_{i+1} - m_i)(p_i - p_r) + (l - r) > 0, and for l < r it is at
// least sum 2 (m_{i+1} - m_i)(p_r - p_i) - (r - l) >= (r - l)^2 > 0.  Rows
// of consecutive sweep index still alternate in parity.  The surviving
// lines are known: their windows are staged into their rings from the image
// instead of bins, so the sweep reads their pixels as it reads the lost
// lines' (no pass removes them from the parity bins first).
//
// ALIGN (pool mode): each row's bins are loaded as the 128-byte line where
// the tile's window starts, and the words of that line that belong to the
// next tile are kept in registers until then, so no line is fetched for two
// tiles (an unaligned 16-word window shares a line with the next tile's,
// and the line is gone from L2 by then).  The held words cost registers:
// only the bodies compiled for half the slots take it.
//
// RCLS: the launch sweeps one ring class only (a.ring_mode, see below).  A
// separate instantiation, so that launches over every block carry none of
// its code (with it, they measured up to 30% slower).
//
// W: words per pixel.  W = 2 sweeps 128-bit pixels (Section 3.1) in the
// 16-byte image's own geometry: ring slots, bins and pixels of 16 bytes,
// P, strides and offsets counted in pixels.  A lane of a row window then
// moves the pixels of columns c and c - TW/2, so each memory instruction
// covers TW/2 consecutive pixels (a 128-byte line when aligned).  Whole-
// block pool sweeps only.
template <int Q, int TW, bool POOL, int CHUNK, int NBT, class Args, int STPOL = kStreamPolicy,
          bool SYS = false, bool ALIGN = false, bool RCLS = false, int W = 1>
__device__ __forceinline__ void decode_batch(const Args &a, const int64_t batch,
                                             const int64_t gather_blk = -1,
                                             const int64_t gather_lo = 0,
                                             const int64_t gather_hi = 0) {
    static_assert(W == 1 || (W == 2 && POOL && CHUNK == kWhole && !SYS && !RCLS),
                  "16-byte pixels: whole-block pool sweeps only");
    using T = PixT<W>;
    extern __shared__ uint64_t lds_words[];
    T *const lds = reinterpret_cast<T *>(lds_words);
    constexpr int LPB = (Q + 1) / 2;        // lanes per block
    constexpr int NBMAX = NBT;              // blocks per wavefront at most
    // Lanes per row window: each moves two words (W = 1) or two 16-byte
    // pixels TW/2 columns apart (W = 2).
    constexpr int LPS = TW / 2;
    constexpr int SPI = kWave / LPS;        // row windows per iteration
    constexpr int NIT = (NBMAX * Q + SPI - 1) / SPI;
    constexpr int QM = RowState<Q, T>::QM;

    const int lane = threadIdx.x;
    const int slot = lane / LPB;
    const int j = lane - slot * LPB;
    const int NB = a.nb;
    const bool lane_used = slot < NB;
    // Slot -> (block, chunk).  A wave's slots cover consecutive blocks
    // [blk_lo, blk_hi]; `rel` is the slot's block relative to blk_lo.
    int per = 1;                             // slots per block
    if constexpr (CHUNK == kChunkA || CHUNK == kChunkC) per = a.chunk.nchunks - 1;
    if constexpr (CHUNK == kTwoCorner) per = 2;
    const int64_t item = batch * NB + slot;
    // Gathered slots (ring class 2, see decode_deep_kernel): the slot's block
    // is given, within the wave's slice [gather_lo, gather_hi).
    const bool gathered = RCLS && gather_blk >= 0;
    const int64_t blk = gathered ? gather_blk : item / per;
    int chunk = 0, shift = 0;                // chunk index, its first column offset
    if constexpr (CHUNK == kChunkA || CHUNK == kChunkC) {
        chunk = (int)(item - blk * per) + (CHUNK == kChunkC ? 1 : 0);
        shift = chunk * a.chunk.tiles * TW;
    }
    // two-corner sweeps: side 1 sweeps the column-mirrored block
    const bool mir = CHUNK == kTwoCorner && (item - blk * per) == 1;
    const int64_t blk_lo = gathered ? gather_lo : batch * NB / per;
    const int rel = (int)(blk - blk_lo);
    // Rings (ring_stride_of): aligned to their length R for ring_aligned(Q),
    // else R + 1 words apart in block slots of an odd number of words.
    constexpr bool ALN = ring_aligned(Q);
    const int RS = a.ring_stride;
    const int SS = Q * RS + (ALN ? 0 : 1);  // pixels per block slot
    const int Rmask = a.R - 1;
    // Aligned rings: column c of row l of block slot sl at slot
    // (c + rot(sl, l)) mod R.  The rotation spreads equal columns of
    // different rows and slots over the LDS banks as the odd strides do.
    auto rot_of = [&](int sl, int l) { return ALN ? (sl * (Q + 1) + l) & Rmask : 0; };
    if (RS != ring_stride_of(Q, a.R)) {
        // anything but the host's layout would break the slot addresses
        if (lane == 0 && a.status) a.status[0] = MOJETTE_EINVAL;
        return;
    }
    const int P = a.P;
    // pointer mode and chunked sweeps, 128-bit pixels as the word image of
    // twice the width: word bin j stored at word j ^ 1.  Read once: a class
    // table is global memory that the loop's stores might alias, so a field
    // read inside it is a vector load each time (and its wait would also
    // wait for the bins loaded ahead).
    int bswap = 0;
    if constexpr (kIsDesc<Args> || kIsDecodeArgs<Args>)
        if (!POOL || CHUNK == kChunkA || CHUNK == kChunkC)
            bswap = __builtin_amdgcn_readfirstlane(a.bin_swap);
    T *slot_base = lds + (size_t)(lane_used ? slot : 0) * SS;
    const uint32_t RM = (uint32_t)Rmask * sizeof(T);   // byte mask of a ring
    // LDS address of the dynamic array (0 in these kernels, which declare no
    // other LDS): rings are aligned to their byte length within it
    const uint32_t lds_at = (uint32_t)(uintptr_t)(LdsPtr<T>)lds;
    if (ALN && (lds_at & (RM | (sizeof(T) - 1))) != 0) {
        if (lane == 0 && a.status) a.status[0] = MOJETTE_EINVAL;
        return;
    }
    const int r0 = 2 * j, r1 = 2 * j + 1;   // this lane's rows
    const int q = lane % LPS;
    const int QP = Q * P;

    {
        const bool blk_ok = lane_used && blk < (gathered ? gather_hi : a.nblocks);
        uint32_t mask = a.mask_uniform;
        if constexpr (kIsDesc<Args>) {
            if (blk_ok) mask = a.mask_of(blk);
        } else {
            if (blk_ok && a.masks) mask = a.masks[blk];
        }

        // Survivors in ascending p; row r takes the r-th.
        int p0 = 0, p1 = 0, id0 = 0, id1 = 0, A0 = 0, A1 = 0;
        int A_max = INT_MIN, A_min = INT_MAX, cnt = 0, psum = 0;
        uint32_t used = 0;
        // Systematic code: the rows are the block's lines.  The `nrows` lost
        // ones are the sweep rows: sweep row s is line msw[s] (ascending)
        // and takes the s-th surviving parity projection in ascending p
        // (its p in psw[s], its A in Asw[s]).  The others are known: their
        // rings are filled from the image, and they are never swept.
        int nrows = Q;
        uint32_t pbase = 0;                 // mask bit of projection 0
        uint32_t lost = 0;
        constexpr int QS = SYS ? Q : 1;
        int msw[QS], Asw[QS], psw[QS];
        if constexpr (SYS) {
            lost = mask & ((1u << Q) - 1u);
            nrows = __builtin_popcount(lost);
            uint32_t rest = lost;
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                msw[r] = rest ? __builtin_ctz(rest) : 0;
                rest &= rest - 1u;
                Asw[r] = 0;
                psw[r] = 0;
            }
            pbase = Q;
        }
        int A_next = 0;                     // SYS: A of sweep row cnt
        for (int s = 0; s < a.n; ++s) {
            // the mirrored block's directions, -p, ascend in reverse order
            const int sx = mir ? a.n - 1 - s : s;
            const int id = a.id_sorted[sx];
            const int p = mir ? -a.p_sorted[sx] : a.p_sorted[sx];
            if (!((mask >> (pbase + id)) & 1u) && cnt < nrows) {
                int A = 2 * psum + cnt;
                if constexpr (SYS) {
                    A = A_next;
                    int m_here = 0, m_next = 0;   // lines of sweep rows cnt, cnt + 1
#pragma unroll
                    for (int r = 0; r < Q; ++r) {
                        m_here = r == cnt ? msw[r] : m_here;
                        m_next = r == cnt + 1 ? msw[r] : m_next;
                        if (r == cnt) {
                            Asw[r] = A;
                            psw[r] = p;
                        }
                    }
                    A_next = A + 2 * (m_next - m_here) * p + 1;
                    if (m_here == r0) { p0 = p; id0 = id; A0 = A; }
                    if (m_here == r1) { p1 = p; id1 = id; A1 = A; }
                } else {
                    if (cnt == r0) { p0 = p; id0 = id; A0 = A; }
                    if (cnt == r1) { p1 = p; id1 = id; A1 = A; }
                }
                A_max = max(A_max, A);
                A_min = min(A_min, A);
                psum += p;
                used |= 1u << id;
                ++cnt;
            }
        }
        bool valid = blk_ok;
        if constexpr (SYS) {
            if (nrows == 0) valid = false;   // every line survived: nothing to rebuild
        }
        if (valid && cnt < nrows) {
            // reported once per block: by its whole sweep or its first chunk
            if (blk_ok && j == 0 && a.status &&
                (CHUNK == kWhole || (CHUNK == kChunkA && chunk == 0) || (CHUNK == kTwoCorner && !mir)))
                a.status[0] = MOJETTE_ENOTRECON;
            valid = false;
        }
        // Ring classes (whole-block pool sweeps of DecodeArgs): ring_mode 1
        // takes only the blocks whose survivor set reads at most
        // a.ring_depth columns behind the newest pixel of a row (the short
        // ring of this launch serves them), ring_mode 2 only the others.
        // The depth of a set is the largest ceil((A_l - A_r)/2) - 1 -
        // (l - r) p_r.
        if constexpr (RCLS && CHUNK == kWhole && !SYS && POOL && kIsDecodeArgs<Args>) {
            {
                int depth = INT_MIN;
                if (valid) {
                    int c2 = 0, ps2 = 0;
                    for (int s = 0; s < a.n; ++s) {
                        const int id = a.id_sorted[s];
                        const int p = a.p_sorted[s];
                        if (!((mask >> id) & 1u) && c2 < Q) {
                            const int A = 2 * ps2 + c2;
                            if (c2 != r0 && r0 < Q)
                                depth = max(depth, ceil_half(A - A0) - 1 - (c2 - r0) * p0);
                            if (c2 != r1 && r1 < Q)
                                depth = max(depth, ceil_half(A - A1) - 1 - (c2 - r1) * p1);
                            ps2 += p;
                            ++c2;
                        }
                    }
                }
                // a block's rows are spread over its LPB lanes
                int bdepth = depth;
#pragma unroll
                for (int jj = 0; jj < LPB; ++jj) bdepth = max(bdepth, __shfl(depth, slot * LPB + jj));
                const bool fits = bdepth <= a.ring_depth;
                if (a.ring_mode == 1 ? !fits : fits) valid = false;
                if (!__any(valid)) return;   // nothing for this wavefront in this launch
            }
        }
        // Chunked sweeps: the state width E of this survivor set.
        int E = 0;
        if constexpr (CHUNK == kChunkA || CHUNK == kChunkC) {
            if (valid) E = a.chunk.state_cols[a.chunk.lut[used]];
        }
        // Half-step of pixel (k, r) within the block: h = 2k - A_r + A_max.
        // Rows with (r & 1) == (A_max & 1) have even h (row X of a lane),
        // the others odd h (row Y).  In tile t, half-steps [2TW t, 2TW(t+1)),
        // row X handles column t*TW + d + i at half-step 2i and row Y column
        // t*TW + d + i at half-step 2i + 1 (d <= 0 per row).  A row stores
        // window m = t - L at the end of tile t, L = ceil(-d / TW); the
        // block is done once its rows have stored the window of column P-1.
        const int par = A_max & 1;
        const int dmin = valid ? -((A_max - A_min) >> 1) : 0;
        const int ntiles_all = valid ? (P - 1) / TW + (-dmin + TW - 1) / TW + 1 : 0;
        int ntiles = ntiles_all;                 // tiles this slot sweeps
        // Chunked sweeps store a window at local tile t < a.chunk.tiles when
        // bit `it` of store_in is set, at later tiles when bit `it` of
        // store_past is: the first sweep stores chunk 0 only, the final
        // sweep every chunk, the last one through its end.
        int first_last = 0;                      // this slot's chunk is the first (1), last (2)
        if constexpr (CHUNK == kChunkA) {
            ntiles = valid ? a.chunk.tiles : 0;
            first_last = chunk == 0 ? 1 : 0;
        } else if constexpr (CHUNK == kChunkC) {
            const int first_tile = chunk * a.chunk.tiles;
            ntiles = !valid ? 0
                     : chunk < a.chunk.nchunks - 1 ? a.chunk.tiles
                                                   : ntiles_all - first_tile;
            first_last = chunk == a.chunk.nchunks - 1 ? 2 : 0;
        } else if constexpr (CHUNK == kTwoCorner) {
            // every row reaches column H (side 0) or P - H (side 1, from its
            // end) once the sweep has passed the row with the largest skew
            const int H = (P + 1) / 2;
            const int half = mir ? P - H : H;
            ntiles = valid ? min(ntiles_all, (half - dmin + TW - 1) / TW) : 0;
        }
        const int ntiles_wave = wave_max(ntiles);

        RowState<Q, T> X, Y;
        // Swept rows: every row, or (systematic code) the lost lines.  Row X
        // of a lane is the one whose A has the parity of A_max (A_r = r mod
        // 2 without the systematic code; with it, a lane's two lines are
        // consecutive sweep rows when both are lost, so their A differ in
        // parity).
        const bool sw0 = SYS ? ((lost >> r0) & 1u) != 0 : r0 < nrows;
        const bool sw1 = SYS ? r1 < Q && ((lost >> r1) & 1u) != 0 : r1 < nrows;
        bool r0_is_x = ((r0 & 1) == par);
        if constexpr (SYS) r0_is_x = sw0 ? (A0 & 1) == par : !(sw1 && (A1 & 1) == par);
        int jb0 = 0, jb1 = 0;   // bin index of column 0 for rows r0 and r1
        {
            const int rx = r0_is_x ? r0 : r1, ry = r0_is_x ? r1 : r0;
            const int px = r0_is_x ? p0 : p1, py = r0_is_x ? p1 : p0;
            const int Ax = r0_is_x ? A0 : A1, Ay = r0_is_x ? A1 : A0;
            X.on = valid && (r0_is_x ? sw0 : sw1);
            Y.on = valid && (r0_is_x ? sw1 : sw0);
            const uint32_t sb = lds_at + (uint32_t)((slot_base - lds) * sizeof(T));   // slot's address
            const int ss = lane_used ? slot : 0;
            X.ring = sb + (uint32_t)((rx < Q ? rx : 0) * RS * sizeof(T));
            Y.ring = sb + (uint32_t)((ry < Q ? ry : 0) * RS * sizeof(T));
            X.rot = rot_of(ss, rx < Q ? rx : 0);
            Y.rot = rot_of(ss, ry < Q ? ry : 0);
#pragma unroll
            for (int m = 0; m < Q - 1; ++m) {
                const int lx = m + (m >= rx ? 1 : 0), ly = m + (m >= ry ? 1 : 0);
                X.dep[m] = sb + (uint32_t)((lx < Q ? lx : 0) * RS * sizeof(T));
                Y.dep[m] = sb + (uint32_t)((ly < Q ? ly : 0) * RS * sizeof(T));
                X.delta[m] = (lx - rx) * px + rot_of(ss, lx < Q ? lx : 0);
                Y.delta[m] = (ly - ry) * py + rot_of(ss, ly < Q ? ly : 0);
            }
            X.d = X.on ? -((A_max - Ax) >> 1) : 0;       // (Ax - A_max)/2, exact
            Y.d = Y.on ? -((A_max - Ay - 1) >> 1) : 0;   // (Ay - A_max + 1)/2, exact
            jb0 = r0 * p0 - (bin_offset(p0, P, Q) + a.kept_first(id0));
            jb1 = r1 * p1 - (bin_offset(p1, P, Q) + a.kept_first(id1));
            if (mir) {
                // bin j of the mirrored block's projection is bin B-1-j of the
                // stored one: column 0's bin, whose index then ascends with c
                jb0 = proj_bins(p0, P, Q) - 1 - jb0;
                jb1 = proj_bins(p1, P, Q) - 1 - jb1;
            }
        }

        // Per-iteration row windows, from the lanes that own their rows.
        int dr0 = r0_is_x ? X.d : Y.d;           // first column of tile 0, unshifted
        int dr1 = r0_is_x ? Y.d : X.d;
        // Systematic code: a known line l is read by sweep row s at columns
        // t*TW + d_s + (l - msw[s]) psw[s] + i during tile t (i < TW), so its
        // windows are staged at the furthest of those offsets; the ring
        // (long enough for the spread of the offsets, with a.sys_lead tiles
        // staged ahead of the sweep) keeps the nearest.
        if constexpr (SYS) {
            int k0 = INT_MIN, k1 = INT_MIN;
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                if (r < nrows) {
                    const int ds = -((A_max - Asw[r]) >> 1);
                    k0 = max(k0, ds + (r0 - msw[r]) * psw[r]);
                    k1 = max(k1, ds + (r1 - msw[r]) * psw[r]);
                }
            }
            if (!sw0) dr0 = k0;
            if (!sw1) dr1 = k1;
        }
        SegParam sp[NIT];
        uint32_t store_in = 0, store_past = 0;   // chunked sweeps: see first_last
        constexpr bool AL = POOL && ALIGN;
        // loads two tiles ahead (the 64-bit body's registers allow it)
        constexpr bool DEEP = AL && W == 1;
        // aligned loads: offset of the wave's pool slice past a 128-byte
        // line, in pixels (16 words or 8 pixels of 16 bytes per line)
        constexpr int kLinePix = 128 / (8 * W);
        const int slice_mis =
            AL ? (int)(((uintptr_t)(a.pool + blk_lo * a.proj_stride * W) >> (W == 1 ? 3 : 4)) &
                       (kLinePix - 1))
               : 0;
        {
            // pool mode: word offset of column 0's bin within the wave's
            // slice (a known line: of its column 0 in the image slice)
            int g0 = POOL ? rel * (int)a.proj_stride + a.off[id0] + jb0 : jb0;
            int g1 = POOL ? rel * (int)a.proj_stride + a.off[id1] + jb1 : jb1;
            if constexpr (SYS) {
                if (!sw0) g0 = rel * QP + r0 * P;
                if (!sw1) g1 = rel * QP + r1 * P;
            }
            // rows whose windows are staged (and, unless known, stored)
            const bool st0 = SYS ? r0 < Q : sw0, st1 = SYS ? r1 < Q : sw1;
            const int own0 = valid && st0 ? dr0 : INT_MIN;
            const int own1 = valid && st1 ? dr1 : INT_MIN;
            const int known = SYS && valid ? (!sw0 ? 1 : 0) | (!sw1 ? 2 : 0) : 0;
            // pointer mode: the projections of this lane's two rows (and,
            // for descriptor classes, its block's image)
            uint64_t pb0 = 0, pb1 = 0, ib = 0;
            if constexpr (!POOL) {
                if (valid) {
                    pb0 = (uint64_t)a.proj_base(blk, id0);
                    pb1 = (uint64_t)a.proj_base(blk, id1);
                    if constexpr (kIsDesc<Args>) ib = (uint64_t)a.image_of(blk);
                }
            }
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int seg = it * SPI + lane / LPS;
                const int sslot = seg / Q;
                const int srow = seg - sslot * Q;
                const int owner = sslot * LPB + (srow >> 1);
                const int src = owner < kWave ? owner : 0;
                const int od0 = __shfl(own0, src), od1 = __shfl(own1, src);
                const int og0 = __shfl(g0, src), og1 = __shfl(g1, src);
                const int orow = srow;           // image row of the segment
                int orel = sslot, oshift = 0;   // whole blocks: slot = block
                if constexpr (RCLS) {
                    // gathered slots: the owner's block, not the slot's index
                    const int srel = __shfl(rel, src);
                    if (gathered) orel = srel;
                }
                if constexpr (CHUNK == kTwoCorner) orel = __shfl(rel, src);
                if constexpr (CHUNK == kChunkA || CHUNK == kChunkC) {
                    orel = __shfl(rel, src);
                    oshift = __shfl(shift, src);
                    const int ofl = __shfl(first_last, src);
                    const bool in = CHUNK == kChunkC || (ofl & 1);
                    store_in |= (uint32_t)in << it;
                    store_past |= (uint32_t)((ofl >> 1) & 1) << it;
                }
                const bool odd = srow & 1;
                const int sd = odd ? od1 : od0;
                SegParam &s = sp[it];
                s.on = sslot < NB && sd != INT_MIN;
                s.known = false;
                if constexpr (SYS) {
                    const int okn = __shfl(known, src);
                    s.known = s.on && ((okn >> (odd ? 1 : 0)) & 1);
                }
                const int dd = s.on ? sd : 0;
                s.mir = false;
                s.last = INT_MAX;
                if constexpr (CHUNK == kTwoCorner) {
                    s.mir = __shfl(mir ? 1 : 0, src) != 0;
                    // the last column the sweep computes in this row
                    s.last = ntiles_wave * TW + dd - 1;
                }
                s.ring = (sslot < NB ? sslot : 0) * SS + srow * RS;
                s.rot = rot_of(sslot < NB ? sslot : 0, srow);
                s.gbin = odd ? og1 : og0;
                s.bins = nullptr;
                s.dst = nullptr;
                if constexpr (!POOL) {
                    // both rows' pointers come over; the requester picks
                    const uint32_t lo0 = __shfl((uint32_t)pb0, src);
                    const uint32_t hi0 = __shfl((uint32_t)(pb0 >> 32), src);
                    const uint32_t lo1 = __shfl((uint32_t)pb1, src);
                    const uint32_t hi1 = __shfl((uint32_t)(pb1 >> 32), src);
                    s.bins = (const global_u64 *)(odd ? (((uint64_t)hi1 << 32) | lo1)
                                                    : (((uint64_t)hi0 << 32) | lo0));
                    if constexpr (kIsDesc<Args>) {
                        const uint32_t ilo = __shfl((uint32_t)ib, src);
                        const uint32_t ihi = __shfl((uint32_t)(ib >> 32), src);
                        s.dst = (global_u64 *)(((uint64_t)ihi << 32) | ilo) + orow * P;
                    }
                }
                s.col0 = dd + TW - 1 - (W == 1 ? 2 * q : q) + oshift;
                // the window of tile t starts at word gbin - col0 - 2q - TW*t
                s.mis = AL ? (slice_mis + s.gbin - s.col0 - (W == 1 ? 2 * q : q)) & (kLinePix - 1)
                           : 0;
                const int L = (-dd + TW - 1) / TW;
                s.scol0 = -TW * L + (W == 1 ? 2 * q : q) + oshift;
                s.img = orel * QP + orow * P;
            }
        }

        // The sweep of a chunk starts `shift` columns in.
        X.d += shift;
        Y.d += shift;

        // Buffer descriptors of this wave's pool and image slices.
        const int64_t first = blk_lo;
        const int64_t blk_hi =
            gathered ? gather_hi : min(a.nblocks, (batch * NB + NB + per - 1) / per);
        const int64_t nblk = blk_hi - first;
        __amdgpu_buffer_rsrc_t rin, rout;
        if constexpr (POOL) {
            rin = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.pool + first * a.proj_stride * W), 0,
                (int)(nblk * a.proj_stride * sizeof(T)), kBufferWord3);
            rout = __builtin_amdgcn_make_buffer_rsrc(
                (void *)(a.images + first * a.img_stride * W), 0,
                (int)(nblk * a.img_stride * sizeof(T)), kBufferWord3);
        }

        // Loads the bins of tile t: words 2q, 2q+1 of each row window are the
        // bins of columns c and c - 1, c = t*TW + col0.  Aligned loads take
        // the line where the window starts instead: its words 2q, 2q+1 are
        // window words 2q - mis and 2q + 1 - mis, and those below 0 belong
        // to the window of tile t+1 (see stage_tile).
        auto load_tile = [&](int t, u32x4 (&buf)[NIT * W]) {
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const SegParam &s = sp[it];
                const int c = t * TW + s.col0;
                if constexpr (W == 2) {
                    // 16-byte bins of columns c and c - TW/2: each load
                    // instruction covers TW/2 consecutive bins of a row
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        // aligned loads: the two lines from where the window
                        // starts; pixels below mis belong to tile t+1
                        const int ch = c + (AL ? s.mis : 0) - h * LPS;
                        const bool in = s.on && (unsigned)ch < (unsigned)P;
                        const uint32_t off = in ? (uint32_t)(s.gbin - ch) * 16u : kOffNone;
                        buf[it * W + h] = __builtin_amdgcn_raw_buffer_load_b128(rin, off, 0, 0);
                    }
                } else if constexpr (POOL) {
                    // one 8-byte load per word, so each word is bounds checked
                    // on its own (a window may start just before the slice).
                    // Only columns inside the image load: the sweep zeroes the
                    // pixels of the others whatever their bins hold, so the
                    // lines a row's window covers before column 0 and past
                    // column P-1 are never fetched.
                    int w = s.gbin - c - (AL ? s.mis : 0);
                    int wn = w + 1;                           // the word of column cw - 1
                    if constexpr (CHUNK == kTwoCorner) {
                        // a mirrored sweep's bins ascend with its column
                        if (s.mir) {
                            w = s.gbin + c;
                            wn = w - 1;
                        }
                    }
                    if constexpr (CHUNK == kChunkA || CHUNK == kChunkC) {
                        // 128-bit pixels (the projections of the block's
                        // slice have even lengths, so a word's pair
                        // partner is in the same projection)
                        w ^= bswap;
                        wn ^= bswap;
                    }
                    const int cw = c + (AL ? s.mis : 0);     // column of word 2q
                    const bool in0 = s.on && (unsigned)cw < (unsigned)P;
                    const bool in1 = s.on && (unsigned)(cw - 1) < (unsigned)P;
                    const uint32_t off0 = in0 && !s.known ? (uint32_t)w * 8u : kOffNone;
                    const uint32_t off1 = in1 && !s.known ? (uint32_t)wn * 8u : kOffNone;
                    u32x2 w0 = __builtin_amdgcn_raw_buffer_load_b64(rin, off0, 0, 0);
                    u32x2 w1 = __builtin_amdgcn_raw_buffer_load_b64(rin, off1, 0, 0);
                    if constexpr (SYS) {
                        // a known line's pixels from the image (words ascend
                        // with the column); the other load of each pair is
                        // disabled and reads zero
                        const int wi = s.gbin + c;
                        const bool k0 = in0 && s.known, k1 = in1 && s.known;
                        const uint32_t oi0 = k0 ? (uint32_t)wi * 8u : kOffNone;
                        const uint32_t oi1 = k1 ? (uint32_t)(wi - 1) * 8u : kOffNone;
                        const u32x2 i0 = __builtin_amdgcn_raw_buffer_load_b64(rout, oi0, 0, 0);
                        const u32x2 i1 = __builtin_amdgcn_raw_buffer_load_b64(rout, oi1, 0, 0);
                        w0 = w0 | i0;
                        w1 = w1 | i1;
                    }
                    buf[it] = u32x4{w0.x, w0.y, w1.x, w1.y};
                } else {
                    const global_u64 *bins = s.bins;
                    const int c0 = min(max(c, 0), P - 1), c1 = min(max(c - 1, 0), P - 1);
                    // a mirrored sweep's bins ascend with its column
                    const int sg = CHUNK == kTwoCorner && s.mir ? -1 : 1;
                    const uint64_t w0 = s.on ? bins[(s.gbin - sg * c0) ^ bswap] : 0;
                    const uint64_t w1 = s.on ? bins[(s.gbin - sg * c1) ^ bswap] : 0;
                    buf[it] = u32x4{(uint32_t)w0, (uint32_t)(w0 >> 32), (uint32_t)w1,
                                    (uint32_t)(w1 >> 32)};
                }
            }
        };
        // Writes the bins of tile t into the rings: `buf` holds the loads of
        // tile t, `prev` (aligned loads) those of tile t-1.  Window word v of
        // tile t is column t*TW + col0 + 2q - v; with aligned loads it is word
        // v + mis of this tile's line when v + mis < TW, else word
        // v + mis - TW of the previous tile's line.
        auto stage_tile = [&](int t, const u32x4 (&buf)[NIT * W],
                              const u32x4 (&prev)[AL ? NIT : 1]) {
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const SegParam &s = sp[it];
                if (!s.on) continue;
                T *row = lds + s.ring;
                if constexpr (W == 2) {
                    const int c = t * TW + s.col0 + (AL ? s.mis : 0);
                    // the first pixel: held for tile t+1 when below mis (the
                    // previous tile's, from `prev`, goes in instead)
                    const bool held = AL && q < s.mis;
                    const u32x4 v0 = held ? prev[AL ? it : 0] : buf[it * W];
                    row[(c - (held ? TW : 0) + s.rot) & Rmask] = Pix128{lo64(v0), hi64(v0)};
                    row[(c - LPS + s.rot) & Rmask] =
                        Pix128{lo64(buf[it * W + 1]), hi64(buf[it * W + 1])};
                } else if constexpr (AL) {
                    const int c = t * TW + s.col0 + s.mis;   // column of this line's word 2q
                    const bool h0 = 2 * q < s.mis, h1 = 2 * q + 1 < s.mis;
                    row[(c - (h0 ? TW : 0) + s.rot) & Rmask] = h0 ? lo64(prev[it]) : lo64(buf[it]);
                    row[(c - 1 - (h1 ? TW : 0) + s.rot) & Rmask] = h1 ? hi64(prev[it]) : hi64(buf[it]);
                } else {
                    const int c = t * TW + s.col0 + s.rot;
                    row[c & Rmask] = lo64(buf[it]);
                    row[(c - 1) & Rmask] = hi64(buf[it]);
                }
            }
        };
        // Stores the completed TW-aligned window of every row at the end of
        // tile t: columns t*TW + scol0 and the next one (16-byte pixels:
        // t*TW + scol0 and TW/2 columns further).
        auto store_tile = [&](int t, bool flush = false) {
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const SegParam &s = sp[it];
                const int c = t * TW + s.scol0;
                const T *row = lds + s.ring;
                if constexpr (W == 2) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int ch = c + h * LPS;
                        const Pix128 v = row[(ch + s.rot) & Rmask];
                        const bool in = s.on && (unsigned)ch < (unsigned)P;
                        const uint32_t off = in ? (uint32_t)(s.img + ch) * 16u : kOffNone;
                        __builtin_amdgcn_raw_buffer_store_b128(
                            u32x4{(uint32_t)v.lo, (uint32_t)(v.lo >> 32), (uint32_t)v.hi,
                                  (uint32_t)(v.hi >> 32)},
                            rout, off, 0, STPOL);
                    }
                } else {
                    const uint64_t w0 = row[(c + s.rot) & Rmask], w1 = row[(c + 1 + s.rot) & Rmask];
                    bool in_chunk = true;
                    if constexpr (CHUNK == kChunkA || CHUNK == kChunkC)
                        in_chunk = ((t < a.chunk.tiles ? store_in : store_past) >> it) & 1u;
                    const bool put = s.on && !s.known && in_chunk;
                    // the last column to store: P - 1, or (a two-corner
                    // sweep's final store) the last one it computed
                    int hi = P - 1;
                    if constexpr (CHUNK == kTwoCorner) {
                        if (flush) hi = min(hi, s.last);
                    }
                    const bool both = put && c >= 0 && c + 1 <= hi;
                    const bool last = put && c >= 0 && c == hi;
                    if constexpr (POOL) {
                        // a mirrored sweep's columns c, c+1 are the block's
                        // columns P-1-c, P-2-c: the pair goes in reverse
                        int cp = c, cs = c;
                        uint64_t lo = w0, hi2 = w1;
                        if constexpr (CHUNK == kTwoCorner) {
                            if (s.mir) {
                                cp = P - 2 - c;
                                cs = P - 1 - c;
                                lo = w1;
                                hi2 = w0;
                            }
                        }
                        const uint32_t off2 = both ? (uint32_t)(s.img + cp) * 8u : kOffNone;
                        const uint32_t off1 = last ? (uint32_t)(s.img + cs) * 8u : kOffNone;
                        __builtin_amdgcn_raw_buffer_store_b128(
                            u32x4{(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi2,
                                  (uint32_t)(hi2 >> 32)},
                            rout, off2, 0, STPOL);
                        // only an odd row length leaves a single last word
                        // (and a two-corner sweep's last computed column)
                        if ((P & 1) || CHUNK == kTwoCorner)
                            __builtin_amdgcn_raw_buffer_store_b64(
                                u32x2{(uint32_t)w0, (uint32_t)(w0 >> 32)}, rout, off1, 0, STPOL);
                    } else {
                        global_u64 *dst;
                        if constexpr (kIsDesc<Args>)
                            dst = s.dst;
                        else
                            dst = (global_u64 *)(a.images + first * a.img_stride + s.img);
                        if (CHUNK == kTwoCorner && s.mir) {
                            // the mirrored columns c, c+1: P-1-c, P-2-c
                            if (both) {
                                store_pair(dst + (P - 2 - c), w1, w0);
                            } else if (last) {
                                dst[P - 1 - c] = w0;
                            }
                        } else if (both) {
                            store_pair(dst + c, w0, w1);
                        } else if (last) {
                            dst[c] = w0;
                        }
                    }
                }
            }
        };

        // Rings start zeroed; then the bins of tile 0 go in.
        if (lane_used) {
            for (int c = 0; c < a.R; ++c) {
                if (r0 < Q) slot_base[r0 * RS + c] = pix_zero<T>();
                if (r1 < Q) slot_base[r1 * RS + c] = pix_zero<T>();
            }
        }
        // A chunk after the first starts from the exact state left by the
        // chunks before it: the last E pixels of every row.
        if constexpr (CHUNK == kChunkC) {
            if (valid) {
                const uint64_t *st =
                    a.chunk.ws + (blk * per + (chunk - 1)) * (int64_t)(Q * a.chunk.max_cols);
                for (int e = 0; e < E; ++e) {
                    if (r0 < Q)
                        slot_base[r0 * RS + ((shift + dr0 - E + e + rot_of(slot, r0)) & Rmask)] = st[r0 * E + e];
                    if (r1 < Q)
                        slot_base[r1 * RS + ((shift + dr1 - E + e + rot_of(slot, r1)) & Rmask)] = st[r1 * E + e];
                }
            }
        }
        u32x4 buf[NIT * W];
        // aligned loads: the previous tile's lines (16-byte pixels: its
        // first pixel per lane, the only one that can be held)
        u32x4 prev[AL ? NIT : 1];
        // Systematic code: known lines are read up to a.sys_lead tiles
        // behind their staged windows, so those tiles go in first (the
        // swept rows' tiles before 0 lie before column 0 and stage zeros).
        if constexpr (SYS) {
            for (int tt = -a.sys_lead; tt < 0; ++tt) {
                load_tile(tt, buf);
                wave_sync();
                stage_tile(tt, buf, prev);
                wave_sync();
            }
        }
        if constexpr (AL && W == 1) load_tile(-1, prev);
        if constexpr (AL && W == 2) {
            u32x4 first[NIT * W];
            load_tile(-1, first);
            load_tile(0, buf);
#pragma unroll
            for (int it = 0; it < NIT; ++it) prev[it] = first[it * W];
        } else {
            load_tile(0, buf);
        }
        wave_sync();
        stage_tile(0, buf, prev);
        if constexpr (AL) {
#pragma unroll
            for (int it = 0; it < NIT; ++it) prev[it] = buf[it * W];
        }
        load_tile(1, buf);

        // Sweeps tile t and stores the rows' completed windows.
        auto sweep_tile = [&](int t) {
            const int kx = t * TW + X.d, ky = t * TW + Y.d;
            // byte offsets (before masking) of this tile's first column in
            // each ring: the multiple of the pixel size keeps the offset
            // modulo the ring's bytes right for negative columns too
            constexpr uint32_t PB = sizeof(T);
            const uint32_t ownx = (uint32_t)(kx + X.rot) * PB, owny = (uint32_t)(ky + Y.rot) * PB;
            uint32_t ox[QM], oy[QM];
#pragma unroll
            for (int m = 0; m < Q - 1; ++m) {
                ox[m] = (uint32_t)(kx + X.delta[m]) * PB;
                oy[m] = (uint32_t)(ky + Y.delta[m]) * PB;
            }
            // a tile inside the image for every row of the wavefront (most
            // tiles of a long row) zeroes nothing
            const bool in_x = !X.on || (kx >= 0 && kx + TW <= P);
            const bool in_y = !Y.on || (ky >= 0 && ky + TW <= P);
            if (__all(in_x && in_y)) {
#pragma unroll
                for (int i = 0; i < TW; ++i) {
                    sweep_pixel<Q, false>(X, ownx, ox, kx, i, RM, P);
                    wave_sync();
                    sweep_pixel<Q, false>(Y, owny, oy, ky, i, RM, P);
                    wave_sync();
                }
            } else {
#pragma unroll
                for (int i = 0; i < TW; ++i) {
                    sweep_pixel<Q, true>(X, ownx, ox, kx, i, RM, P);
                    wave_sync();
                    sweep_pixel<Q, true>(Y, owny, oy, ky, i, RM, P);
                    wave_sync();
                }
            }
            store_tile(t);
            wave_sync();
        };
        // Stages tile t+1 from `cur`, which then takes the loads of tile
        // t+1+ahead.
        auto advance = [&](int t, u32x4 (&cur)[NIT * W], int ahead) {
            stage_tile(t + 1, cur, prev);
            if constexpr (AL) {
#pragma unroll
                for (int it = 0; it < NIT; ++it) prev[it] = cur[it * W];
            }
            load_tile(t + 1 + ahead, cur);
            wave_sync();
        };
        if constexpr (DEEP) {
            // Two tiles of loads in flight: the two buffers take turns (a
            // copy between them would wait for the younger loads).
            u32x4 buf2[NIT * W];
            load_tile(2, buf2);
            wave_sync();
            for (int t = 0; t < ntiles_wave; t += 2) {
                sweep_tile(t);
                advance(t, buf, 2);
                if (t + 1 >= ntiles_wave) break;
                sweep_tile(t + 1);
                advance(t + 1, buf2, 2);
            }
        } else {
            wave_sync();
            for (int t = 0; t < ntiles_wave; ++t) {
                sweep_tile(t);
                advance(t, buf, 1);
            }
        }
        // A two-corner sweep stops before its rows' last windows are
        // complete: the pixels it computed in them go out now.
        if constexpr (CHUNK == kTwoCorner) store_tile(ntiles_wave, true);
        // The end state of a chunk: the last E pixels of every row.
        if constexpr (CHUNK == kChunkA) {
            if (valid) {
                uint64_t *st = a.chunk.ws + (blk * per + chunk) * (int64_t)(Q * a.chunk.max_cols);
                const int end = shift + a.chunk.tiles * TW;
                for (int e = 0; e < E; ++e) {
                    if (r0 < Q)
                        st[r0 * E + e] = slot_base[r0 * RS + ((end + dr0 - E + e + rot_of(slot, r0)) & Rmask)];
                    if (r1 < Q)
                        st[r1 * E + e] = slot_base[r1 * RS + ((end + dr1 - E + e + rot_of(slot, r1)) & Rmask)];
                }
            }
        }
    }
}

template <int Q>
constexpr int full_slots() { return kWave / ((Q + 1) / 2); }

template <int Q>
constexpr int half_slots() { return kWave / ((Q + 1) / 2) >= 2 ? kWave / ((Q + 1) / 2) / 2 : 1; }

template <int Q, int TW, bool POOL, int CHUNK, int NBT, bool ALIGN = false, bool RCLS = false,
          int W = 1>
__global__ __launch_bounds__(kWave) void decode_kernel(DecodeArgs a) {
    const int64_t per = CHUNK == kWhole ? 1 : CHUNK == kTwoCorner ? 2 : a.chunk.nchunks - 1;
    const int64_t nbatches = (a.nblocks * per + a.nb - 1) / a.nb;
    for (int64_t batch = blockIdx.x; batch < nbatches; batch += gridDim.x)
        decode_batch<Q, TW, POOL, CHUNK, NBT, DecodeArgs, kStreamPolicy, false, ALIGN, RCLS, W>(
            a, batch);
}

// Ring class of block b for the whole-block pool sweeps split by ring
// length: true when its survivor set reads more than a.ring_depth columns
// behind a row's newest pixel (the depth rule of decode_batch), false for
// the others and for undecodable blocks.
template <int Q>
__device__ __forceinline__ bool block_is_deep(const DecodeArgs &a, int64_t b) {
    const uint32_t mask = a.masks ? a.masks[b] : a.mask_uniform;
    int A[Q], pr[Q];
    int cnt = 0, psum = 0;
    for (int s = 0; s < a.n; ++s) {
        const int id = a.id_sorted[s];
        const int p = a.p_sorted[s];
        if (!((mask >> id) & 1u) && cnt < Q) {
#pragma unroll
            for (int r = 0; r < Q; ++r) {
                if (r == cnt) {
                    A[r] = 2 * psum + cnt;
                    pr[r] = p;
                }
            }
            psum += p;
            ++cnt;
        }
    }
    if (cnt < Q) return false;
    int depth = INT_MIN;
#pragma unroll
    for (int r = 0; r < Q; ++r)
#pragma unroll
        for (int l = 0; l < Q; ++l)
            if (l != r) depth = max(depth, ceil_half(A[l] - A[r]) - 1 - (l - r) * pr[r]);
    return depth > a.ring_depth;
}

constexpr int kGatherWords = 8;   // a gathering wavefront scans up to 8 x 64 blocks

// The deep ring class (a.ring_mode 2), gathered: its blocks are few (13 of
// the 495 survivor sets of the (12,8) code) and scattered, so instead of
// sweeping batches of consecutive blocks, mostly empty, each wavefront scans
// a.gather_range consecutive blocks for the class's members (one block per
// lane and pass, ballot) and sweeps them a.nb at a time, every slot in use.
template <int Q, int TW, int NBT>
__global__ __launch_bounds__(kWave) void decode_deep_kernel(DecodeArgs a) {
    constexpr int LPB = (Q + 1) / 2;
    const int lane = threadIdx.x;
    const int slot = lane / LPB;
    const int SR = a.gather_range;
    const int U = SR / kWave;
    const int64_t nranges = (a.nblocks + SR - 1) / SR;
    for (int64_t range = blockIdx.x; range < nranges; range += gridDim.x) {
        const int64_t lo = range * SR, hi = min(a.nblocks, lo + SR);
        uint64_t deep[kGatherWords];
        int total = 0;
#pragma unroll
        for (int u = 0; u < kGatherWords; ++u) {
            const int64_t b = lo + kWave * u + lane;
            const bool d = u < U && b < hi && block_is_deep<Q>(a, b);
            deep[u] = __ballot(d);
            total += __popcll(deep[u]);
        }
        for (int base = 0; base < total; base += a.nb) {
            const int idx = base + slot;
            int64_t blk = hi;   // an empty slot
            if (slot < a.nb && idx < total) {
                int k = idx;
#pragma unroll
                for (int u = 0; u < kGatherWords; ++u) {
                    const int c = __popcll(deep[u]);
                    if (k >= 0 && k < c) {
                        uint64_t m = deep[u];
                        for (int i = 0; i < k; ++i) m &= m - 1;
                        blk = lo + kWave * u + __builtin_ctzll(m);
                    }
                    k -= c;
                }
            }
            decode_batch<Q, TW, true, kWhole, NBT, DecodeArgs, kStreamPolicy, false, false, true>(
                a, 0, blk, lo, hi);
        }
    }
}

// Carry pass of the chunked decode.  For every block, with y_c the end state
// of chunk c swept from a zero start (saved by the first sweep) and T the
// transfer matrix of the block's survivor set, the exact start state of
// chunk c+1 is z_{c+1} = T z_c XOR y_c, z_1 = y_0 (chunk 0 starts from the
// true, all-zero state).  z_{c+1} overwrites y_c in place.
//
// One workgroup per block, up to kCarryWaves wavefronts.  A product T z is
// taken four state words at a time (the "four Russians" method of Arlazarov,
// Dinic, Kronrod and Faradzev): for every group g of words 4g..4g+3 of z the
// 16 XOR combinations are tabulated in LDS, and output word i is the XOR over
// g of the entry that row i's 4-bit slice of T selects, so an output costs
// Q*E/4 independent LDS lookups.  Tables are built over as many groups at a
// time as fit in kCarryTableWords.
constexpr int kCarryWaves = 8;
constexpr int kCarryTableWords = 5888;   // 46 KB of tables (a multiple of 256); z up to 16 KB
constexpr int kCarryOutPerThread = kCarryMaxState / (kWave * kCarryWaves);
constexpr int kCarryAhead = 4;           // chunks whose end states are loaded ahead

// RWC > 0: every thread owns at most one output word and keeps its matrix row
// (RW <= RWC words) in registers for all chunks; RWC == 0: rows are read from
// memory at every chunk.  `Args`: DecodeArgs or DecodeChunkClass.
template <int RWC, class Args>
__device__ __forceinline__ void carry_block(const Args &a, const int Q, const int64_t blk) {
    extern __shared__ uint64_t lds_carry[];
    constexpr int OPT = RWC > 0 ? 1 : kCarryOutPerThread;   // outputs per thread
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int per = a.chunk.nchunks - 1;
    const int64_t stride = (int64_t)Q * a.chunk.max_cols;
    const int64_t zwords = stride + 4;                // z, zero past the state
    uint64_t *z = lds_carry;
    uint64_t *tab = lds_carry + zwords;               // kCarryTableWords words
    const uint32_t mask = a.masks ? a.masks[blk] : a.mask_uniform;
    uint32_t used = 0;
    int cnt = 0;
    for (int s = 0; s < a.n; ++s) {
        const int id = a.id_sorted[s];
        if (!((mask >> id) & 1u) && cnt < Q) {
            used |= 1u << id;
            ++cnt;
        }
    }
    if (cnt < Q) return;   // undecodable: reported by the sweep (uniform per block)
    const int set = a.chunk.lut[used];
    const int d = Q * a.chunk.state_cols[set];
    const int RW = (d + 63) / 64;
    const int G = (d + 3) / 4;                        // 4-word groups
    const int GP = kCarryTableWords / 16;             // groups per table pass
    const uint64_t *T = a.chunk.tmat + a.chunk.tmat_off[set];
    uint64_t *ws = a.chunk.ws + blk * per * stride;
    uint64_t trow[RWC > 0 ? RWC : 1];
    if constexpr (RWC > 0) {
#pragma unroll
        for (int w = 0; w < RWC; ++w) trow[w] = (tid < d && w < RW) ? T[(int64_t)tid * RW + w] : 0;
    }
    __syncthreads();   // the previous block's last reads of z are done
    for (int i = tid; i < zwords; i += nthreads) z[i] = i < d ? ws[i] : 0;
    // y_c of the next kCarryAhead chunks, loaded ahead of their step
    uint64_t yq[kCarryAhead][OPT];
#pragma unroll
    for (int k = 0; k < kCarryAhead; ++k)
#pragma unroll
        for (int u = 0; u < OPT; ++u) {
            const int i = tid + nthreads * u;
            yq[k][u] = (i < d && 1 + k < per) ? ws[(1 + k) * stride + i] : 0;
        }
    __syncthreads();
    for (int c = 1; c < per; ++c) {
        uint64_t *y = ws + c * stride;
        uint64_t acc[OPT];
#pragma unroll
        for (int u = 0; u < OPT; ++u) {
            const int i = tid + nthreads * u;
            acc[u] = yq[0][u];
#pragma unroll
            for (int k = 0; k + 1 < kCarryAhead; ++k) yq[k][u] = yq[k + 1][u];
            yq[kCarryAhead - 1][u] =
                (i < d && c + kCarryAhead < per) ? ws[(c + kCarryAhead) * stride + i] : 0;
        }
        for (int g0 = 0; g0 < G; g0 += GP) {
            const int g1 = min(G, g0 + GP);
            for (int e = tid; e < (g1 - g0) * 16; e += nthreads) {
                const int g = g0 + (e >> 4), m = e & 15;
                uint64_t v = 0;
#pragma unroll
                for (int k = 0; k < 4; ++k)
                    if ((m >> k) & 1) v ^= z[4 * g + k];
                tab[e] = v;
            }
            __syncthreads();
            if constexpr (RWC > 0) {
                // one pass covers every group (RWC * 16 <= GP)
                if (tid < d) {
#pragma unroll
                    for (int w = 0; w < RWC; ++w) {
                        if (w >= RW) break;
                        const uint64_t bits = trow[w];
                        const int gn = min(16, G - 16 * w);
                        for (int q = 0; q < gn; ++q)
                            acc[0] ^= tab[((16 * w + q) << 4) | (int)((bits >> (4 * q)) & 15)];
                    }
                }
            } else {
#pragma unroll
                for (int u = 0; u < OPT; ++u) {
                    const int i = tid + nthreads * u;
                    if (i >= d) continue;
                    const uint64_t *row = T + (int64_t)i * RW;
                    for (int g = g0; g < g1; g += 16) {    // one matrix word: 16 groups
                        const uint64_t bits = row[g >> 4];
                        const int gn = min(16, g1 - g);
                        for (int q = 0; q < gn; ++q)
                            acc[u] ^= tab[((g - g0 + q) << 4) | (int)((bits >> (4 * q)) & 15)];
                    }
                }
            }
            __syncthreads();   // tables are rebuilt or z is overwritten next
        }
#pragma unroll
        for (int u = 0; u < OPT; ++u) {
            const int i = tid + nthreads * u;
            if (i < d) {
                z[i] = acc[u];
                y[i] = acc[u];
            }
        }
        __syncthreads();
    }
}

// One item of a parallel-carry step: entry c of block blk.  dst[c] =
// src[c] XOR M src[c - h] with M = T^h, h = 2^step (table-lookup product as in
// carry_block), or dst[c] = src[c] when c < h.  State at most kScanMaxState
// words, so every thread owns at most one output word.
template <class Args>
__device__ __forceinline__ void scan_item(const Args &a, const int Q, const int64_t blk,
                                          const int c, const int step, const uint64_t *src,
                                          uint64_t *dst) {
    extern __shared__ uint64_t lds_carry[];
    const int tid = threadIdx.x;
    const int nthreads = blockDim.x;
    const int per = a.chunk.nchunks - 1;
    const int64_t stride = (int64_t)Q * a.chunk.max_cols;
    const int64_t zwords = stride + 4;
    uint64_t *z = lds_carry;
    uint64_t *tab = lds_carry + zwords;
    const uint32_t mask = a.masks ? a.masks[blk] : a.mask_uniform;
    uint32_t used = 0;
    int cnt = 0;
    for (int s = 0; s < a.n; ++s) {
        const int id = a.id_sorted[s];
        if (!((mask >> id) & 1u) && cnt < Q) {
            used |= 1u << id;
            ++cnt;
        }
    }
    if (cnt < Q) return;   // undecodable: reported by the sweep (uniform per block)
    const int set = a.chunk.lut[used];
    const int d = Q * a.chunk.state_cols[set];
    const int RW = (d + 63) / 64;
    const int G = (d + 3) / 4;
    const int h = 1 << step;
    const uint64_t *in = src + (blk * per + c) * stride;
    uint64_t *out = dst + (blk * per + c) * stride;
    if (c < h) {
        for (int i = tid; i < d; i += nthreads) out[i] = in[i];
        return;
    }
    const uint64_t *M = a.chunk.tmat + a.chunk.tmat_off[set] + (int64_t)step * d * RW;
    const uint64_t *zin = in - (int64_t)h * stride;
    __syncthreads();   // the previous item's reads of z and tab are done
    for (int i = tid; i < zwords; i += nthreads) z[i] = i < d ? zin[i] : 0;
    __syncthreads();
    for (int e = tid; e < G * 16; e += nthreads) {
        const int g = e >> 4, m = e & 15;
        uint64_t v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if ((m >> k) & 1) v ^= z[4 * g + k];
        tab[e] = v;
    }
    __syncthreads();
    if (tid < d) {
        uint64_t acc = in[tid];
        const uint64_t *row = M + (int64_t)tid * RW;
        for (int w = 0; w < RW; ++w) {
            const uint64_t bits = row[w];
            const int gn = min(16, G - 16 * w);
            for (int q = 0; q < gn; ++q)
                acc ^= tab[((16 * w + q) << 4) | (int)((bits >> (4 * q)) & 15)];
        }
        out[tid] = acc;
    }
}

template <int RWC>
__global__ __launch_bounds__(kWave * kCarryWaves) void decode_carry_kernel(DecodeArgs a, int Q) {
    for (int64_t blk = blockIdx.x; blk < a.nblocks; blk += gridDim.x) carry_block<RWC>(a, Q, blk);
}

template <int RWC>
__global__ __launch_bounds__(kWave * kCarryWaves) void decode_carry_classes_kernel(
    DecodeChunkTable tab) {
    const int64_t total = tab.first_block[tab.nclasses];
    for (int64_t item = blockIdx.x; item < total; item += gridDim.x) {
        int c = 0;
        while (item >= tab.first_block[c + 1]) ++c;
        carry_block<RWC>(tab.cls[c], tab.cls[c].Q, item - tab.first_block[c]);
    }
}

// Single-geometry launchers (static: one copy per translation unit that uses them).
template <int Q, int NBT>
static hipError_t launch_qn(int mode, const DecodeArgs &a, int grid, hipStream_t s) {
    const size_t lds = decode_lds_bytes(Q, a.nb, a.ring_stride);
    // Pool sweeps of the half-slot body load whole lines (ALIGN) for 4 rows
    // when the host asks (a.align: the shortest rings); measured with other
    // row counts the extra registers cost more than the fetches saved (8 KB
    // (8,4): 5.49 against 5.06 ms; 4 KB (3,3): 3.19 against 3.02 ms), and so
    // they did with 64-word rings (the 128-bit pixel geometry: 1,565 against
    // 1,823 GB/s).
    constexpr bool kAlign = NBT < full_slots<Q>() && Q == 4;
    switch (mode) {
        case kLaunchPool:
#define MJ_POOL_LAUNCH(AL, RC)                                                                \
    hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, true, kWhole, NBT, AL, RC>), dim3(grid), \
                       dim3(kWave), lds, s, a)
            // the held words' registers leave room for 2 wavefronts per SIMD:
            // worth it only while the wavefront's slots are mostly in use
            if (a.ring_mode == 2 && a.gather_range > 0) {
                hipLaunchKernelGGL((decode_deep_kernel<Q, kDecodeTile, NBT>), dim3(grid),
                                   dim3(kWave), lds, s, a);
            } else if (a.ring_mode != 0) {
                if (kAlign && a.align && 2 * a.nb > NBT) MJ_POOL_LAUNCH(kAlign, true);
                else MJ_POOL_LAUNCH(false, true);
            } else {
                if (kAlign && a.align && 2 * a.nb > NBT) MJ_POOL_LAUNCH(kAlign, false);
                else MJ_POOL_LAUNCH(false, false);
            }
#undef MJ_POOL_LAUNCH
            break;
        case kLaunchPointers:
            hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, false, kWhole, NBT>), dim3(grid),
                               dim3(kWave), lds, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Chunked sweeps: chunks are plentiful, so they always run the half-slot body.
template <int Q>
static hipError_t launch_chunk(int mode, const DecodeArgs &a, int grid, hipStream_t s) {
    constexpr int full = full_slots<Q>();
    constexpr int NBT = full >= 2 ? full / 2 : 1;
    if (a.nb > NBT) return hipErrorInvalidValue;
    const size_t lds = decode_lds_bytes(Q, a.nb, a.ring_stride);
    switch (mode) {
        case kLaunchChunkA:
            hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, true, kChunkA, NBT>), dim3(grid),
                               dim3(kWave), lds, s, a);
            break;
        case kLaunchChunkC:
            hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, true, kChunkC, NBT>), dim3(grid),
                               dim3(kWave), lds, s, a);
            break;
        case kLaunchChunkAGather:
            hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, false, kChunkA, NBT>), dim3(grid),
                               dim3(kWave), lds, s, a);
            break;
        case kLaunchChunkCGather:
            hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, false, kChunkC, NBT>), dim3(grid),
                               dim3(kWave), lds, s, a);
            break;
        case kLaunchTwoCorner:
            hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, true, kTwoCorner, NBT>), dim3(grid),
                               dim3(kWave), lds, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// 16-byte pixels (whole blocks from a pool): the body compiled for half the
// slots (the full one would need twice the row-window registers), with
// whole-line loads when a.align is set.
template <int Q>
static hipError_t launch_wide_q(const DecodeArgs &a, int grid, hipStream_t s) {
    constexpr int NBT = half_slots<Q>();
    if (a.nb > NBT) return hipErrorInvalidValue;
    const size_t lds = 2 * decode_lds_bytes(Q, a.nb, a.ring_stride);
    if (a.align)
        hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, true, kWhole, NBT, true, false, 2>),
                           dim3(grid), dim3(kWave), lds, s, a);
    else
        hipLaunchKernelGGL((decode_kernel<Q, kDecodeTile, true, kWhole, NBT, false, false, 2>),
                           dim3(grid), dim3(kWave), lds, s, a);
    return hipGetLastError();
}

// The body compiled for half the slots serves launches whose LDS allows no
// more (one block alone in pointer mode included).
template <int Q>
static hipError_t launch_q(int mode, const DecodeArgs &a, int grid, hipStream_t s) {
    constexpr int full = full_slots<Q>();
    if (mode >= kLaunchChunkA) return launch_chunk<Q>(mode, a, grid, s);
    if (full >= 2 && a.nb <= full / 2) return launch_qn<Q, (full >= 2 ? full / 2 : 1)>(mode, a, grid, s);
    return launch_qn<Q, full>(mode, a, grid, s);
}

}  // namespace mj
