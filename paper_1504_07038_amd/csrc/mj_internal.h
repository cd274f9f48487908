// Internal declarations shared by the host API and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/mojette.h"

namespace mj {

constexpr int kMaxDirs = MOJETTE_MAX_DIRS;
constexpr int kMaxRows = MOJETTE_MAX_ROWS;
constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kDecodeTile = 16;    // columns per row per decode tile
// Decode rings (decode_body.h) of codes of 5 to 8 rows are aligned to their
// length R (a power of two): a slot's LDS address is then one add and one
// and-or from the tile's offset, and rotations spread the rows over the
// banks.  Other row counts keep rings R + 1 words apart (odd strides spread
// them): with 4 rows the one more register per row window costs the
// whole-line body its second wavefront per SIMD, and the descriptor body of
// 12 rows likewise (measured 4 KB (6,4) decode 1.7x, 1 MB (12,4) descriptor
// decode 1.5x slower aligned; 8 KB (12,8) unchanged, 1 MB (8,4) 10% faster).
__host__ __device__ constexpr bool ring_aligned(int Q) { return Q >= 5 && Q <= 8; }
// LDS words between the rings of two rows of a block slot.
__host__ __device__ constexpr int ring_stride_of(int Q, int R) { return ring_aligned(Q) ? R : R + 1; }
constexpr int kEncodeWaves = 4;    // most waves per encode workgroup

// Orders LDS traffic between the lanes of one wavefront.  The LDS
// instructions of a wave execute in issue order, so a compiler-level fence at
// wavefront scope is enough: no wait for the LDS queue to drain.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Device memory addressed through a pointer read from a table in memory:
// held in the global address space, so that the accesses through it are
// global instructions rather than flat ones (flat ones also count against
// the LDS wait counter, so every wait for an LDS read would wait for them).
typedef __attribute__((address_space(1))) uint64_t global_u64;
typedef __attribute__((address_space(1))) const mojette_block global_block;
typedef __attribute__((address_space(1))) const int32_t global_i32;

// Smallest line position b = -k + l*p over a P x Q image (q = 1).
__host__ __device__ inline int32_t bin_offset(int32_t p, int32_t P, int32_t Q) {
    int32_t m = (Q - 1) * p;
    return -(P - 1) + (m < 0 ? m : 0);
}

// Eq. 2 with q = 1.
__host__ __device__ inline int32_t proj_bins(int32_t p, int32_t P, int32_t Q) {
    return (p < 0 ? -p : p) * (Q - 1) + P;
}

// ---- encode --------------------------------------------------------------
// One work item is (block, column tile).  A tile covers image columns
// [x0, x0 + W) and produces every bin whose row-0 crossing -b lies in that
// range (the first and last tiles also take the edge bins outside [0, P)).
// The wave stages columns [x0 - H, x0 + W + H) of all Q rows into LDS with
// zeros outside the image, H = (Q-1) * max|p|, so no bin read is bounds
// checked.
struct EncodeArgs {
    const uint64_t *images;          // block b's image at images + b*P*Q
    uint64_t *out[kMaxDirs];         // projection i of block b: out[i] + b*proj_stride
    const int64_t *slots;            // if set, block b's projections at slice slots[b] instead
    int64_t proj_stride;
    int64_t nblocks;
    int32_t P, Q, n;
    int32_t W, H, S, ntiles;         // tile width, halo, LDS row stride, tiles per block
    int32_t waves;                   // waves per workgroup (1, 2 or 4), one LDS tile each
    int32_t bin_swap;                // 1: bin j is stored at word j ^ 1 (128-bit pixels), else 0
    int32_t p[kMaxDirs];
    // Projection i stores keep_n[i] bins from bin index keep_lo[i] on (the
    // never-used bins left out); keep_n[i] == 0: all of Eq. 2's bins.
    int32_t keep_lo[kMaxDirs], keep_n[kMaxDirs];
    __device__ int dir(int i) const { return p[i]; }
    // block blk's slice index, then projection i within slice `slice`
    __device__ int64_t slice(int64_t blk) const { return slots ? slots[blk] : blk; }
    __device__ uint64_t *proj_in(int i, int64_t slice) const {
        return out[i] + slice * proj_stride;
    }
    __device__ int kept_first(int i) const { return keep_lo[i]; }
    __device__ int kept_count(int i, int full) const { return keep_n[i] ? keep_n[i] : full; }
    __device__ const uint64_t *image_of(int64_t blk) const { return images + blk * (int64_t)P * Q; }
};

// Consistency check: every surviving projection recomputed from the image and
// compared with the stored one (par[i] + b*proj_stride).
struct VerifyArgs : EncodeArgs {
    const uint64_t *par[kMaxDirs];
    const uint16_t *masks;           // bit i: projection i lost (not checked); may be null
    uint32_t mask_uniform;           // the mask of every block when masks is null
    int32_t *status;
};

// One geometry class of a mixed launch: nblocks blocks with the same P, Q and
// directions, images back to back at `images`, projection slices back to back
// at `projs`.
struct EncodeClass {
    const uint64_t *images;
    uint64_t *projs;
    const int64_t *slots;            // block b's slice is slice slots[b] of projs (null: b)
    int64_t nblocks;
    int32_t proj_stride;             // words per block slice
    int32_t P, Q, n, W, H, S, ntiles;
    int32_t bin_swap;                // always 0: mixed launches take 64-bit pixels
    int32_t off[kMaxDirs];           // projection i at off[i] within a slice
    int16_t p[kMaxDirs];
    __device__ int dir(int i) const { return p[i]; }
    __device__ int64_t slice(int64_t blk) const { return slots ? slots[blk] : blk; }
    __device__ uint64_t *proj_in(int i, int64_t slice) const {
        return projs + slice * proj_stride + off[i];
    }
    __device__ int kept_first(int) const { return 0; }      // mixed launches keep every bin
    __device__ int kept_count(int, int full) const { return full; }
    __device__ const uint64_t *image_of(int64_t blk) const { return images + blk * (int64_t)P * Q; }
};

constexpr int kMaxClasses = MOJETTE_MAX_CLASSES;

struct EncodeClassTable {
    EncodeClass cls[kMaxClasses];
    int64_t first_item[kMaxClasses + 1];   // items of class c: [first_item[c], first_item[c+1])
    int32_t nclasses;
};

// ---- decode --------------------------------------------------------------
// Rows of a block are swept left to right in the order fixed by the sorted
// directions (see decode_body.h).  Each lane owns two rows of one block; a wave
// holds up to 64/ceil(Q/2) blocks.  Each row keeps its last R pixels in an
// LDS ring.
// Chunked decode of long rows.  The tiles of a block are cut into nchunks
// chunks of `tiles` tiles (the last one takes the rest).  Chunks 0..nchunks-2
// are first swept from zeroed rings, each saving its end state (the last E
// pixels of every row, E fixed by the survivor set); a carry pass turns those
// into the exact start states of chunks 1..nchunks-1 with the GF(2) transfer
// matrix of the survivor set; the chunks are then swept again from their
// exact states.  The decode is linear over GF(2) (XOR), so a chunk's end
// state is its end state from a zero start XOR the transfer matrix applied
// to its true start state.
constexpr int kWhole = 0;     // sweep whole blocks
constexpr int kChunkA = 1;    // sweep chunks from zero states, save end states
constexpr int kChunkC = 2;    // sweep chunks from exact start states
constexpr int kTwoCorner = 3; // sweep each block from both ends, each sweep half-way

constexpr int kCarryMaxState = 2048;   // most state words (Q * E) the carry pass handles

struct ChunkInfo {
    uint64_t *ws;                    // per (block, chunk boundary): Q * max_cols words
    uint64_t *ws_alt;                // second buffer of the same layout (parallel carry)
    const int32_t *lut;              // survivor id mask -> set index (-1: none)
    const int32_t *state_cols;       // per set: E
    const int64_t *tmat_off;         // per set: word offset of its matrices in tmat
    const uint64_t *tmat;            // per set: T, T^2, T^4, ... (npow matrices), each
                                     // Q*E rows of ceil(Q*E/64) words
    int32_t tiles;                   // tiles per chunk
    int32_t nchunks;                 // chunks per block (>= 2 in chunked launches)
    int32_t max_cols;                // largest E over the sets
    int32_t npow;                    // matrices per set
};

// The carry as a parallel prefix (Kogge-Stone) over the chunks of a block,
// for survivor sets of at most kScanMaxState state words: after step s,
// entry c holds sum_{c - 2^(s+1) < j <= c} T^(c-j) y_j; ceil(log2(C-1))
// steps leave z_{c+1} in entry c.  Plans keep kScanPowers powers T^(2^s).
constexpr int kScanMaxState = 512;
constexpr int kScanPowers = 10;

// Launch modes of launch_decode.
constexpr int kLaunchPool = 0;       // whole blocks from a projection pool
constexpr int kLaunchPointers = 1;   // one whole block from projection pointers
constexpr int kLaunchChunkA = 2;     // pool, first chunk sweep
constexpr int kLaunchChunkC = 3;     // pool, final chunk sweep
constexpr int kLaunchChunkAGather = 4;   // projection slices at slots, first chunk sweep
constexpr int kLaunchChunkCGather = 5;   // projection slices at slots, final chunk sweep
constexpr int kLaunchTwoCorner = 8;      // whole blocks from a pool, swept from both ends

struct DecodeArgs {
    // Pool mode (batches): block b's n projections start at word
    // b*proj_stride of `pool`, projection i at word off[i] of that slice.
    const uint64_t *pool;
    int32_t off[kMaxDirs];
    // Pointer mode: projection i of the one block at in[i] (null if not
    // given) when `pool` is null; else block b's slice is slice slots[b] of
    // `pool` (gathering launches).
    const uint64_t *in[kMaxDirs];
    const int64_t *slots;
    int64_t proj_stride;
    uint64_t *images;
    int64_t img_stride;
    const uint16_t *masks;           // per-block erasure masks, or null
    uint32_t mask_uniform;           // mask used when masks is null
    int32_t *status;                 // may be null
    int64_t nblocks;
    int32_t P, n;
    int32_t R, ring_stride;          // ring length (power of two), words per LDS ring row
    int32_t nb;                      // blocks per wavefront (at most 64/ceil(Q/2), fewer if LDS is short)
    int32_t p_sorted[kMaxDirs];      // directions in ascending p
    int32_t id_sorted[kMaxDirs];     // their indices in the caller's dirs
    ChunkInfo chunk;                 // chunked launches only
    int32_t keep_lo[kMaxDirs];       // projection i's first stored bin index (0: Eq. 2's first)
    int32_t sys_lead;                // systematic decode: tiles staged ahead of the sweep
    int32_t ring_mode;               // whole-block pool sweeps: 0 every block; 1 only blocks
                                     // whose survivor set's depth is <= ring_depth; 2 the others
    int32_t ring_depth;
    int32_t align;                   // whole-block pool sweeps: whole-line loads where compiled
    int32_t gather_range;            // ring_mode 2: blocks scanned per wavefront for members of
                                     // the class (a multiple of 64), 0: every block in batches
    int32_t bin_swap;                // pointer mode: 1 reads word bin j at word j ^ 1 (128-bit pixels)
    __device__ const uint64_t *proj_base(int64_t blk, int id) const {
        return pool ? pool + slots[blk] * proj_stride + off[id] : in[id];
    }
    __device__ int kept_first(int id) const { return keep_lo[id]; }
};

// One geometry class of a mixed decode launch (pool mode only).  Field names
// match DecodeArgs so that the same per-batch body serves both.
struct DecodeClass {
    const uint64_t *pool;            // projection slices of the class
    const int64_t *slots;            // block b's slice is slice slots[b] of pool (null: b)
    uint64_t *images;                // images of the class, back to back
    const uint16_t *masks;           // erasure masks of the class, one per block
    int32_t *status;
    int64_t nblocks;
    int64_t proj_stride;
    int64_t img_stride;
    int32_t P, Q, n, nb, R, ring_stride;
    uint32_t mask_uniform;
    int32_t off[kMaxDirs];
    int16_t p_sorted[kMaxDirs];
    int8_t id_sorted[kMaxDirs];
    __device__ const uint64_t *proj_base(int64_t blk, int id) const {
        return pool + (slots ? slots[blk] : blk) * proj_stride + off[id];
    }
    __device__ int kept_first(int) const { return 0; }      // mixed launches keep every bin
};

struct DecodeClassTable {
    DecodeClass cls[kMaxClasses];
    int64_t first_item[kMaxClasses + 1];   // batches of class c: [first_item[c], first_item[c+1])
    int32_t nclasses;
};

// ---- descriptor-driven batched calls ----------------------------------------
// Blocks are described by device descriptors (mojette_block): each names its
// code (geom_id into the plan's geometry table), its row length P, where its
// image and projections sit in one word pool, and its erasure mask.  A call
// first sorts the blocks into classes of equal (code, P, decode ring class)
// on the device (bucket kernels, in the caller's workspace), then one
// persistent launch walks the classes' work items, heaviest first.

// One code of a plan, as the device kernels read it.
struct GeomDev {
    int32_t Q, n;
    int32_t sumabs;                  // sum of |p_i|: projection offsets are P-dependent
    int32_t H;                       // encode halo, (Q-1) * max |p|
    // encode row windows (codes of 9 to 12 rows): row l of a tile at column
    // x0 stages columns [x0 + l*plo, x0 + W + l*(plo + pspan)),
    // plo = min(min p, 0), pspan = max(max p, 0) - plo
    int32_t plo, pspan;
    int32_t enc_w;                   // encode tile width cap (columns)
    int32_t R, nb;                   // decode ring and blocks per wavefront, full ring
    int32_t R_short, nb_short;       // short-ring class (0: none)
    int32_t depth_short;             // survivor sets of depth <= this take the short ring
    int32_t two_min_P;               // rows at least this long decode from both ends (0: never)
    int32_t R_two, nb_two;           // their ring (both direction orders) and blocks per wave
    // 128-bit pixels (MOJETTE_GEOM_WIDE) run as the word image of 2P columns
    // with the directions doubled (dirs, p_sorted below hold 2p), and word
    // bin j stored at word j ^ 1: pshift = 1, else 0
    int32_t pshift;
    // never-used bins left out (MOJETTE_GEOM_TRIMMED): projection i keeps
    // P + keep_rows[i] * |p_i| bins from index keep_lo[i] on; keep_rows[i]
    // < 0: all of Eq. 2's bins
    int32_t keep_lo[kMaxDirs], keep_rows[kMaxDirs];
    int32_t dirs[kMaxDirs];          // in the caller's order
    int16_t p_sorted[kMaxDirs];      // ascending
    int8_t id_sorted[kMaxDirs];
};

constexpr int kDescSlots = 4096;     // hash slots = most classes per call
constexpr int kDescMaxP = 1 << 24;

// One class of a descriptor-driven decode: field names follow DecodeClass so
// that the same per-batch body serves it (pointer mode: a block's bins and
// image are found through its descriptor).
struct DecodeDesc {
    global_block *desc;
    global_i32 *idx;                 // the class's blocks: descriptor indices
    global_u64 *pool;
    int32_t *status;
    uint64_t *images;                // unused (images are found per block)
    const uint16_t *masks;           // unused (masks come with the descriptors)
    const int64_t *slots;            // unused
    int64_t nblocks;
    int64_t proj_stride, img_stride;
    int32_t P, Q, n, nb, R, ring_stride;
    uint32_t mask_uniform;
    int32_t off[kMaxDirs];
    int32_t p_sorted[kMaxDirs];      // 32-bit: read with scalar loads
    int32_t id_sorted[kMaxDirs];
    int32_t bin_swap;                // 1: bin j of a projection is stored at word j ^ 1
    int32_t keep_lo[kMaxDirs];       // index of projection i's first stored bin
    static constexpr bool kDesc = true;
    __device__ const mojette_block &block(int64_t blk) const {
        return *(const mojette_block *)(desc + idx[blk]);
    }
    __device__ const uint64_t *proj_base(int64_t blk, int id) const {
        return (const uint64_t *)(pool + block(blk).proj_off + off[id]);
    }
    __device__ uint64_t *image_of(int64_t blk) const {
        return (uint64_t *)(pool + block(blk).image_off);
    }
    __device__ uint32_t mask_of(int64_t blk) const { return block(blk).erasure_mask; }
    __device__ int kept_first(int i) const { return keep_lo[i]; }
};

// One class of a descriptor-driven encode (fields as EncodeClass).
struct EncodeDesc {
    global_block *desc;
    global_i32 *idx;
    global_u64 *pool;
    int64_t nblocks;
    int32_t P, Q, n, W, H, S, ntiles;
    int32_t plo, pspan;              // row windows (see GeomDev)
    int32_t bin_swap;                // 1: word bin j stored at word j ^ 1 (128-bit pixels)
    int32_t off[kMaxDirs];
    int32_t p[kMaxDirs];             // 32-bit: read with scalar loads
    int32_t keep_lo[kMaxDirs], keep_n[kMaxDirs];   // stored bins (keep_n 0: all)
    __device__ int dir(int i) const { return p[i]; }
    __device__ const mojette_block &block(int64_t blk) const {
        return *(const mojette_block *)(desc + idx[blk]);
    }
    __device__ int64_t slice(int64_t blk) const { return (int64_t)block(blk).proj_off; }
    __device__ uint64_t *proj_in(int i, int64_t slice) const {
        return (uint64_t *)(pool + slice + off[i]);
    }
    __device__ int kept_first(int i) const { return keep_lo[i]; }
    __device__ int kept_count(int i, int full) const { return keep_n[i] ? keep_n[i] : full; }
    __device__ const uint64_t *image_of(int64_t blk) const {
        return (const uint64_t *)(pool + block(blk).image_off);
    }
};

// Workspace of a descriptor-driven call (byte offsets from its start; the
// layout depends on nblocks only).
struct DescWorkspace {
    static constexpr size_t kHeader = 0;           // DescHeader
    static constexpr size_t kKeys = 1024;          // kDescSlots uint64 keys (0: empty)
    static constexpr size_t kCounts = kKeys + 8 * kDescSlots;      // uint32 per slot
    static constexpr size_t kSlotClass = kCounts + 4 * kDescSlots; // int32 per slot
    static constexpr size_t kSegStart = kSlotClass + 4 * kDescSlots;  // int64 per class + 1
    static constexpr size_t kFirstItem = kSegStart + 8 * (kDescSlots + 8); // int64 per class + 1
    static constexpr size_t kOrder = kFirstItem + 8 * (kDescSlots + 8);    // uint64 sort keys
    static constexpr size_t kClasses = kOrder + 8 * kDescSlots;
    static constexpr size_t kClassBytes =
        sizeof(DecodeDesc) > sizeof(EncodeDesc) ? sizeof(DecodeDesc) : sizeof(EncodeDesc);
    static constexpr size_t kSlotOf = (kClasses + kClassBytes * kDescSlots + 255) / 256 * 256;
    // per block: (slot, rank) as int2, then the index list (int32)
    __host__ __device__ static size_t idx_at(int64_t nblocks) { return kSlotOf + (size_t)(8 * nblocks + 255) / 256 * 256; }
    __host__ __device__ static size_t bytes(int64_t nblocks) { return idx_at(nblocks) + (size_t)(4 * nblocks + 255) / 256 * 256; }
};

// Launch groups: row count Q, plus kTwoGroup for the classes decoded from
// both ends.
constexpr int kTwoGroup = kMaxRows + 1;
constexpr int kDescGroups = 2 * kTwoGroup;

struct DescHeader {   // at most DescWorkspace::kKeys bytes
    int32_t nclasses;
    int32_t error;                   // a status stored by the bucket kernels (table full)
    int64_t range[2 * kDescGroups];  // items of launch group g: [range[2g], range[2g+1])
};

// What the bucket kernels need of a call.
struct DescCall {
    const mojette_block *desc;
    int64_t nblocks;
    const GeomDev *geoms;
    int32_t ngeoms;
    uint8_t *ws;
    uint64_t *pool;
    int32_t *status;
    int32_t decode;                  // 1: decode classes (ring classes, survivor check)
    int32_t group_by_q;              // 1: one launch group per row count, else one group
};

hipError_t launch_desc_buckets(const DescCall &c, hipStream_t s);
// One launch of a descriptor-driven decode or encode over launch group g
// (the classes of row count Q = g).
hipError_t launch_decode_desc(int Q, bool two, const DescCall &c, int g, size_t lds, int grid,
                              hipStream_t s);
// Descriptor encode of codes of 9 to 12 rows with register prefetch: each
// row's LDS window holds only the columns its bins cross (see GeomDev.plo),
// row l at word row_window_off(l, W, pspan) of the tile.
constexpr bool encode_row_windows(int Q) { return Q >= 9 && Q <= 12; }
__host__ __device__ constexpr int row_window_off(int l, int W, int pspan) {
    return l * W + pspan * (l * (l - 1) / 2);
}
// Register prefetch chunks of a descriptor encode of Q rows whose widest
// staged row has max_s columns (0: no prefetch).
int encode_desc_prefetch(int Q, int max_s);
// max_row: the widest staged row of the launch's tiles (words).
hipError_t launch_encode_desc(int Q, const DescCall &c, int g, int waves, int tile_words,
                              int max_row, int grid, hipStream_t s);

// Status of a HIP call as a library status code; a failure is remembered for
// mojette_last_hip_error() on the calling thread.
int hip_status(hipError_t e);

// One class of a merged chunked decode launch: a DecodeClass with its chunk
// layout (plan tables, workspace, chunk length and count).
struct DecodeChunkClass : DecodeClass {
    ChunkInfo chunk;
};

constexpr int kMaxChunkClasses = 8;   // keeps the table within the kernel-argument limit

struct DecodeChunkTable {
    DecodeChunkClass cls[kMaxChunkClasses];
    int64_t first_item[kMaxChunkClasses + 1];    // sweeps: batches of class c
    int64_t first_block[kMaxChunkClasses + 1];   // carry: blocks of class c
    int64_t first_pair[kMaxChunkClasses + 1];    // parallel carry: (block, chunk) of class c
    int32_t nclasses;
};

bool decode_chunk_classes_supported(unsigned qmask, bool gather);
// mode: kLaunchChunkA or kLaunchChunkC (sweeps, one wave per workgroup), or
// kLaunchCarry (carry pass, `threads` per workgroup).
constexpr int kLaunchCarry = 6;
// kLaunchScan + s: step s of the parallel carry (ws -> ws_alt for even s,
// ws_alt -> ws for odd s).
constexpr int kLaunchScan = 16;
hipError_t launch_decode_chunk_classes(int mode, unsigned qmask, bool gather,
                                       const DecodeChunkTable &tab, size_t lds, int grid,
                                       int threads, bool rows_in_registers, hipStream_t s);
int carry_waves(int state);
size_t carry_lds_bytes(int state);
bool carry_rows_in_registers(int state);

hipError_t launch_encode(const EncodeArgs &a, int grid, hipStream_t s);
hipError_t launch_verify(const VerifyArgs &a, int grid, hipStream_t s);
hipError_t launch_decode_sys(int Q, const DecodeArgs &a, int grid, hipStream_t s);
hipError_t launch_encode_classes(int qmax, const EncodeClassTable &tab, size_t lds, int grid,
                                 hipStream_t s);
hipError_t launch_decode_classes(unsigned qmask, bool gather, const DecodeClassTable &tab,
                                 size_t lds, int grid, hipStream_t s);
bool decode_classes_supported(unsigned qmask, bool gather);
hipError_t launch_decode(int Q, int mode, const DecodeArgs &a, int grid, hipStream_t s);
// Whole blocks of 16-byte pixels from a pool (P, p, offsets and strides in
// pixels; a.nb at most half the full slot count).
hipError_t launch_decode_wide(int Q, const DecodeArgs &a, int grid, hipStream_t s);
// State width E and transfer matrix (Q*E rows of ceil(Q*E/64) words) of an
// interior chunk of `tiles` tiles for the survivor directions ps[0..Q) in
// ascending order.  False if chunks that short cannot be interior.
bool chunk_transfer(const int32_t *ps, int Q, int tiles, int &E, std::vector<uint64_t> &T);
// The state width E alone (no matrix); false as for chunk_transfer.
bool chunk_state_cols(const int32_t *ps, int Q, int tiles, int &E);
// T^(2^s), s = 0..npow-1, of a dim x dim transfer matrix, back to back.
void chunk_powers(const std::vector<uint64_t> &T, int dim, int npow, std::vector<uint64_t> &out);
// One step of the parallel carry: entry c of dst = entry c of src XOR
// T^(2^step) (entry c - 2^step of src), or a copy of entry c when c < 2^step.
hipError_t launch_decode_scan(const DecodeArgs &a, int Q, int step, const uint64_t *src,
                              uint64_t *dst, hipStream_t s);
hipError_t launch_decode_carry(const DecodeArgs &a, int Q, int grid, hipStream_t s);
size_t decode_lds_bytes(int Q, int nb, int ring_stride);
int decode_max_blocks_per_wave(int Q);
int decode_tile(int Q);
size_t encode_lds_bytes(int Q, int S, int waves);

}  // namespace mj
