// Descriptor-driven batched calls on gfx950: the bucket kernels that group
// the described blocks into classes of equal (code, row length, decode ring
// class) in the caller's workspace, and the decode launch over those
// classes.  The encode launch over the same classes is in encode.hip.
//
// Bucketing is four short launches:
//   clear    zeroes the hash table of class keys and the header;
//   count    one thread per descriptor checks it, finds its class key (the
//            decode also checks that Q projections survive and sorts the
//            survivor set into the short- or full-ring class of its code),
//            inserts the key into an open-addressing hash table, and takes
//            its rank within the class (one atomic per distinct key per
//            wavefront);
//   layout   one workgroup compacts the table into a class list sorted by
//            launch group, longest rows first, and fills each class's launch
//            parameters and the prefix sums of blocks and work items;
//   scatter  places every block in its class's segment of the index list
//            (its place is its class's start plus its rank, so no second
//            round of atomics is needed).
// The transform launches then walk the work items of one group, class by
// class in that order; every block of a class has the same geometry, so a
// wavefront's slots share the sweep of the whole-block decode.
#include "decode_body.h"

namespace mj {

namespace {

// The layout is one workgroup per call, launched while other streams may
// fill the chip: four wavefronts and 2 KB of LDS find a compute unit where
// sixteen wavefronts and 40 KB waited for one (its sort keys live in the
// workspace).  Serving trace, 1M requests/s: 85 us average per call with
// 1,024 threads and the keys in LDS (p99 375 us), 34 us like this (p99 74).
constexpr int kLayoutThreads = 256;

__device__ __forceinline__ uint64_t class_key(int geom, int ring, uint32_t P) {
    return ((uint64_t)(geom + 1) << 32) | ((uint64_t)ring << 31) | P;   // never 0
}

// Fibonacci hashing (Knuth, TAOCP vol. 3, 6.4): the top bits of key * 2^64/phi.
__device__ __forceinline__ uint32_t slot_hash(uint64_t key) {
    return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 52) & (kDescSlots - 1);
}

// The deepest read behind a row's newest pixel for the survivor set of
// `mask` (the Q survivors of smallest p, the r-th rebuilding row r):
// max over rows r != l of ceil((A_l - A_r)/2) - 1 - (l - r) p_r, with
// A_r = 2 (p_0 + ... + p_{r-1}) + r.
__device__ int survivor_depth(const GeomDev &g, uint32_t mask) {
    int ps[kMaxRows], A[kMaxRows];
    int cnt = 0, psum = 0;
    for (int s = 0; s < g.n && cnt < g.Q; ++s) {
        if ((mask >> g.id_sorted[s]) & 1u) continue;
        ps[cnt] = g.p_sorted[s];
        A[cnt] = 2 * psum + cnt;
        psum += g.p_sorted[s];
        ++cnt;
    }
    int depth = 0;
    for (int r = 0; r < cnt; ++r)
        for (int l = 0; l < cnt; ++l)
            if (l != r) depth = max(depth, ceil_half(A[l] - A[r]) - 1 - (l - r) * ps[r]);
    return depth;
}

__global__ void desc_clear_kernel(uint8_t *ws) {
    uint64_t *keys = reinterpret_cast<uint64_t *>(ws + DescWorkspace::kKeys);
    uint32_t *counts = reinterpret_cast<uint32_t *>(ws + DescWorkspace::kCounts);
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < kDescSlots;
         s += gridDim.x * blockDim.x) {
        keys[s] = 0;
        counts[s] = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x < sizeof(DescHeader) / 4)
        reinterpret_cast<uint32_t *>(ws + DescWorkspace::kHeader)[threadIdx.x] = 0;
}

// Inserts `key` (or finds it) and returns its slot, -1 if the table is full.
__device__ int insert_key(uint64_t *keys, uint64_t key) {
    uint32_t h = slot_hash(key);
    for (int probe = 0; probe < kDescSlots; ++probe) {
        const uint64_t seen = __atomic_load_n(&keys[h], __ATOMIC_RELAXED);
        if (seen == key) return (int)h;
        if (seen == 0) {
            const uint64_t prev = atomicCAS((unsigned long long *)&keys[h], 0ull,
                                            (unsigned long long)key);
            if (prev == 0 || prev == key) return (int)h;
        }
        h = (h + 1) & (kDescSlots - 1);
    }
    return -1;
}

__global__ __launch_bounds__(256) void desc_count_kernel(DescCall c) {
    uint64_t *keys = reinterpret_cast<uint64_t *>(c.ws + DescWorkspace::kKeys);
    uint32_t *counts = reinterpret_cast<uint32_t *>(c.ws + DescWorkspace::kCounts);
    int2 *slot_of = reinterpret_cast<int2 *>(c.ws + DescWorkspace::kSlotOf);
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // every lane of a wavefront runs the same number of rounds (ballots below)
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1));
         base < c.nblocks; base += stride) {
        const int64_t i = base + lane;
        int st = MOJETTE_OK;
        uint64_t key = 0;
        if (i < c.nblocks) {
            const mojette_block b = c.desc[i];
            if (b.geom_id >= c.ngeoms || b.P < 1 ||
                b.P > (uint32_t)(kDescMaxP >> c.geoms[b.geom_id].pshift)) {
                st = MOJETTE_EINVAL;
            } else {
                const GeomDev &g = c.geoms[b.geom_id];
                // the row in words: 2P for 128-bit pixels
                const uint32_t Pw = b.P << g.pshift;
                int ring = 0;
                if ((int64_t)Pw * g.Q > ((int64_t)1 << 30)) {
                    st = MOJETTE_EINVAL;
                } else if (c.decode) {
                    const uint32_t all = (1u << g.n) - 1u;
                    const bool two = g.two_min_P > 0 && (int)Pw >= g.two_min_P;
                    if (__builtin_popcount(~(uint32_t)b.erasure_mask & all) < g.Q)
                        st = MOJETTE_ENOTRECON;
                    else if (!two && g.R_short > 0 &&
                             survivor_depth(g, b.erasure_mask) <= g.depth_short)
                        ring = 1;
                }
                if (st == MOJETTE_OK) key = class_key(b.geom_id, ring, Pw);
            }
        }
        // one insertion and one count per distinct key of the wavefront
        int slot = -1, rank = 0;
        uint64_t todo = __ballot(key != 0);
        while (todo) {
            const int leader = __builtin_ctzll(todo);
            const uint64_t lk = __shfl(key, leader);
            const uint64_t same = __ballot(key == lk);
            int ls = -1;
            uint32_t base_rank = 0;
            if (lane == leader) {
                ls = insert_key(keys, lk);
                if (ls >= 0) base_rank = atomicAdd(&counts[ls], (uint32_t)__popcll(same));
            }
            ls = __shfl(ls, leader);
            base_rank = __shfl(base_rank, leader);
            if (key == lk) {
                slot = ls;
                rank = (int)base_rank + __popcll(same & ((1ull << lane) - 1ull));
            }
            todo &= ~same;
        }
        if (key != 0 && slot < 0) st = MOJETTE_ENOTSUP;
        if (i < c.nblocks) slot_of[i] = make_int2(st == MOJETTE_OK ? slot : -1, rank);
        if (st != MOJETTE_OK && c.status) *c.status = st;
    }
}

// Whether blocks of row length P of code g decode from both ends.
__device__ __forceinline__ bool two_corner(const DescCall &c, const GeomDev &g, int P) {
    return c.decode && g.two_min_P > 0 && P >= g.two_min_P;
}

__device__ __forceinline__ int64_t class_weight_items(const DescCall &c, const GeomDev &g,
                                                      int ring, int P, int64_t count, int &nb,
                                                      int &W) {
    if (c.decode) {
        if (two_corner(c, g, P)) {
            nb = g.nb_two;
            return (2 * count + nb - 1) / nb;   // two slots per block
        }
        nb = ring ? g.nb_short : g.nb;
        return (count + nb - 1) / nb;
    }
    W = min(g.enc_w, P);
    return count * ((P + W - 1) / W);
}

__global__ __launch_bounds__(kLayoutThreads) void desc_layout_kernel(DescCall c) {
    __shared__ int64_t scan[kLayoutThreads];
    __shared__ int nclasses;
    // sort keys: group, longest rows first, slot (global memory: the
    // workgroup's own writes, ordered by its barriers)
    uint64_t *order = reinterpret_cast<uint64_t *>(c.ws + DescWorkspace::kOrder);
    const uint64_t *keys = reinterpret_cast<const uint64_t *>(c.ws + DescWorkspace::kKeys);
    const uint32_t *counts = reinterpret_cast<const uint32_t *>(c.ws + DescWorkspace::kCounts);
    int32_t *slot_class = reinterpret_cast<int32_t *>(c.ws + DescWorkspace::kSlotClass);
    int64_t *seg_start = reinterpret_cast<int64_t *>(c.ws + DescWorkspace::kSegStart);
    int64_t *first_item = reinterpret_cast<int64_t *>(c.ws + DescWorkspace::kFirstItem);
    DescHeader &hd = *reinterpret_cast<DescHeader *>(c.ws + DescWorkspace::kHeader);
    const int tid = threadIdx.x;
    constexpr int PER = kDescSlots / kLayoutThreads;

    // 1. compact the occupied slots (in slot order) into sort keys
    int occ = 0;
    for (int k = 0; k < PER; ++k) occ += keys[tid * PER + k] != 0 && counts[tid * PER + k] > 0;
    scan[tid] = occ;
    __syncthreads();
    for (int off = 1; off < kLayoutThreads; off <<= 1) {   // inclusive scan (Hillis-Steele)
        const int64_t v = tid >= off ? scan[tid - off] : 0;
        __syncthreads();
        scan[tid] += v;
        __syncthreads();
    }
    int at = (int)scan[tid] - occ;
    if (tid == kLayoutThreads - 1) nclasses = (int)scan[tid];
    for (int k = 0; k < PER; ++k) {
        const int s = tid * PER + k;
        const uint64_t key = keys[s];
        if (key == 0 || counts[s] == 0) continue;
        const int geom = (int)(key >> 32) - 1;
        const uint32_t P = (uint32_t)key & 0x7FFFFFFFu;
        const int Q = c.geoms[geom].Q;
        const int two = two_corner(c, c.geoms[geom], (int)P) ? kTwoGroup : 0;
        const uint64_t group = c.group_by_q ? (uint64_t)(Q + two) : 0;
        // ascending: group, then P descending, then Q descending, then slot
        order[at++] = (group << 58) | ((uint64_t)(0x1FFFFFFu - P) << 33) |
                      ((uint64_t)(0xFF - Q) << 25) | (uint64_t)s;
    }
    __syncthreads();
    const int nc = nclasses;
    int n2 = 1;
    while (n2 < nc) n2 <<= 1;
    for (int s = nc + tid; s < n2; s += kLayoutThreads) order[s] = ~0ull;
    __syncthreads();
    // 2. bitonic sort of the n2 keys
    for (int k = 2; k <= n2; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = tid; i < n2; i += kLayoutThreads) {
                const int ixj = i ^ j;
                if (ixj > i) {
                    const uint64_t a = order[i], b = order[ixj];
                    const bool up = (i & k) == 0;
                    if ((a > b) == up) {
                        order[i] = b;
                        order[ixj] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
    // 3. per class (sorted): blocks and work items, scanned in order; rounds
    // of one class per thread (one round for up to kLayoutThreads classes)
    int32_t *idx = reinterpret_cast<int32_t *>(c.ws + DescWorkspace::idx_at(c.nblocks));
    int64_t run_blocks = 0, run_items = 0;   // totals of the earlier rounds
    for (int base = 0; base < nc; base += kLayoutThreads) {
        const int ci = base + tid;
        int64_t my_blocks = 0, my_items = 0;
        int s = 0, geom = 0, ring = 0, P = 0, nb = 1, W = 1;
        if (ci < nc) {
            s = (int)(order[ci] & (kDescSlots - 1));
            const uint64_t key = keys[s];
            geom = (int)(key >> 32) - 1;
            ring = (int)((key >> 31) & 1);
            P = (int)(key & 0x7FFFFFFFu);
            my_blocks = counts[s];
            my_items = class_weight_items(c, c.geoms[geom], ring, P, counts[s], nb, W);
        }
        // exclusive scans of blocks and items over the round (two passes of one buffer)
        int64_t blocks_before = 0, items_before = 0, tot_blocks = 0, tot_items = 0;
        for (int pass = 0; pass < 2; ++pass) {
            const int64_t mine = pass == 0 ? my_blocks : my_items;
            scan[tid] = mine;
            __syncthreads();
            for (int off = 1; off < kLayoutThreads; off <<= 1) {
                const int64_t v = tid >= off ? scan[tid - off] : 0;
                __syncthreads();
                scan[tid] += v;
                __syncthreads();
            }
            const int64_t excl = scan[tid] - mine, tot = scan[kLayoutThreads - 1];
            if (pass == 0) {
                blocks_before = run_blocks + excl;
                tot_blocks = tot;
            } else {
                items_before = run_items + excl;
                tot_items = tot;
            }
            __syncthreads();
        }
        run_blocks += tot_blocks;
        run_items += tot_items;
        if (ci >= nc) continue;
        const GeomDev &g = c.geoms[geom];
        slot_class[s] = ci;
        seg_start[ci] = blocks_before;
        first_item[ci] = items_before;
        // projection i's stored bins: Eq. 2's, or the kept ones
        int32_t off[kMaxDirs], kept[kMaxDirs];
        int32_t o = 0;
        for (int i = 0; i < g.n; ++i) {
            off[i] = o;
            kept[i] = g.keep_rows[i] < 0 ? 0 : P + g.keep_rows[i] * abs(g.dirs[i]);
            o += kept[i] ? kept[i] : proj_bins(g.dirs[i], P, g.Q);
        }
        if (c.decode) {
            DecodeDesc &d = reinterpret_cast<DecodeDesc *>(c.ws + DescWorkspace::kClasses)[ci];
            d.desc = (global_block *)c.desc;
            d.idx = (global_i32 *)(idx + blocks_before);
            d.pool = (global_u64 *)c.pool;
            d.status = c.status;
            d.images = nullptr;
            d.masks = nullptr;
            d.slots = nullptr;
            d.nblocks = my_blocks;
            d.proj_stride = o;
            d.img_stride = (int64_t)P * g.Q;
            d.P = P;
            d.Q = g.Q;
            d.n = g.n;
            d.nb = nb;
            d.R = two_corner(c, g, P) ? g.R_two : ring ? g.R_short : g.R;
            d.ring_stride = ring_stride_of(g.Q, d.R);
            d.mask_uniform = 0;
            d.bin_swap = g.pshift;
            for (int i = 0; i < kMaxDirs; ++i) {
                d.off[i] = i < g.n ? off[i] : 0;
                d.p_sorted[i] = g.p_sorted[i];
                d.id_sorted[i] = g.id_sorted[i];
                d.keep_lo[i] = i < g.n && kept[i] ? g.keep_lo[i] : 0;
            }
        } else {
            EncodeDesc &e = reinterpret_cast<EncodeDesc *>(c.ws + DescWorkspace::kClasses)[ci];
            e.desc = (global_block *)c.desc;
            e.idx = (global_i32 *)(idx + blocks_before);
            e.pool = (global_u64 *)c.pool;
            e.nblocks = my_blocks;
            e.P = P;
            e.Q = g.Q;
            e.n = g.n;
            e.W = W;
            e.H = g.H;
            e.S = W + 2 * g.H;
            e.plo = g.plo;
            e.pspan = g.pspan;
            e.ntiles = (P + W - 1) / W;
            e.bin_swap = g.pshift;
            for (int i = 0; i < kMaxDirs; ++i) {
                e.off[i] = i < g.n ? off[i] : 0;
                e.p[i] = i < g.n ? g.dirs[i] : 0;
                e.keep_lo[i] = i < g.n && kept[i] ? g.keep_lo[i] : 0;
                e.keep_n[i] = i < g.n ? kept[i] : 0;
            }
        }
        // launch groups: where the group of consecutive classes changes
        const int grp = (int)(order[ci] >> 58);
        if (ci == 0 || (int)(order[ci - 1] >> 58) != grp) hd.range[2 * grp] = items_before;
        if (ci == nc - 1 || (int)(order[ci + 1] >> 58) != grp)
            hd.range[2 * grp + 1] = items_before + my_items;
    }
    if (tid == 0) {
        seg_start[nc] = run_blocks;
        first_item[nc] = run_items;
        hd.nclasses = nc;
    }
}

__global__ __launch_bounds__(256) void desc_scatter_kernel(DescCall c) {
    const int2 *slot_of = reinterpret_cast<const int2 *>(c.ws + DescWorkspace::kSlotOf);
    const int32_t *slot_class = reinterpret_cast<const int32_t *>(c.ws + DescWorkspace::kSlotClass);
    const int64_t *seg_start = reinterpret_cast<const int64_t *>(c.ws + DescWorkspace::kSegStart);
    int32_t *idx = reinterpret_cast<int32_t *>(c.ws + DescWorkspace::idx_at(c.nblocks));
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.nblocks;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int2 sr = slot_of[i];
        if (sr.x < 0) continue;
        idx[seg_start[slot_class[sr.x]] + sr.y] = (int32_t)i;
    }
}

// The decode of the work items of launch group g: batches of every class of
// the group, in class order, one wavefront per workgroup.  QMASK has bit Q
// set for every row count the launch may meet (only those bodies are
// compiled in); bodies are compiled for half the block slots.
template <unsigned QMASK, int CH>
__global__ __launch_bounds__(kWave) void decode_desc_kernel(const uint8_t *__restrict__ ws, int g) {
    const DescHeader &hd = *reinterpret_cast<const DescHeader *>(ws + DescWorkspace::kHeader);
    const int64_t *first = reinterpret_cast<const int64_t *>(ws + DescWorkspace::kFirstItem);
    const DecodeDesc *cls = reinterpret_cast<const DecodeDesc *>(ws + DescWorkspace::kClasses);
    const int64_t lo = hd.range[2 * g], hi = hd.range[2 * g + 1];
    const int nc = hd.nclasses;
    for (int64_t item = lo + blockIdx.x; item < hi; item += gridDim.x) {
        int c0 = 0, c1 = nc;
        while (c1 - c0 > 1) {
            const int m = (c0 + c1) >> 1;
            if (first[m] <= item) c0 = m; else c1 = m;
        }
        const DecodeDesc &a = cls[c0];
        const int64_t batch = item - first[c0];
        switch (a.Q) {
#define MJ_DEC_CASE(QQ)                                                                    \
    case QQ:                                                                               \
        if constexpr ((QMASK >> QQ) & 1u)                                                 \
            decode_batch<QQ, kDecodeTile, false, CH, half_slots<QQ>(), DecodeDesc, 0>(    \
                a, batch);                                                                 \
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

}  // namespace

hipError_t launch_desc_buckets(const DescCall &c, hipStream_t s) {
    hipLaunchKernelGGL(desc_clear_kernel, dim3(kDescSlots / 256), dim3(256), 0, s, c.ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((c.nblocks + 255) / 256, 4096));
    hipLaunchKernelGGL(desc_count_kernel, dim3(grid), dim3(256), 0, s, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(desc_layout_kernel, dim3(1), dim3(kLayoutThreads), 0, s, c);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(desc_scatter_kernel, dim3(grid), dim3(256), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_decode_desc(int Q, bool two, const DescCall &c, int g, size_t lds, int grid,
                              hipStream_t s) {
    const uint8_t *ws = c.ws;
    switch (Q) {
#define MJ_LAUNCH(QQ)                                                                          \
    case QQ:                                                                                   \
        if (two)                                                                               \
            hipLaunchKernelGGL((decode_desc_kernel<1u << QQ, kTwoCorner>), dim3(grid),          \
                               dim3(kWave), lds, s, ws, g);                                    \
        else                                                                                   \
            hipLaunchKernelGGL((decode_desc_kernel<1u << QQ, kWhole>), dim3(grid), dim3(kWave), \
                               lds, s, ws, g);                                                 \
        break;
        MJ_LAUNCH(1) MJ_LAUNCH(2) MJ_LAUNCH(3) MJ_LAUNCH(4) MJ_LAUNCH(5) MJ_LAUNCH(6)
        MJ_LAUNCH(7) MJ_LAUNCH(8) MJ_LAUNCH(9) MJ_LAUNCH(10) MJ_LAUNCH(11) MJ_LAUNCH(12)
        MJ_LAUNCH(13) MJ_LAUNCH(14) MJ_LAUNCH(15) MJ_LAUNCH(16)
#undef MJ_LAUNCH
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mj
