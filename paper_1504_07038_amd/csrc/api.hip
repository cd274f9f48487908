// C-ABI entry points: argument checking, per-geometry launch parameters and
// kernel launches.  Only the plan calls of the chunked decode allocate device
// memory or synchronise; every other call does neither.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "mj_internal.h"

namespace {

using mj::kMaxDirs;
using mj::kMaxRows;

constexpr size_t kLdsLimit = 64 * 1024;        // dynamic LDS per workgroup used by the kernels
constexpr size_t kMixedEncodeLds = 20 * 1024;  // per workgroup in mixed encode launches
constexpr size_t kMixedDecodeLds = 40 * 1024;  // per workgroup in mixed decode launches
constexpr size_t kDecodeLdsShare = 34 * 1024;  // decode LDS per wavefront, short rings
constexpr size_t kDecodeLdsLong = 26 * 1024;   // decode LDS per wavefront, long rings
constexpr int64_t kScanWaveBudget = 1024;      // chunked decode: parallel carry below this many waves
constexpr int kMaxP = 1 << 24;                 // keeps every bin index inside int32
constexpr int kMaxAbsP = 1 << 16;
// Workgroups per launch; larger batches loop inside the kernel.  Measured on
// 2^21 4 KB (6,4) blocks: the encode runs 5% faster with one work item per
// wavefront (no loop) than with 2^14 workgroups, the decode 1% faster with
// 2^16 workgroups (4 batches per wavefront at 2^15).
constexpr int kEncodeGridCap = 1 << 19;
constexpr int kDecodeGridCap = 1 << 16;
constexpr int kGatherRange = 256;              // blocks a deep-class wavefront scans (<= 512)
constexpr int kMaxSysParity = 8;               // parity projections of the systematic code

bool geometry_ok(const int32_t *dirs, int32_t n, int32_t P, int32_t Q) {
    if (!dirs || n < 1 || n > kMaxDirs || P < 1 || P > kMaxP || Q < 1 || Q > kMaxRows) return false;
    if ((int64_t)P * Q > ((int64_t)1 << 30)) return false;
    for (int i = 0; i < n; ++i) {
        if (dirs[i] < -kMaxAbsP || dirs[i] > kMaxAbsP) return false;
        for (int j = 0; j < i; ++j)
            if (dirs[i] == dirs[j]) return false;
    }
    return true;
}

// The encode of 128-bit pixels (Section 3.1) runs on the 64-bit kernels:
// half h of pixel k is word column 2k + h of a 2P-wide image of words, whose
// projection along (2p, 1) holds bin j of the 16-byte projection along
// (p, 1) in word bins 2j+1 and 2j (the kernel exchanges the two with
// bin_swap).  Checks the 16-byte geometry and fills dirs2 with the doubled
// directions.
bool wide_geometry(const int32_t *dirs, int32_t n, int32_t P, int32_t Q, int32_t *dirs2) {
    if (!geometry_ok(dirs, n, P, Q) || P > kMaxP / 2) return false;
    for (int i = 0; i < n; ++i) {
        if (dirs[i] < -kMaxAbsP / 2 || dirs[i] > kMaxAbsP / 2) return false;
        dirs2[i] = 2 * dirs[i];
    }
    return geometry_ok(dirs2, n, 2 * P, Q);
}

// Never-used bins (Section 2.3) for the reconstruction path of the decode
// kernels: of the survivors the Q with the smallest p are used, the r-th for
// image row r, which reads bins r*p - k for k in [0, P).  The projection of
// rank i among the sorted directions is the r-th for some erasure pattern
// exactly when max(0, i - (n - Q)) <= r <= min(i, Q - 1), so it keeps the
// bins from min(r_lo*p, r_hi*p) - P + 1 to max(r_lo*p, r_hi*p):
// P + (r_hi - r_lo)*|p| of them.  Fills, per projection in the caller's
// order, the first kept bin index (b - b_min) and the count; false if the
// geometry is invalid or n < Q.
bool kept_layout(const int32_t *dirs, int32_t n, int32_t P, int32_t Q, int32_t *first,
                 int32_t *count) {
    if (!geometry_ok(dirs, n, P, Q) || n < Q) return false;
    for (int i = 0; i < n; ++i) {
        int rank = 0;
        for (int j = 0; j < n; ++j) rank += dirs[j] < dirs[i];
        const int r_lo = std::max(0, rank - (n - Q)), r_hi = std::min(rank, Q - 1);
        const int64_t p = dirs[i];
        const int64_t b_first = std::min(r_lo * p, r_hi * p) - P + 1;
        first[i] = (int32_t)(b_first - mojette_bin_offset(dirs[i], P, Q));
        count[i] = (int32_t)(P + (int64_t)(r_hi - r_lo) * std::llabs(p));
    }
    return true;
}

int status_of(hipError_t e) { return mj::hip_status(e); }

// Kernel launches report through hipGetLastError(), which also returns an
// error left behind by any earlier HIP call of the thread (the caller's or a
// framework's).  Such a stale error is cleared before each launch so that a
// call reports only its own failure.
void clear_stale_error() { (void)hipGetLastError(); }

thread_local hipError_t g_last_hip = hipSuccess;

// Encode tiling: the whole row when it fits, else the widest multiple of 64
// columns whose tile plus halo fits the LDS budget, and at most `max_w`
// columns (0: no cap).  Four waves per workgroup when their four tiles fit
// (at least min(P, 256, max_w) columns each), else two, else one;
// `max_waves` caps that choice.  `lds_budget` (bytes per workgroup) defaults
// to all the LDS a workgroup may take; mixed launches, which give every
// workgroup the LDS of their largest class, pass less so that more
// wavefronts share a compute unit.  Single-geometry launches cap tiles at
// 128 columns: the smaller LDS tiles let twice the wavefronts share a
// compute unit (measured: 8 KB (6,4) blocks encode 1.24x faster than with
// whole 256-column rows).
constexpr int kEncodeTileCols = 128;
bool encode_tiling(const int32_t *dirs, int32_t n, int32_t P, int32_t Q, mj::EncodeArgs &a,
                   int max_waves = mj::kEncodeWaves, size_t lds_budget = kLdsLimit,
                   int max_w = kEncodeTileCols) {
    int maxabs = 0;
    for (int i = 0; i < n; ++i) maxabs = std::max(maxabs, std::abs(dirs[i]));
    const int H = (Q - 1) * maxabs;
    int want = std::min(P, 256);
    if (max_w > 0) want = std::min(want, max_w);
    // a tile of at least 128 columns beside its halo always fits
    lds_budget = std::min(kLdsLimit, std::max(lds_budget, (size_t)Q * (2 * H + 128) * 8));
    int waves = max_waves;
    size_t cols_fit = 0;
    for (; waves >= 1; waves /= 2) {
        cols_fit = lds_budget / ((size_t)waves * Q * sizeof(uint64_t));
        if (cols_fit >= (size_t)(2 * H + want) || (waves == 1 && cols_fit >= (size_t)(2 * H + 64)))
            break;
    }
    if (waves < 1) return false;
    int W = P;
    if ((size_t)(P + 2 * H) > cols_fit) W = (int)((cols_fit - 2 * H) / 64 * 64);
    if (max_w > 0 && W > max_w) W = max_w;
    // Workgroups of several wavefronts whose tiles take more than 48 KB of
    // LDS leave a CU two of them, 8 wavefronts; one wavefront per workgroup
    // then keeps more resident.  Measured, 8 KB (12,8) blocks (13.6 KB
    // tiles): one wavefront 2.31 ms, two 2.41, four 2.60; with smaller tiles
    // four stay best (4 KB (6,4): 4.23 ms against 4.45 with two and 4.58
    // with one; 16-byte pixels at P = 64: 4.49 against 4.65 with two).
    {
        const size_t tile = (size_t)Q * (W + 2 * H) * sizeof(uint64_t);
        if ((size_t)waves * tile > 48 * 1024) waves = 1;
    }
    a.waves = waves;
    a.W = W;
    a.H = H;
    a.S = W + 2 * H;
    a.ntiles = (P + W - 1) / W;
    a.P = P;
    a.Q = Q;
    a.n = n;
    for (int i = 0; i < n; ++i) a.p[i] = dirs[i];
    return true;
}

// Ring length for the decoder: the largest distance D between the newest
// pixel of row l and the pixel (k + (l-r)p_r, l) that row r reads, over
// every Q-subset of the directions, plus one, rounded up to a power of two
// and to at least the tile width.  D = ceil((A_l - A_r)/2) - 1 - (l-r)p_r is
// independent of k.  A negative D would mean a pixel is read before it is
// written; the ordering argument in decode_body.h rules that out, and this
// function re-checks it (returns -1 then).
struct RingKey {
    std::vector<int> p;
    int Q;
    bool operator<(const RingKey &o) const { return Q != o.Q ? Q < o.Q : p < o.p; }
};

// Ring for a depth D: a staged bin must not land on a pixel still needed
// (TW + D + 1) or on one not yet stored (2 TW).
static int ring_for_depth(int D) {
    int R = 2 * mj::kDecodeTile;
    while (R < mj::kDecodeTile + D + 1) R <<= 1;
    return R;
}

// Also returns in *common the shortest ring that serves at least 90% of
// the survivor sets (the whole-block pool decode sweeps the others in a
// second launch with the full ring) and in *deep the fraction of sets it
// does not serve.
struct RingInfo {
    int R, common;
    double deep;
};

int ring_length(const std::vector<int> &sorted_p, int Q, int *common = nullptr,
                double *deep = nullptr) {
    static std::mutex mu;
    static std::map<RingKey, RingInfo> cache;
    RingKey key{sorted_p, Q};
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) {
            if (common) *common = it->second.common;
            if (deep) *deep = it->second.deep;
            return it->second.R;
        }
    }
    const int n = (int)sorted_p.size();
    int Dmax = 0;
    bool ok = true;
    std::vector<int> depths;
    std::vector<int> pick(Q), A(Q);
    for (int i = 0; i < Q; ++i) pick[i] = i;
    while (true) {
        int psum = 0;
        for (int r = 0; r < Q; ++r) {
            A[r] = 2 * psum + r;
            psum += sorted_p[pick[r]];
        }
        int Dset = 0;
        for (int r = 0; r < Q; ++r) {
            const int pr = sorted_p[pick[r]];
            for (int l = 0; l < Q; ++l) {
                if (l == r) continue;
                const int diff = A[l] - A[r];
                const int ceil_half = (diff >= 0) ? (diff + 1) / 2 : -((-diff) / 2);
                const int D = ceil_half - 1 - (l - r) * pr;
                if (D < 0) ok = false;
                Dset = std::max(Dset, D);
            }
        }
        depths.push_back(Dset);
        Dmax = std::max(Dmax, Dset);
        int i = Q - 1;
        while (i >= 0 && pick[i] == n - Q + i) --i;
        if (i < 0) break;
        ++pick[i];
        for (int j = i + 1; j < Q; ++j) pick[j] = pick[j - 1] + 1;
    }
    int R = -1, Rc = -1;
    double frac = 0;
    if (ok) {
        R = ring_for_depth(Dmax);
        std::sort(depths.begin(), depths.end());
        Rc = ring_for_depth(depths[(depths.size() * 9 + 9) / 10 - 1]);   // 90th percentile
        int64_t over = 0;
        for (int d : depths) over += d > Rc - mj::kDecodeTile - 1;
        frac = (double)over / (double)depths.size();
    }
    if (common) *common = Rc;
    if (deep) *deep = frac;
    std::lock_guard<std::mutex> g(mu);
    cache[key] = {R, Rc, frac};
    return R;
}

// Ring length of the systematic decode: as ring_length, over every set of
// lost lines (1 to m of the Q) and every choice of as many parity
// directions, with the sweep rows at the lost lines' image rows (A of the
// next lost line: A + 2 (its row - this row) p + 1).  A known line l is read
// by sweep row r at offset d_r + (l - m_r) p_r from the tile's first column
// (d_r = -floor((A_max - A_r)/2)); its windows are staged at the largest of
// those offsets, so the ring also spans their spread, and *lead tiles of it
// are staged before the sweep starts.  -1 if a pixel would be read before
// it is written (the ordering argument rules it out).
int ring_length_sys(const std::vector<int> &sorted_p, int Q, int *lead) {
    const int m = (int)sorted_p.size();
    int Dmax = 0, spread = 0;
    bool ok = true;
    for (uint32_t lines = 1; lines < (1u << Q); ++lines) {
        const int e = __builtin_popcount(lines);
        if (e > m) continue;
        std::vector<int> rows;
        for (int l = 0; l < Q; ++l)
            if ((lines >> l) & 1u) rows.push_back(l);
        for (uint32_t dirs = 1; dirs < (1u << m); ++dirs) {
            if (__builtin_popcount(dirs) != e) continue;
            std::vector<int> p, A(e);
            for (int i = 0; i < m; ++i)
                if ((dirs >> i) & 1u) p.push_back(sorted_p[i]);
            A[0] = 0;
            for (int r = 0; r + 1 < e; ++r) A[r + 1] = A[r] + 2 * (rows[r + 1] - rows[r]) * p[r] + 1;
            for (int r = 0; r < e; ++r)
                for (int l = 0; l < e; ++l) {
                    if (l == r) continue;
                    const int diff = A[l] - A[r];
                    const int ceil_half = (diff >= 0) ? (diff + 1) / 2 : -((-diff) / 2);
                    const int D = ceil_half - 1 - (rows[l] - rows[r]) * p[r];
                    if (D < 0) ok = false;
                    Dmax = std::max(Dmax, D);
                }
            const int A_max = *std::max_element(A.begin(), A.end());
            for (int l = 0; l < Q; ++l) {
                if ((lines >> l) & 1u) continue;
                int lo = INT32_MAX, hi = INT32_MIN;
                for (int r = 0; r < e; ++r) {
                    const int o = -((A_max - A[r]) >> 1) + (l - rows[r]) * p[r];
                    lo = std::min(lo, o);
                    hi = std::max(hi, o);
                }
                spread = std::max(spread, hi - lo);
            }
        }
    }
    if (!ok) return -1;
    const int TW = mj::kDecodeTile;
    *lead = (spread + TW - 1) / TW;
    int R = 2 * TW;
    while (R < TW + Dmax + 1 || R < TW + spread || R < (*lead + 1) * TW) R <<= 1;
    return R;
}

// Blocks per wavefront: all the lanes allow when their rings fit a 34 KB
// share of LDS (short rings: the (6,4) code's 32 blocks); otherwise at most
// half of them (the body compiled for half the slots needs far fewer
// registers) and no more than 26 KB, so that several wavefronts share a
// compute unit.  Measured on 2^19 blocks: (12,8) 3 blocks per wavefront
// 1.25x faster than 7; (6,3) 10 blocks 1.3x faster than 20; (12,4) 2 blocks
// 1.17x faster than 5.
int default_blocks(int Q, int ring_stride) {
    int nb = mj::decode_max_blocks_per_wave(Q);
    if (mj::decode_lds_bytes(Q, nb, ring_stride) > kDecodeLdsShare) {
        nb = std::max(1, nb / 2);
        while (nb > 1 && mj::decode_lds_bytes(Q, nb, ring_stride) > kDecodeLdsLong) --nb;
    }
    return nb;
}

// Fills the geometry part of decode arguments (DecodeArgs or DecodeClass).
// Returns a status.
template <class A>
int decode_setup(const int32_t *dirs, int32_t n, int32_t P, int32_t Q, A &a) {
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return dirs[x] < dirs[y]; });
    std::vector<int> sp(n);
    for (int s = 0; s < n; ++s) {
        a.p_sorted[s] = dirs[order[s]];
        a.id_sorted[s] = order[s];
        sp[s] = dirs[order[s]];
    }
    if (n < Q) return MOJETTE_ENOTRECON;
    const int R = ring_length(sp, Q);
    if (R < 0) return MOJETTE_EINVAL;
    a.R = R;
    a.ring_stride = mj::ring_stride_of(Q, R);
    a.nb = default_blocks(Q, a.ring_stride);
    if (mj::decode_lds_bytes(Q, a.nb, a.ring_stride) > kLdsLimit) return MOJETTE_ENOTSUP;
    a.P = P;
    a.n = n;
    return MOJETTE_OK;
}

// The library's blocks per wavefront for a single-geometry pool decode.  For
// 4 rows and the shortest ring, at most half of what the lanes allow, so
// that the body compiled for half the slots runs, the one whose loads fetch
// every line once (ALIGN in decode_body.h; 4 KB (6,4): 3.85 ms at 16 blocks
// per wavefront against 4.00 ms at 32 with the unaligned full-slot body).
int pool_default_blocks(int Q, int ring_stride) {
    const int nb = default_blocks(Q, ring_stride);
    if (Q != 4 || ring_stride != mj::ring_stride_of(Q, 2 * mj::kDecodeTile)) return nb;
    return std::min(nb, std::max(1, mj::decode_max_blocks_per_wave(Q) / 2));
}

// Compute units of the current device (cached per device).
static int device_cus() {
    static std::mutex mu;
    static std::map<int, int> cus;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    std::lock_guard<std::mutex> g(mu);
    auto it = cus.find(dev);
    if (it != cus.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n <= 0)
        n = 256;
    return cus[dev] = n;
}

// Launches the whole-block pool decode described by `a` (from decode_setup,
// pool fields filled).  nb_req > 0: blocks per wavefront asked by the caller
// (capped by LDS).  When a shorter ring serves at least 90% of the survivor
// sets and the batch is large enough to keep the chip busy for at least two
// rounds of wavefronts, two launches run: that ring over the blocks whose
// set fits it (more blocks per wavefront), then the full ring over the rest.
// A smaller batch is bound by one block's sweep, which a second launch would
// repeat (256 1 MB (8,4) blocks: 6.2 ms in one launch, 12.6 ms in two).  The
// second launch sweeps every batch that holds a deep block, so the split is
// taken only while, with the deep sets drawn uniformly, at most a quarter
// of its batches would (the 128-bit (6,4) geometry, 1 deep set in 15 at 12
// blocks per wavefront, ran 1,380 against 1,823 GB/s split).
// The launches of a whole-block pool decode (see launch_pool_whole), in
// order, without launching them.  MOJETTE_ENOTSUP when a wave's slice is
// beyond 32-bit byte offsets even in one launch.
int plan_pool_whole(mj::DecodeArgs a, int Q, int nb_req, std::vector<mj::DecodeArgs> &out) {
    out.clear();
    auto pick_nb = [&](mj::DecodeArgs &b) {
        if (nb_req > 0) {
            b.nb = std::min(mj::decode_max_blocks_per_wave(Q), nb_req);
            while (b.nb > 1 && mj::decode_lds_bytes(Q, b.nb, b.ring_stride) > kLdsLimit) --b.nb;
        } else {
            b.nb = pool_default_blocks(Q, b.ring_stride);
        }
    };
    // A wave addresses its slice of the pool and of the images (its nb
    // blocks, or the gather_range blocks it scans) with 32-bit byte offsets.
    auto slice_fits = [](const mj::DecodeArgs &b) {
        const int64_t span = std::max<int64_t>(b.nb, b.gather_range);
        return span * b.proj_stride * 8 < ((int64_t)1 << 31) &&
               span * b.img_stride * 8 < ((int64_t)1 << 31);
    };
    auto add = [&](mj::DecodeArgs b) {
        // whole-line loads pay with the shortest rings only
        b.align = b.R == 2 * mj::kDecodeTile;
        if (!slice_fits(b)) return MOJETTE_ENOTSUP;
        out.push_back(b);
        return MOJETTE_OK;
    };
    std::vector<int> sp(a.p_sorted, a.p_sorted + a.n);
    int common = -1;
    double deep = 1;
    ring_length(sp, Q, &common, &deep);
    bool split = common > 0 && common < a.R;
    if (split) {
        mj::DecodeArgs b = a;
        pick_nb(b);
        const size_t lds = mj::decode_lds_bytes(Q, b.nb, b.ring_stride);
        const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(32, (160 * 1024) / lds));
        const int64_t batches = (b.nblocks + b.nb - 1) / b.nb;
        const int nb2 = pool_default_blocks(Q, a.ring_stride);
        split = batches >= 2 * per_cu * device_cus() && 1.0 - std::pow(1.0 - deep, nb2) <= 0.25;
        // the gathered launch's slices span kGatherRange blocks: blocks too
        // large for 32-bit offsets over that span stay in one launch
        mj::DecodeArgs g = a;
        g.nb = nb2;
        g.gather_range = kGatherRange;
        if (!slice_fits(g)) split = false;
    }
    if (!split) {
        a.ring_mode = 0;
        pick_nb(a);
        return add(a);
    }
    // the short ring serves sets whose depth is at most common - TW - 1
    a.ring_depth = common - mj::kDecodeTile - 1;
    mj::DecodeArgs m1 = a;
    m1.R = common;
    m1.ring_stride = mj::ring_stride_of(Q, common);
    m1.ring_mode = 1;
    pick_nb(m1);
    const int rc = add(m1);
    if (rc != MOJETTE_OK) return rc;
    // the deep class is a few scattered blocks: gathered from ranges of 256
    a.ring_mode = 2;
    a.nb = pool_default_blocks(Q, a.ring_stride);
    a.gather_range = kGatherRange;
    return add(a);
}

// Streams of the descriptor decode's launch groups (one per row count and
// the group decoded from both ends; also the deep class of a split
// whole-block pool decode): each group runs on a stream of its own,
// forked from the caller's stream after the bucketing and joined back to it
// with events, so that a group bound by the chains of its long rows runs
// beside the others instead of before them (a chunk of the mixed workload:
// its 4-row group, 1 MB rows, takes 10 ms of which 7 ms are one chain, the
// chip otherwise idle).  Created once per device, at plan creation or at
// the first pool decode that is not being captured; default priority.  The fork and join are recorded
// under a lock so that calls from several threads do not mix their events.
namespace {
constexpr int kForkStreams = 4;
struct ForkPool {
    hipStream_t st[kForkStreams];
    hipEvent_t fork, join[kForkStreams];
    std::mutex mu;
};

ForkPool *fork_pool(int dev, bool create) {
    static std::mutex mu;
    static std::map<int, ForkPool *> pools;
    std::lock_guard<std::mutex> g(mu);
    auto it = pools.find(dev);
    if (it != pools.end()) return it->second;
    if (!create) return nullptr;
    auto *fp = new (std::nothrow) ForkPool{};
    if (!fp) return nullptr;
    hipError_t e = hipEventCreateWithFlags(&fp->fork, hipEventDisableTiming);
    for (int k = 0; k < kForkStreams && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&fp->st[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&fp->join[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        mj::hip_status(e);
        return nullptr;   // the few handles made stay with the process
    }
    return pools[dev] = fp;
}
}  // namespace

int launch_pool_whole(const mj::DecodeArgs &a, int Q, int nb_req, hipStream_t stream) {
    std::vector<mj::DecodeArgs> launches;
    const int rc = plan_pool_whole(a, Q, nb_req, launches);
    if (rc != MOJETTE_OK) return rc;
    // a split decode (short-ring class, then the deep sets): the deep launch
    // on a fork stream beside the first (they write different blocks)
    ForkPool *fp = nullptr;
    if (launches.size() == 2) {
        int dev = 0;
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipGetDevice(&dev) == hipSuccess) {
            const bool capturing = hipStreamIsCapturing(stream, &cs) == hipSuccess &&
                                   cs != hipStreamCaptureStatusNone;
            fp = fork_pool(dev, !capturing);
        }
        (void)hipGetLastError();   // a failed lookup leaves the launches in order
    }
    std::unique_lock<std::mutex> fork_lock;
    if (fp) {
        fork_lock = std::unique_lock<std::mutex>(fp->mu);
        hipError_t fe = hipEventRecord(fp->fork, stream);
        if (fe == hipSuccess) fe = hipStreamWaitEvent(fp->st[0], fp->fork, 0);
        if (fe != hipSuccess) return mj::hip_status(fe);
    }
    int rc2 = MOJETTE_OK;
    for (size_t i = 0; i < launches.size() && rc2 == MOJETTE_OK; ++i) {
        const mj::DecodeArgs &b = launches[i];
        // gathering launches: one wavefront per range of gather_range blocks
        const int64_t per_wave = b.gather_range > 0 ? b.gather_range : b.nb;
        const int64_t batches = (b.nblocks + per_wave - 1) / per_wave;
        const int grid = (int)std::min<int64_t>(batches, kDecodeGridCap);
        clear_stale_error();
        rc2 = status_of(mj::launch_decode(Q, mj::kLaunchPool, b, grid,
                                          fp && i == 1 ? fp->st[0] : stream));
    }
    if (fp) {
        hipError_t fe = hipEventRecord(fp->join[0], fp->st[0]);
        if (fe == hipSuccess) fe = hipStreamWaitEvent(stream, fp->join[0], 0);
        if (fe != hipSuccess && rc2 == MOJETTE_OK) rc2 = mj::hip_status(fe);
    }
    return rc2;
}

// Checks a class table and returns, per class, block words and pool offsets.
int classes_check(const mojette_class *cls, int32_t ncls, std::vector<int64_t> &bw,
                  std::vector<int64_t> &img_off, std::vector<int64_t> &proj_off,
                  std::vector<int64_t> &mask_off, int64_t &img_total, int64_t &proj_total) {
    if (!cls || ncls < 1 || ncls > mj::kMaxClasses) return MOJETTE_EINVAL;
    bw.assign(ncls, 0);
    img_off.assign(ncls, 0);
    proj_off.assign(ncls, 0);
    mask_off.assign(ncls, 0);
    img_total = proj_total = 0;
    int64_t masks = 0;
    for (int c = 0; c < ncls; ++c) {
        const mojette_class &k = cls[c];
        if (k.nblocks < 0 || !geometry_ok(k.dirs, k.n, k.P, k.Q)) return MOJETTE_EINVAL;
        for (int i = 0; i < k.n; ++i)
            if (k.dirs[i] < -32767 || k.dirs[i] > 32767) return MOJETTE_EINVAL;
        bw[c] = mojette_block_words(k.dirs, k.n, k.P, k.Q);
        img_off[c] = img_total;
        proj_off[c] = proj_total;
        mask_off[c] = masks;
        img_total += k.nblocks * (int64_t)k.P * k.Q;
        proj_total += k.nblocks * bw[c];
        masks += k.nblocks;
    }
    return MOJETTE_OK;
}

}  // namespace

int mj::hip_status(hipError_t e) {
    if (e == hipSuccess) return MOJETTE_OK;
    g_last_hip = e;
    return MOJETTE_EHIP;
}

extern "C" {

const char *mojette_last_hip_error(void) {
    return g_last_hip == hipSuccess ? "no HIP error" : hipGetErrorName(g_last_hip);
}

const char *mojette_strerror(int status) {
    switch (status) {
        case MOJETTE_OK: return "ok";
        case MOJETTE_EINVAL: return "invalid argument";
        case MOJETTE_ENOTRECON: return "fewer than Q projections survive: not reconstructible";
        case MOJETTE_EHIP: return "HIP runtime error";
        case MOJETTE_ENOMEM: return "out of host memory";
        case MOJETTE_ENOTSUP: return "geometry exceeds the kernels' LDS limits";
        case MOJETTE_EINCONSISTENT: return "projections disagree with the image";
        case MOJETTE_ESCRATCH: return "request exceeds the library's fixed scratch memory";
        default: return "unknown status";
    }
}

int64_t mojette_proj_size(int32_t p, int32_t P, int32_t Q) {
    if (P < 1 || Q < 1) return -1;
    return (int64_t)(p < 0 ? -(int64_t)p : p) * (Q - 1) + P;
}

int64_t mojette_bin_offset(int32_t p, int32_t P, int32_t Q) {
    const int64_t m = (int64_t)(Q - 1) * p;
    return -(int64_t)(P - 1) + (m < 0 ? m : 0);
}

int64_t mojette_block_words(const int32_t *dirs, int32_t n, int32_t P, int32_t Q) {
    if (!geometry_ok(dirs, n, P, Q)) return -1;
    int64_t s = 0;
    for (int i = 0; i < n; ++i) s += mojette_proj_size(dirs[i], P, Q);
    return s;
}

int32_t mojette_decode_ring(const int32_t *dirs, int32_t n, int32_t P, int32_t Q) {
    if (!geometry_ok(dirs, n, P, Q) || n < Q) return -1;
    std::vector<int> sp(dirs, dirs + n);
    std::sort(sp.begin(), sp.end());
    return ring_length(sp, Q);
}

// One block; bin_swap: 128-bit pixels as the word image of twice the width;
// keep_first/keep_count: the stored bins of each projection (null: all).
static int encode_one_impl(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs,
                           int32_t n, uint64_t *const *proj_out, void *stream, int bin_swap,
                           const int32_t *keep_first = nullptr,
                           const int32_t *keep_count = nullptr) {
    if (!image || !proj_out || !geometry_ok(dirs, n, P, Q)) return MOJETTE_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!proj_out[i]) return MOJETTE_EINVAL;
    mj::EncodeArgs a{};
    if (!encode_tiling(dirs, n, P, Q, a)) return MOJETTE_ENOTSUP;
    a.images = image;
    a.bin_swap = bin_swap;
    for (int i = 0; i < n; ++i) {
        a.out[i] = proj_out[i];
        if (keep_first) {
            a.keep_lo[i] = keep_first[i];
            a.keep_n[i] = keep_count[i];
        }
    }
    a.proj_stride = 0;
    a.nblocks = 1;
    const int grid = (a.ntiles + a.waves - 1) / a.waves;
    clear_stale_error();
    return status_of(mj::launch_encode(a, grid, (hipStream_t)stream));
}

int mojette_encode(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                   uint64_t *const *proj_out, void *stream) {
    return encode_one_impl(image, P, Q, dirs, n, proj_out, stream, 0);
}

int mojette_encode_wide(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs,
                        int32_t n, uint64_t *const *proj_out, void *stream) {
    int32_t dirs2[kMaxDirs];
    if (!wide_geometry(dirs, n, P, Q, dirs2)) return MOJETTE_EINVAL;
    return encode_one_impl(image, 2 * P, Q, dirs2, n, proj_out, stream, 1);
}

int mojette_encode_trimmed(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs,
                           int32_t n, uint64_t *const *proj_out, void *stream) {
    int32_t f[kMaxDirs], c[kMaxDirs];
    if (!kept_layout(dirs, n, P, Q, f, c)) return MOJETTE_EINVAL;
    return encode_one_impl(image, P, Q, dirs, n, proj_out, stream, 0, f, c);
}

// keep_first/keep_count: the stored bins of each projection (null: all).
static int encode_batch_impl(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                             const int32_t *dirs, int32_t n, uint64_t *projs, void *stream,
                             int bin_swap, const int32_t *keep_first = nullptr,
                             const int32_t *keep_count = nullptr) {
    if (nblocks < 0 || !geometry_ok(dirs, n, P, Q)) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!images || !projs) return MOJETTE_EINVAL;
    mj::EncodeArgs a{};
    if (!encode_tiling(dirs, n, P, Q, a)) return MOJETTE_ENOTSUP;
    a.images = images;
    a.bin_swap = bin_swap;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        a.out[i] = projs + off;
        if (keep_first) {
            a.keep_lo[i] = keep_first[i];
            a.keep_n[i] = keep_count[i];
            off += keep_count[i];
        } else {
            off += mojette_proj_size(dirs[i], P, Q);
        }
    }
    a.proj_stride = off;
    a.nblocks = nblocks;
    const int64_t items = nblocks * a.ntiles;
    const int64_t want = (items + a.waves - 1) / a.waves;
    const int grid = (int)std::min<int64_t>(want, kEncodeGridCap);
    clear_stale_error();
    return status_of(mj::launch_encode(a, grid, (hipStream_t)stream));
}

int mojette_encode_batch(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                         const int32_t *dirs, int32_t n, uint64_t *projs, void *stream) {
    return encode_batch_impl(images, nblocks, P, Q, dirs, n, projs, stream, 0);
}

int mojette_encode_batch_wide(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                              const int32_t *dirs, int32_t n, uint64_t *projs, void *stream) {
    int32_t dirs2[kMaxDirs];
    if (nblocks < 0 || !wide_geometry(dirs, n, P, Q, dirs2)) return MOJETTE_EINVAL;
    return encode_batch_impl(images, nblocks, 2 * P, Q, dirs2, n, projs, stream, 1);
}

int32_t mojette_trimmed_path(void) { return MOJETTE_TRIMMED_PATH; }

int64_t mojette_trimmed_layout(const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                               int64_t *first, int64_t *count) {
    int32_t f[kMaxDirs], c[kMaxDirs];
    if (!kept_layout(dirs, n, P, Q, f, c)) return -1;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) {
        if (first) first[i] = f[i];
        if (count) count[i] = c[i];
        total += c[i];
    }
    return total;
}

int mojette_encode_batch_trimmed(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                                 const int32_t *dirs, int32_t n, uint64_t *projs,
                                 void *stream) {
    int32_t f[kMaxDirs], c[kMaxDirs];
    if (nblocks < 0 || !kept_layout(dirs, n, P, Q, f, c)) return MOJETTE_EINVAL;
    return encode_batch_impl(images, nblocks, P, Q, dirs, n, projs, stream, 0, f, c);
}

// The consistency verdict of a verified one-block decode: a device word per
// device (its address looked up once per device), written by the check and
// read back; verified decodes on one device take turns on it.
static __device__ int32_t verify_word[1];

static int32_t *verify_word_on_current_device() {
    static std::map<int, int32_t *> ptrs;
    int dev = 0;
    const hipError_t ge = hipGetDevice(&dev);
    if (ge != hipSuccess) {
        mj::hip_status(ge);
        return nullptr;
    }
    auto it = ptrs.find(dev);
    if (it != ptrs.end()) return it->second;
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(verify_word));
    if (e != hipSuccess || !ptr) {
        mj::hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol);
        return nullptr;
    }
    return ptrs[dev] = static_cast<int32_t *>(ptr);
}

// Recomputes every given projection from the decoded image and compares all
// its bins (the consistency check of Section 2.2); waits for the result.
static int verify_one_block(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                            const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                            const uint64_t *image, hipStream_t stream, int bin_swap,
                            const int32_t *keep_first, const int32_t *keep_count) {
    static std::mutex mu;
    std::lock_guard<std::mutex> g(mu);
    mj::VerifyArgs a{};
    if (!encode_tiling(dirs, n, P, Q, a)) return MOJETTE_ENOTSUP;
    a.bin_swap = bin_swap;
    if (keep_first)
        for (int i = 0; i < n; ++i) {
            a.keep_lo[i] = keep_first[i];
            a.keep_n[i] = keep_count[i];
        }
    uint32_t have = 0;
    for (int t = 0; t < m; ++t) {
        a.par[proj_ids[t]] = proj[t];
        have |= 1u << proj_ids[t];
    }
    a.images = image;
    a.proj_stride = 0;
    a.nblocks = 1;
    a.masks = nullptr;
    a.mask_uniform = ~have & ((1u << n) - 1u);
    int32_t *word = verify_word_on_current_device();
    if (!word) return MOJETTE_EHIP;
    a.status = word;
    const int32_t zero = 0;
    int32_t verdict = 0;
    hipError_t e = hipMemcpyAsync(word, &zero, sizeof zero, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) return mj::hip_status(e);
    const int grid = (int)std::min<int64_t>((a.ntiles + a.waves - 1) / a.waves, kEncodeGridCap);
    clear_stale_error();
    const int rc = status_of(mj::launch_verify(a, grid, stream));
    if (rc != MOJETTE_OK) return rc;
    e = hipMemcpyAsync(&verdict, word, sizeof verdict, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return mj::hip_status(e);
    return verdict;
}

// One block; bin_swap: 128-bit pixels as the word image of twice the width;
// keep_first/keep_count: the stored bins of each projection (null: all).
static int decode_one_impl(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                           const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                           uint64_t *image_out, uint32_t flags, void *stream, int bin_swap,
                           const int32_t *keep_first = nullptr,
                           const int32_t *keep_count = nullptr) {
    if (!image_out || !geometry_ok(dirs, n, P, Q) || m < 0 || m > n) return MOJETTE_EINVAL;
    if (flags & ~(uint32_t)MOJETTE_VERIFY) return MOJETTE_EINVAL;
    if (m > 0 && (!proj || !proj_ids)) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    uint32_t have = 0;
    for (int t = 0; t < m; ++t) {
        const int id = proj_ids[t];
        if (id < 0 || id >= n || ((have >> id) & 1u) || !proj[t]) return MOJETTE_EINVAL;
        have |= 1u << id;
        a.in[id] = proj[t];
    }
    if (m < Q) return MOJETTE_ENOTRECON;
    const int rc = decode_setup(dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    a.pool = nullptr;
    a.proj_stride = 0;
    a.images = image_out;
    a.img_stride = (int64_t)P * Q;
    a.masks = nullptr;
    a.mask_uniform = ~have & ((1u << n) - 1u);
    a.status = nullptr;
    a.nblocks = 1;
    a.nb = 1;   // one block: one slot
    a.bin_swap = bin_swap;
    if (keep_first)
        for (int i = 0; i < n; ++i) a.keep_lo[i] = keep_first[i];
    clear_stale_error();
    const int st = status_of(mj::launch_decode(Q, mj::kLaunchPointers, a, 1, (hipStream_t)stream));
    if (st != MOJETTE_OK || !(flags & MOJETTE_VERIFY)) return st;
    return verify_one_block(proj, proj_ids, m, dirs, n, P, Q, image_out, (hipStream_t)stream,
                            bin_swap, keep_first, keep_count);
}

int mojette_decode(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                   const int32_t *dirs, int32_t n, int32_t P, int32_t Q, uint64_t *image_out,
                   uint32_t flags, void *stream) {
    return decode_one_impl(proj, proj_ids, m, dirs, n, P, Q, image_out, flags, stream, 0);
}

int mojette_decode_wide(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                        const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                        uint64_t *image_out, uint32_t flags, void *stream) {
    int32_t dirs2[kMaxDirs];
    if (!wide_geometry(dirs, n, P, Q, dirs2)) return MOJETTE_EINVAL;
    return decode_one_impl(proj, proj_ids, m, dirs2, n, 2 * P, Q, image_out, flags, stream, 1);
}

int mojette_decode_trimmed(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                           const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                           uint64_t *image_out, uint32_t flags, void *stream) {
    int32_t f[kMaxDirs], c[kMaxDirs];
    if (!kept_layout(dirs, n, P, Q, f, c)) return MOJETTE_EINVAL;
    return decode_one_impl(proj, proj_ids, m, dirs, n, P, Q, image_out, flags, stream, 0, f, c);
}

static int decode_batch_impl(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                             int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                             uint64_t *images, int32_t *status, void *stream,
                             const int32_t *keep_first = nullptr,
                             const int32_t *keep_count = nullptr) {
    if (nblocks < 0 || !geometry_ok(dirs, n, P, Q)) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!projs || !images) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    const int rc = decode_setup(dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        a.off[i] = (int32_t)off;
        if (keep_first) {
            a.keep_lo[i] = keep_first[i];
            off += keep_count[i];
        } else {
            off += mojette_proj_size(dirs[i], P, Q);
        }
    }
    a.pool = projs;
    a.proj_stride = off;
    a.images = images;
    a.img_stride = (int64_t)P * Q;
    a.masks = erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = nblocks;
    return launch_pool_whole(a, Q, 0, (hipStream_t)stream);
}

int mojette_decode_batch(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                         int32_t P, int32_t Q, const int32_t *dirs, int32_t n, uint64_t *images,
                         int32_t *status, void *stream) {
    return decode_batch_impl(projs, erased, nblocks, P, Q, dirs, n, images, status, stream);
}

// Blocks per wavefront of the 16-byte pixel decode: the count that keeps the
// most blocks resident per compute unit (rings of 16-byte slots; at most 8
// wavefronts per CU, at most half the full slot count), the larger on ties.
static int wide_blocks(int Q, int ring_stride) {
    const int most = std::max(1, mj::decode_max_blocks_per_wave(Q) / 2);
    int best = 1;
    int64_t best_res = 0;
    for (int nb = most; nb >= 1; --nb) {
        const size_t lds = 2 * mj::decode_lds_bytes(Q, nb, ring_stride);
        if (lds > kLdsLimit) continue;
        const int64_t waves = std::min<int64_t>(8, (160 * 1024) / lds);
        if (waves * nb > best_res) {
            best_res = waves * nb;
            best = nb;
        }
    }
    return best;
}

// 128-bit pixels (Section 3.1), decoded in the 16-byte geometry itself: P
// pixels per row, directions p, rings of 16-byte slots.
int mojette_decode_batch_wide(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                              int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                              uint64_t *images, int32_t *status, void *stream) {
    int32_t dirs2[kMaxDirs];
    if (nblocks < 0 || !wide_geometry(dirs, n, P, Q, dirs2)) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!projs || !images) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    const int rc = decode_setup(dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    a.nb = wide_blocks(Q, a.ring_stride);
    if (2 * mj::decode_lds_bytes(Q, a.nb, a.ring_stride) > kLdsLimit) return MOJETTE_ENOTSUP;
    // whole-line loads for 4-row codes (measured, 4 KB (6,4) at P = 64: 4.51
    // -> 4.38 ms; 8 rows: 12.5 -> 12.9 ms, so the others load unaligned)
    a.align = Q == 4;
    int64_t off = 0;   // in 16-byte bins
    for (int i = 0; i < n; ++i) {
        a.off[i] = (int32_t)off;
        off += mojette_proj_size(dirs[i], P, Q);
    }
    // a wave's slice of the pool and of the images: 32-bit byte offsets
    if ((int64_t)a.nb * off * 16 >= ((int64_t)1 << 31) ||
        (int64_t)a.nb * P * Q * 16 >= ((int64_t)1 << 31))
        return MOJETTE_ENOTSUP;
    a.pool = projs;
    a.proj_stride = off;
    a.images = images;
    a.img_stride = (int64_t)P * Q;
    a.masks = erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = nblocks;
    const int64_t batches = (nblocks + a.nb - 1) / a.nb;
    const int grid = (int)std::min<int64_t>(batches, kDecodeGridCap);
    clear_stale_error();
    return status_of(mj::launch_decode_wide(Q, a, grid, (hipStream_t)stream));
}

int mojette_decode_batch_trimmed(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                                 int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                                 uint64_t *images, int32_t *status, void *stream) {
    int32_t f[kMaxDirs], c[kMaxDirs];
    if (nblocks < 0 || !kept_layout(dirs, n, P, Q, f, c)) return MOJETTE_EINVAL;
    return decode_batch_impl(projs, erased, nblocks, P, Q, dirs, n, images, status, stream,
                             f, c);
}

int mojette_verify_batch(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                         int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                         const uint64_t *images, int32_t *status, void *stream) {
    if (nblocks < 0 || !geometry_ok(dirs, n, P, Q) || !status) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!projs || !images) return MOJETTE_EINVAL;
    mj::VerifyArgs a{};
    if (!encode_tiling(dirs, n, P, Q, a)) return MOJETTE_ENOTSUP;
    a.images = images;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        a.par[i] = projs + off;
        off += mojette_proj_size(dirs[i], P, Q);
    }
    a.proj_stride = off;
    a.nblocks = nblocks;
    a.masks = erased;
    a.status = status;
    const int64_t items = nblocks * a.ntiles;
    const int grid = (int)std::min<int64_t>((items + a.waves - 1) / a.waves, kEncodeGridCap);
    clear_stale_error();
    return status_of(mj::launch_verify(a, grid, (hipStream_t)stream));
}

// ---- systematic code -----------------------------------------------------

static bool sys_geometry_ok(const int32_t *pdirs, int32_t m, int32_t P, int32_t Q) {
    return geometry_ok(pdirs, m, P, Q) && m <= kMaxSysParity && Q + m <= 16;
}

int64_t mojette_sys_workspace(const int32_t *pdirs, int32_t m, int32_t P, int32_t Q,
                              int64_t nblocks) {
    if (nblocks < 0 || !sys_geometry_ok(pdirs, m, P, Q)) return -1;
    return 0;   // the decode needs none
}

int mojette_encode_batch_sys(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                             const int32_t *pdirs, int32_t m, uint64_t *parity, void *stream) {
    if (!sys_geometry_ok(pdirs, m, P, Q)) return MOJETTE_EINVAL;
    return encode_batch_impl(images, nblocks, P, Q, pdirs, m, parity, stream, 0);
}

int mojette_decode_batch_sys(uint64_t *images, const uint64_t *parity, const uint16_t *erased,
                             int64_t nblocks, int32_t P, int32_t Q, const int32_t *pdirs,
                             int32_t m, uint64_t *workspace, int32_t *status, void *stream) {
    (void)workspace;   // not needed: the sweep reads the surviving lines itself
    if (nblocks < 0 || !sys_geometry_ok(pdirs, m, P, Q)) return MOJETTE_EINVAL;
    if (nblocks == 0 || !erased) return MOJETTE_OK;   // nothing lost: the lines are the data
    if (!images || !parity) return MOJETTE_EINVAL;

    // the sweep: rows = the Q lines (the lost ones swept), projections = parity
    mj::DecodeArgs a{};
    std::vector<int> order(m), sp(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return pdirs[x] < pdirs[y]; });
    for (int s = 0; s < m; ++s) {
        a.p_sorted[s] = pdirs[order[s]];
        a.id_sorted[s] = order[s];
        sp[s] = pdirs[order[s]];
    }
    static std::mutex mu;
    static std::map<RingKey, std::pair<int, int>> cache;   // ring length, lead tiles
    std::pair<int, int> rl;
    {
        std::lock_guard<std::mutex> g(mu);
        RingKey key{sp, Q};
        auto it = cache.find(key);
        if (it != cache.end()) {
            rl = it->second;
        } else {
            int lead = 0;
            const int R = ring_length_sys(sp, Q, &lead);
            rl = cache[key] = {R, lead};
        }
    }
    if (rl.first < 0) return MOJETTE_EINVAL;
    a.R = rl.first;
    a.ring_stride = mj::ring_stride_of(Q, rl.first);
    a.sys_lead = rl.second;
    // the kernels are compiled for half the slots
    a.nb = std::min(default_blocks(Q, a.ring_stride),
                    std::max(1, mj::decode_max_blocks_per_wave(Q) / 2));
    if (mj::decode_lds_bytes(Q, a.nb, a.ring_stride) > kLdsLimit) return MOJETTE_ENOTSUP;
    int64_t off = 0;
    for (int i = 0; i < m; ++i) {
        a.off[i] = (int32_t)off;
        off += mojette_proj_size(pdirs[i], P, Q);
    }
    if ((int64_t)a.nb * off * 8 >= ((int64_t)1 << 31) ||
        (int64_t)a.nb * P * Q * 8 >= ((int64_t)1 << 31))
        return MOJETTE_ENOTSUP;
    a.P = P;
    a.n = m;
    a.pool = parity;
    a.proj_stride = off;
    a.images = images;
    a.img_stride = (int64_t)P * Q;
    a.masks = erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = nblocks;
    const int64_t batches = (nblocks + a.nb - 1) / a.nb;
    const int grid = (int)std::min<int64_t>(batches, kDecodeGridCap);
    clear_stale_error();
    return status_of(mj::launch_decode_sys(Q, a, grid, (hipStream_t)stream));
}

// ---- chunked decode of long rows -------------------------------------------

struct mojette_chunk_plan {
    int32_t n, Q, tiles, max_cols, R, nsets;
    int32_t npow;            // matrices per set: T, T^2, ..., T^(2^(npow-1))
    int32_t dirs[MOJETTE_MAX_DIRS];
    // 128-bit pixels: dirs (and tiles, max_cols, R) describe the word image
    // of twice the width; dirs1 holds the caller's directions
    int32_t wide;
    int32_t dirs1[MOJETTE_MAX_DIRS];
    int32_t *lut;            // device, 2^n entries
    int32_t *state_cols;     // device, per set
    int64_t *tmat_off;       // device, per set
    uint64_t *tmat;          // device
};

static void plan_free(mojette_chunk_plan *pl) {
    if (!pl) return;
    if (pl->lut) (void)hipFree(pl->lut);
    if (pl->state_cols) (void)hipFree(pl->state_cols);
    if (pl->tmat_off) (void)hipFree(pl->tmat_off);
    if (pl->tmat) (void)hipFree(pl->tmat);
    delete pl;
}

static int chunk_plan_create_impl(const int32_t *dirs, int32_t n, int32_t Q, int32_t chunk_cols,
                                  mojette_chunk_plan **plan) {
    if (!plan) return MOJETTE_EINVAL;
    *plan = nullptr;
    if (!geometry_ok(dirs, n, 1, Q) || n < Q || chunk_cols < 1) return MOJETTE_EINVAL;
    const int TW = mj::kDecodeTile;
    const int tiles = (chunk_cols + TW - 1) / TW;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return dirs[x] < dirs[y]; });
    std::vector<int> sp(n);
    for (int i = 0; i < n; ++i) sp[i] = dirs[order[i]];
    // every Q-subset of the directions, in lexicographic order of sorted index
    std::vector<std::vector<int>> subsets;
    {
        std::vector<int> pick(Q);
        for (int i = 0; i < Q; ++i) pick[i] = i;
        while (true) {
            subsets.push_back(pick);
            int i = Q - 1;
            while (i >= 0 && pick[i] == n - Q + i) --i;
            if (i < 0) break;
            ++pick[i];
            for (int j = i + 1; j < Q; ++j) pick[j] = pick[j - 1] + 1;
        }
    }
    const size_t nsub = subsets.size();
    // powers for the parallel carry when every survivor set's state is small
    // enough; the state widths are known only after the matrices, so a first
    // pass sizes them (cheap next to the products)
    int npow = 1;
    {
        int emax = 0;
        for (size_t k = 0; k < nsub; ++k) {
            int32_t ps[MOJETTE_MAX_ROWS];
            for (int r = 0; r < Q; ++r) ps[r] = sp[subsets[k][r]];
            int E = 0;
            if (mj::chunk_state_cols(ps, Q, tiles, E)) emax = std::max(emax, E);
        }
        if (Q * emax <= mj::kScanMaxState) npow = mj::kScanPowers;
    }
    std::vector<int> Es(nsub, 0);
    std::vector<std::vector<uint64_t>> Ts(nsub);
    std::vector<char> ok(nsub, 0);
    // the matrices are independent: host threads share the subsets
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    const unsigned nth = (unsigned)std::min<size_t>(hw, (nsub + 7) / 8);
    auto work = [&](unsigned w) {
        for (size_t k = w; k < nsub; k += nth) {
            int32_t ps[MOJETTE_MAX_ROWS];
            for (int r = 0; r < Q; ++r) ps[r] = sp[subsets[k][r]];
            ok[k] = mj::chunk_transfer(ps, Q, tiles, Es[k], Ts[k]) ? 1 : 0;
            if (ok[k] && npow > 1) {
                std::vector<uint64_t> pw;
                mj::chunk_powers(Ts[k], Q * Es[k], npow, pw);
                Ts[k].swap(pw);
            }
        }
    };
    if (nth <= 1) {
        work(0);
    } else {
        std::vector<std::thread> pool;
        for (unsigned w = 0; w < nth; ++w) pool.emplace_back(work, w);
        for (auto &th : pool) th.join();
    }
    std::vector<int32_t> lut((size_t)1 << n, -1), cols;
    std::vector<int64_t> toff;
    std::vector<uint64_t> tmat;
    int max_cols = 0;
    for (size_t k = 0; k < nsub; ++k) {
        if (!ok[k]) return MOJETTE_ENOTSUP;
        uint32_t used = 0;
        for (int r = 0; r < Q; ++r) used |= 1u << order[subsets[k][r]];
        lut[used] = (int32_t)cols.size();
        cols.push_back(Es[k]);
        toff.push_back((int64_t)tmat.size());
        tmat.insert(tmat.end(), Ts[k].begin(), Ts[k].end());
        max_cols = std::max(max_cols, Es[k]);
    }
    if (Q * max_cols > mj::kCarryMaxState) return MOJETTE_ENOTSUP;
    int R = ring_length(sp, Q);
    if (R < 0) return MOJETTE_EINVAL;
    while (R < max_cols + TW) R <<= 1;   // a chunk's start state and its first tile of bins
    if (tmat.empty()) tmat.push_back(0);
    auto *pl = new (std::nothrow) mojette_chunk_plan{};
    if (!pl) return MOJETTE_ENOMEM;
    pl->n = n;
    pl->Q = Q;
    pl->tiles = tiles;
    pl->max_cols = max_cols;
    pl->R = R;
    pl->nsets = (int32_t)cols.size();
    pl->npow = npow;
    for (int i = 0; i < n; ++i) pl->dirs[i] = dirs[i];
    hipError_t e = hipSuccess;
    auto up = [&](void **dst, const void *src, size_t bytes) {
        if (e != hipSuccess) return;
        e = hipMalloc(dst, bytes);
        if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    up((void **)&pl->lut, lut.data(), lut.size() * sizeof(int32_t));
    up((void **)&pl->state_cols, cols.data(), cols.size() * sizeof(int32_t));
    up((void **)&pl->tmat_off, toff.data(), toff.size() * sizeof(int64_t));
    up((void **)&pl->tmat, tmat.data(), tmat.size() * sizeof(uint64_t));
    if (e != hipSuccess) {
        mj::hip_status(e);
        plan_free(pl);
        return MOJETTE_EHIP;
    }
    *plan = pl;
    return MOJETTE_OK;
}

int mojette_chunk_plan_create(const int32_t *dirs, int32_t n, int32_t Q, int32_t chunk_cols,
                              mojette_chunk_plan **plan) {
    return chunk_plan_create_impl(dirs, n, Q, chunk_cols, plan);
}

int mojette_chunk_plan_create_wide(const int32_t *dirs, int32_t n, int32_t Q,
                                   int32_t chunk_cols, mojette_chunk_plan **plan) {
    if (!plan) return MOJETTE_EINVAL;
    *plan = nullptr;
    int32_t dirs2[kMaxDirs];
    if (chunk_cols < 1 || chunk_cols > (1 << 29) || !wide_geometry(dirs, n, 1, Q, dirs2))
        return MOJETTE_EINVAL;
    const int rc = chunk_plan_create_impl(dirs2, n, Q, 2 * chunk_cols, plan);
    if (rc != MOJETTE_OK) return rc;
    (*plan)->wide = 1;
    for (int i = 0; i < n; ++i) (*plan)->dirs1[i] = dirs[i];
    return MOJETTE_OK;
}

int64_t mojette_chunk_matrix(const int32_t *p_sorted, int32_t Q, int32_t chunk_cols,
                             int32_t *state_cols, uint64_t *rows, int64_t cap_words) {
    if (!p_sorted || Q < 1 || Q > kMaxRows || chunk_cols < 1 || !state_cols) return -1;
    for (int r = 0; r < Q; ++r) {
        if (p_sorted[r] < -kMaxAbsP || p_sorted[r] > kMaxAbsP) return -1;
        if (r > 0 && p_sorted[r] <= p_sorted[r - 1]) return -1;
    }
    const int tiles = (chunk_cols + mj::kDecodeTile - 1) / mj::kDecodeTile;
    int E = 0;
    std::vector<uint64_t> T;
    if (!mj::chunk_transfer(p_sorted, Q, tiles, E, T)) return -2;
    *state_cols = E;
    if (rows && cap_words >= (int64_t)T.size()) std::copy(T.begin(), T.end(), rows);
    return (int64_t)T.size();
}

int mojette_chunk_plan_destroy(mojette_chunk_plan *plan) {
    plan_free(plan);
    return MOJETTE_OK;
}

static int plan_chunks(const mojette_chunk_plan *pl, int32_t P) {
    return std::max(1, (P / mj::kDecodeTile) / pl->tiles);
}

// Steps of the parallel carry over `per` chunk boundaries, or 0 when the
// sequential carry runs (one boundary, or not enough powers in the plan).
static int scan_steps(const mojette_chunk_plan *pl, int per, int64_t nblocks) {
    if (per < 2 || pl->npow < 2) return 0;
    int steps = 0;
    while ((1 << steps) < per) ++steps;
    if (steps > pl->npow) return 0;
    // The scan does about log2(per) times the sequential carry's products;
    // it pays while the blocks' sequential carries would leave the chip
    // mostly idle.  Measured with 256 blocks of 1 MB: (4,2) 0.41 against
    // 0.45 ms (scan), (8,4) 1.98 against 1.42 ms (sequential).
    const int waves = mj::carry_waves(pl->Q * pl->max_cols);
    return nblocks * waves <= kScanWaveBudget ? steps : 0;
}

int64_t mojette_decode_chunked_workspace(const mojette_chunk_plan *plan, int32_t P, int64_t nblocks) {
    if (!plan || P < 1 || P > (plan->wide ? kMaxP / 2 : kMaxP) || nblocks < 0) return -1;
    if (plan->wide) P *= 2;   // word columns
    const int nchunks = plan_chunks(plan, P);
    if (nchunks < 2) return 0;
    const int64_t one = nblocks * (nchunks - 1) * (int64_t)plan->Q * plan->max_cols;
    // The second buffer of the parallel carry is reserved whenever the plan
    // could use it, whatever nblocks is: the carry chosen for a call depends
    // on its block count, and a workspace sized for nblocks must serve every
    // call with fewer blocks (a smaller batch may take the parallel carry
    // where the larger one would not).
    return scan_steps(plan, nchunks - 1, 1) ? 2 * one : one;
}

// The three launches of a chunked decode of one geometry: `a` holds the
// geometry and buffers (pool mode, or pointer mode with slots when gathering).
static int chunked_launch(const mojette_chunk_plan *plan, int nchunks, mj::DecodeArgs &a, int Q,
                          bool gather, uint64_t *workspace, hipStream_t s) {
    a.R = std::max(a.R, plan->R);
    a.ring_stride = mj::ring_stride_of(Q, a.R);
    // chunks are plentiful: half-full waves keep the sweep's registers and
    // LDS share small
    a.nb = std::max(1, mj::decode_max_blocks_per_wave(Q) / 2);
    while (a.nb > 0 && mj::decode_lds_bytes(Q, a.nb, a.ring_stride) > kLdsLimit) --a.nb;
    if (a.nb < 1) return MOJETTE_ENOTSUP;
    if (!gather && ((int64_t)a.nb * a.proj_stride * 8 >= ((int64_t)1 << 31) ||
                    (int64_t)a.nb * a.img_stride * 8 >= ((int64_t)1 << 31)))
        return MOJETTE_ENOTSUP;
    const int steps = scan_steps(plan, nchunks - 1, a.nblocks);
    a.chunk.ws = workspace;
    a.chunk.ws_alt = steps ? workspace + a.nblocks * (nchunks - 1) * (int64_t)Q * plan->max_cols
                           : nullptr;
    a.chunk.lut = plan->lut;
    a.chunk.state_cols = plan->state_cols;
    a.chunk.tmat_off = plan->tmat_off;
    a.chunk.tmat = plan->tmat;
    a.chunk.tiles = plan->tiles;
    a.chunk.nchunks = nchunks;
    a.chunk.max_cols = plan->max_cols;
    a.chunk.npow = plan->npow;
    const int64_t items = a.nblocks * (nchunks - 1);
    const int grid = (int)std::min<int64_t>((items + a.nb - 1) / a.nb, kDecodeGridCap);
    clear_stale_error();
    int st = status_of(mj::launch_decode(Q, gather ? mj::kLaunchChunkAGather : mj::kLaunchChunkA,
                                         a, grid, s));
    if (st != MOJETTE_OK) return st;
    if (steps) {
        // parallel carry: ping-pong between the two buffers, the result
        // where the last step wrote it
        for (int k = 0; k < steps; ++k) {
            st = status_of(mj::launch_decode_scan(a, Q, k, (k & 1) ? a.chunk.ws_alt : a.chunk.ws,
                                                  (k & 1) ? a.chunk.ws : a.chunk.ws_alt, s));
            if (st != MOJETTE_OK) return st;
        }
        if (steps & 1) a.chunk.ws = a.chunk.ws_alt;
    } else if (nchunks > 2) {
        st = status_of(mj::launch_decode_carry(
            a, Q, (int)std::min<int64_t>(a.nblocks, kDecodeGridCap), s));
        if (st != MOJETTE_OK) return st;
    }
    return status_of(mj::launch_decode(Q, gather ? mj::kLaunchChunkCGather : mj::kLaunchChunkC,
                                       a, grid, s));
}

static bool plan_matches(const mojette_chunk_plan *plan, const int32_t *dirs, int32_t n, int32_t Q) {
    // jobs take 64-bit pixels only
    if (!plan || plan->wide || plan->n != n || plan->Q != Q) return false;
    for (int i = 0; i < n; ++i)
        if (plan->dirs[i] != dirs[i]) return false;
    return true;
}

// trimmed: projections in the layout without never-used bins.
static int decode_chunked_impl(const mojette_chunk_plan *plan, const uint64_t *projs,
                               const uint16_t *erased, int64_t nblocks, int32_t P,
                               uint64_t *images, int32_t *status, uint64_t *workspace,
                               void *stream, bool trimmed) {
    if (!plan || nblocks < 0 || P < 1 || P > kMaxP) return MOJETTE_EINVAL;
    const int n = plan->n, Q = plan->Q;
    if (plan->wide && (trimmed || P > kMaxP / 2)) return MOJETTE_EINVAL;
    int32_t kf[kMaxDirs], kc[kMaxDirs];
    if (trimmed && !kept_layout(plan->dirs, n, P, Q, kf, kc)) return MOJETTE_EINVAL;
    const int P1 = P;   // row length in the caller's pixels
    if (plan->wide) P *= 2;   // 128-bit pixels: the word image of twice the width
    const int nchunks = plan_chunks(plan, P);
    if (nchunks < 2) {
        if (plan->wide)
            return mojette_decode_batch_wide(projs, erased, nblocks, P1, Q, plan->dirs1, n,
                                             images, status, stream);
        return trimmed ? mojette_decode_batch_trimmed(projs, erased, nblocks, P, Q, plan->dirs, n,
                                                      images, status, stream)
                       : mojette_decode_batch(projs, erased, nblocks, P, Q, plan->dirs, n,
                                              images, status, stream);
    }
    if (!geometry_ok(plan->dirs, n, P, Q)) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!projs || !images || !workspace) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    const int rc = decode_setup(plan->dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        a.off[i] = (int32_t)off;
        if (trimmed) {
            a.keep_lo[i] = kf[i];
            off += kc[i];
        } else {
            off += mojette_proj_size(plan->dirs[i], P, Q);
        }
    }
    a.pool = projs;
    a.slots = nullptr;
    a.proj_stride = off;
    a.images = images;
    a.img_stride = (int64_t)P * Q;
    a.masks = erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = nblocks;
    a.bin_swap = plan->wide;
    return chunked_launch(plan, nchunks, a, Q, false, workspace, (hipStream_t)stream);
}

int mojette_decode_batch_chunked(const mojette_chunk_plan *plan, const uint64_t *projs,
                                 const uint16_t *erased, int64_t nblocks, int32_t P,
                                 uint64_t *images, int32_t *status, uint64_t *workspace,
                                 void *stream) {
    return decode_chunked_impl(plan, projs, erased, nblocks, P, images, status, workspace,
                               stream, false);
}

int mojette_decode_batch_chunked_trimmed(const mojette_chunk_plan *plan, const uint64_t *projs,
                                         const uint16_t *erased, int64_t nblocks, int32_t P,
                                         uint64_t *images, int32_t *status,
                                         uint64_t *workspace, void *stream) {
    return decode_chunked_impl(plan, projs, erased, nblocks, P, images, status, workspace,
                               stream, true);
}

int mojette_decode_batch_two_corner(const uint64_t *projs, const uint16_t *erased,
                                    int64_t nblocks, int32_t P, int32_t Q, const int32_t *dirs,
                                    int32_t n, uint64_t *images, int32_t *status,
                                    int32_t blocks_per_wave, void *stream) {
    if (nblocks < 0 || blocks_per_wave < 0 || !geometry_ok(dirs, n, P, Q)) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!projs || !images) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    int rc = decode_setup(dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    // the mirrored sweeps take the survivors in ascending -p: the ring
    // covers the survivor sets of the negated directions too
    std::vector<int> neg(n);
    for (int s = 0; s < n; ++s) neg[s] = -a.p_sorted[n - 1 - s];
    const int Rn = ring_length(neg, Q);
    if (Rn < 0) return MOJETTE_EINVAL;
    a.R = std::max(a.R, Rn);
    a.ring_stride = mj::ring_stride_of(Q, a.R);
    // two slots per block: the half-slot body, within the LDS share
    const int half = std::max(1, mj::decode_max_blocks_per_wave(Q) / 2);
    a.nb = blocks_per_wave > 0 ? std::min(blocks_per_wave, half) : default_blocks(Q, a.ring_stride);
    a.nb = std::min(a.nb, half);
    while (a.nb > 1 && mj::decode_lds_bytes(Q, a.nb, a.ring_stride) > kLdsLimit) --a.nb;
    if (mj::decode_lds_bytes(Q, a.nb, a.ring_stride) > kLdsLimit) return MOJETTE_ENOTSUP;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        a.off[i] = (int32_t)off;
        off += mojette_proj_size(dirs[i], P, Q);
    }
    a.pool = projs;
    a.proj_stride = off;
    a.images = images;
    a.img_stride = (int64_t)P * Q;
    a.masks = erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = nblocks;
    // a wave's slots span nb/2 + 1 blocks, addressed with 32-bit offsets
    const int64_t span = a.nb / 2 + 1;
    if (span * a.proj_stride * 8 >= ((int64_t)1 << 31) || span * a.img_stride * 8 >= ((int64_t)1 << 31))
        return MOJETTE_ENOTSUP;
    const int64_t batches = (2 * nblocks + a.nb - 1) / a.nb;
    const int grid = (int)std::min<int64_t>(batches, kDecodeGridCap);
    clear_stale_error();
    return status_of(mj::launch_decode(Q, mj::kLaunchTwoCorner, a, grid, (hipStream_t)stream));
}

int mojette_decode_batch_tuned(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                               int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                               uint64_t *images, int32_t *status, int32_t blocks_per_wave,
                               void *stream) {
    if (nblocks < 0 || blocks_per_wave < 0 || !geometry_ok(dirs, n, P, Q)) return MOJETTE_EINVAL;
    if (nblocks == 0) return MOJETTE_OK;
    if (!projs || !images) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    const int rc = decode_setup(dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        a.off[i] = (int32_t)off;
        off += mojette_proj_size(dirs[i], P, Q);
    }
    a.pool = projs;
    a.proj_stride = off;
    a.images = images;
    a.img_stride = (int64_t)P * Q;
    a.masks = erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = nblocks;
    return launch_pool_whole(a, Q, blocks_per_wave, (hipStream_t)stream);
}

// Ring stride of the main launch of launch_pool_whole for a large batch.
static int main_ring_stride(const mj::DecodeArgs &a, int Q) {
    std::vector<int> sp(a.p_sorted, a.p_sorted + a.n);
    int common = -1;
    double deep = 1;
    ring_length(sp, Q, &common, &deep);
    const int nb2 = pool_default_blocks(Q, a.ring_stride);
    const bool split =
        common > 0 && common < a.R && 1.0 - std::pow(1.0 - deep, nb2) <= 0.25;
    return split ? mj::ring_stride_of(Q, common) : a.ring_stride;
}

int32_t mojette_decode_max_blocks_per_wave(const int32_t *dirs, int32_t n, int32_t P,
                                           int32_t Q) {
    if (!geometry_ok(dirs, n, P, Q)) return -1;
    mj::DecodeArgs a{};
    if (decode_setup(dirs, n, P, Q, a) != MOJETTE_OK) return -1;
    const int rs = main_ring_stride(a, Q);
    int nb = mj::decode_max_blocks_per_wave(Q);
    while (nb > 1 && mj::decode_lds_bytes(Q, nb, rs) > kLdsLimit) --nb;
    return nb;
}

int32_t mojette_decode_default_blocks_per_wave(const int32_t *dirs, int32_t n, int32_t P,
                                               int32_t Q) {
    if (!geometry_ok(dirs, n, P, Q)) return -1;
    mj::DecodeArgs a{};
    if (decode_setup(dirs, n, P, Q, a) != MOJETTE_OK) return -1;
    return pool_default_blocks(Q, main_ring_stride(a, Q));
}

int32_t mojette_decode_batch_launches(const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                                      int64_t nblocks, int32_t blocks_per_wave, int32_t *ring,
                                      int32_t *blocks, int32_t *mode, int32_t cap) {
    if (nblocks < 1 || blocks_per_wave < 0 || cap < 0 || !geometry_ok(dirs, n, P, Q))
        return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    const int rc = decode_setup(dirs, n, P, Q, a);
    if (rc != MOJETTE_OK) return rc;
    int64_t words = 0;
    for (int i = 0; i < n; ++i) words += mojette_proj_size(dirs[i], P, Q);
    a.proj_stride = words;
    a.img_stride = (int64_t)P * Q;
    a.nblocks = nblocks;
    std::vector<mj::DecodeArgs> launches;
    const int st = plan_pool_whole(a, Q, blocks_per_wave, launches);
    if (st != MOJETTE_OK) return st;
    for (int t = 0; t < (int)launches.size() && t < cap; ++t) {
        if (ring) ring[t] = launches[t].R;
        if (blocks) blocks[t] = launches[t].nb;
        if (mode) mode[t] = launches[t].ring_mode;
    }
    return (int32_t)launches.size();
}

int mojette_classes_layout(const mojette_class *classes, int32_t nclasses, int64_t *image_words,
                           int64_t *proj_words) {
    std::vector<int64_t> bw, io, po, mo;
    int64_t it = 0, pt = 0;
    const int rc = classes_check(classes, nclasses, bw, io, po, mo, it, pt);
    if (rc != MOJETTE_OK) return rc;
    if (image_words) *image_words = it;
    if (proj_words) *proj_words = pt;
    return MOJETTE_OK;
}

// Checks jobs; returns per-job block words.
static int jobs_check(const mojette_job *jobs, int32_t njobs, std::vector<int64_t> &bw) {
    if (!jobs || njobs < 1 || njobs > mj::kMaxClasses) return MOJETTE_EINVAL;
    bw.assign(njobs, 0);
    for (int c = 0; c < njobs; ++c) {
        const mojette_job &j = jobs[c];
        if (j.nblocks < 0 || !geometry_ok(j.dirs, j.n, j.P, j.Q)) return MOJETTE_EINVAL;
        for (int i = 0; i < j.n; ++i)
            if (j.dirs[i] < -32767 || j.dirs[i] > 32767) return MOJETTE_EINVAL;
        if (j.nblocks > 0 && (!j.images || !j.projs)) return MOJETTE_EINVAL;
        bw[c] = mojette_block_words(j.dirs, j.n, j.P, j.Q);
    }
    return MOJETTE_OK;
}

// A job whose single-geometry launch has at least this many work items
// (enough to fill the chip alone) gets a launch of its own, with the
// single-geometry kernel's tiles and waves; the rest share one mixed launch.
// Measured on the mixed batch of 16 classes: the 1 MB classes encode ~3x
// faster alone than as items of the mixed launch, whose one-wavefront
// workgroups and shared LDS budget leave few wavefronts per compute unit.
constexpr int64_t kOwnEncodeItems = 8192;

int mojette_encode_jobs(const mojette_job *jobs, int32_t njobs, void *stream) {
    std::vector<int64_t> bw;
    int rc = jobs_check(jobs, njobs, bw);
    if (rc != MOJETTE_OK) return rc;
    // big jobs: a launch each
    std::vector<char> own(njobs, 0);
    for (int c = 0; c < njobs; ++c) {
        const mojette_job &j = jobs[c];
        mj::EncodeArgs a{};
        if (j.nblocks == 0 || !encode_tiling(j.dirs, j.n, j.P, j.Q, a)) continue;
        if (j.nblocks * a.ntiles < kOwnEncodeItems) continue;
        own[c] = 1;
        a.images = j.images;
        a.slots = j.slots;
        int64_t off = 0;
        for (int i = 0; i < j.n; ++i) {
            a.out[i] = j.projs + off;
            off += mojette_proj_size(j.dirs[i], j.P, j.Q);
        }
        a.proj_stride = off;
        a.nblocks = j.nblocks;
        const int64_t want = (j.nblocks * a.ntiles + a.waves - 1) / a.waves;
        const int grid = (int)std::min<int64_t>(want, kEncodeGridCap);
        clear_stale_error();
        rc = status_of(mj::launch_encode(a, grid, (hipStream_t)stream));
        if (rc != MOJETTE_OK) return rc;
    }
    // heaviest items (widest tiles x rows x directions) first
    std::vector<int> order(njobs);
    std::vector<mj::EncodeArgs> geo(njobs);
    for (int c = 0; c < njobs; ++c) {
        order[c] = c;
        const mojette_job &j = jobs[c];
        if (!encode_tiling(j.dirs, j.n, j.P, j.Q, geo[c], 1, kMixedEncodeLds, 0))
            return MOJETTE_ENOTSUP;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        const int64_t wx = (int64_t)geo[x].W * jobs[x].Q * jobs[x].n;
        const int64_t wy = (int64_t)geo[y].W * jobs[y].Q * jobs[y].n;
        return wx > wy;
    });
    mj::EncodeClassTable tab{};
    size_t lds = 0;
    int qmax = 1;
    int64_t items = 0;
    int k = 0;
    for (int oc : order) {
        const mojette_job &jb = jobs[oc];
        if (jb.nblocks == 0 || own[oc]) continue;
        mj::EncodeClass &e = tab.cls[k];
        e.images = jb.images;
        e.projs = jb.projs;
        e.slots = jb.slots;
        e.nblocks = jb.nblocks;
        e.proj_stride = (int32_t)bw[oc];
        e.P = jb.P;
        e.Q = jb.Q;
        e.n = jb.n;
        e.W = geo[oc].W;
        e.H = geo[oc].H;
        e.S = geo[oc].S;
        e.ntiles = geo[oc].ntiles;
        int32_t off = 0;
        for (int i = 0; i < jb.n; ++i) {
            e.off[i] = off;
            e.p[i] = (int16_t)jb.dirs[i];
            off += (int32_t)mojette_proj_size(jb.dirs[i], jb.P, jb.Q);
        }
        tab.first_item[k] = items;
        items += jb.nblocks * e.ntiles;
        lds = std::max(lds, mj::encode_lds_bytes(jb.Q, e.S, 1));
        qmax = std::max(qmax, (int)jb.Q);
        ++k;
    }
    if (k == 0) return MOJETTE_OK;
    tab.nclasses = k;
    tab.first_item[k] = items;
    const int grid = (int)std::min<int64_t>(items, kEncodeGridCap * mj::kEncodeWaves);
    clear_stale_error();
    return status_of(mj::launch_encode_classes(qmax, tab, lds, grid, (hipStream_t)stream));
}

// One mixed decode launch over the jobs listed in `which` (heaviest first).
static int decode_jobs_launch(const mojette_job *jobs, const std::vector<int> &which,
                              const std::vector<int64_t> &bw, bool gather, int32_t *status,
                              hipStream_t stream) {
    mj::DecodeClassTable tab{};
    size_t lds = 0;
    unsigned qmask = 0;
    int64_t items = 0;
    int k = 0;
    for (int oc : which) {
        const mojette_job &jb = jobs[oc];
        if (jb.nblocks == 0) continue;
        mj::DecodeClass &d = tab.cls[k];
        const int rc = decode_setup(jb.dirs, jb.n, jb.P, jb.Q, d);
        if (rc != MOJETTE_OK) return rc;
        // every workgroup of a mixed launch gets the LDS of its largest
        // class: long-ring classes take fewer blocks per wavefront so that
        // more wavefronts share a compute unit
        while (d.nb > 1 && mj::decode_lds_bytes(jb.Q, d.nb, d.ring_stride) > kMixedDecodeLds) --d.nb;
        d.nb = std::min(d.nb, std::max(1, mj::decode_max_blocks_per_wave(jb.Q) / 2));   // half-slot bodies
        if (!gather && ((int64_t)d.nb * bw[oc] * 8 >= ((int64_t)1 << 31) ||
                        (int64_t)d.nb * jb.P * jb.Q * 8 >= ((int64_t)1 << 31)))
            return MOJETTE_ENOTSUP;
        d.Q = jb.Q;
        d.pool = jb.projs;
        d.slots = jb.slots;
        d.images = jb.images;
        d.masks = jb.erased;
        d.status = status;
        d.nblocks = jb.nblocks;
        d.proj_stride = bw[oc];
        d.img_stride = (int64_t)jb.P * jb.Q;
        d.mask_uniform = 0;
        int32_t off = 0;
        for (int i = 0; i < jb.n; ++i) {
            d.off[i] = off;
            off += (int32_t)mojette_proj_size(jb.dirs[i], jb.P, jb.Q);
        }
        tab.first_item[k] = items;
        items += (jb.nblocks + d.nb - 1) / d.nb;
        lds = std::max(lds, mj::decode_lds_bytes(jb.Q, d.nb, d.ring_stride));
        qmask |= 1u << jb.Q;
        ++k;
    }
    if (k == 0) return MOJETTE_OK;
    tab.nclasses = k;
    tab.first_item[k] = items;
    const int grid = (int)std::min<int64_t>(items, kDecodeGridCap);
    clear_stale_error();
    return status_of(mj::launch_decode_classes(qmask, gather, tab, lds, grid, stream));
}

// A job decoded in chunks: its plan fits and its rows are long enough to cut.
static bool job_chunked(const mojette_job &j) {
    return j.plan && j.nblocks > 0 && plan_chunks(j.plan, j.P) >= 2;
}

static int decode_job_chunked(const mojette_job &j, int64_t bw, int32_t *status,
                              hipStream_t stream) {
    if (!plan_matches(j.plan, j.dirs, j.n, j.Q) || !j.workspace) return MOJETTE_EINVAL;
    mj::DecodeArgs a{};
    const int rc = decode_setup(j.dirs, j.n, j.P, j.Q, a);
    if (rc != MOJETTE_OK) return rc;
    int64_t off = 0;
    for (int i = 0; i < j.n; ++i) {
        a.off[i] = (int32_t)off;
        off += mojette_proj_size(j.dirs[i], j.P, j.Q);
    }
    a.pool = j.projs;
    a.slots = j.slots;
    a.proj_stride = bw;
    a.images = j.images;
    a.img_stride = (int64_t)j.P * j.Q;
    a.masks = j.erased;
    a.mask_uniform = 0;
    a.status = status;
    a.nblocks = j.nblocks;
    return chunked_launch(j.plan, plan_chunks(j.plan, j.P), a, j.Q, j.slots != nullptr,
                          j.workspace, stream);
}

// Merged chunked decode of up to kMaxChunkClasses jobs: one launch per phase.
// Returns MOJETTE_ENOTSUP (nothing launched) when their row counts have no
// merged kernel.
static int decode_jobs_chunked_merged(const mojette_job *jobs, const std::vector<int> &which,
                                      const std::vector<int64_t> &bw, int32_t *status,
                                      hipStream_t stream) {
    unsigned qmask = 0;
    bool gather = false;
    for (int c : which) {
        qmask |= 1u << jobs[c].Q;
        gather = gather || jobs[c].slots != nullptr;
    }
    if (!mj::decode_chunk_classes_supported(qmask, gather)) return MOJETTE_ENOTSUP;
    mj::DecodeChunkTable tab{};
    size_t lds = 0;
    int64_t items = 0, blocks = 0, pairs = 0, carry_waves = 0;
    int state = 0, k = 0, max_steps = 0;
    bool all_scan = true;
    for (int c : which) {
        const mojette_job &j = jobs[c];
        mj::DecodeChunkClass &d = tab.cls[k];
        int rc = decode_setup(j.dirs, j.n, j.P, j.Q, d);
        if (rc != MOJETTE_OK) return rc;
        const mojette_chunk_plan *pl = j.plan;
        d.R = std::max(d.R, pl->R);
        d.ring_stride = mj::ring_stride_of(j.Q, d.R);
        d.nb = std::max(1, mj::decode_max_blocks_per_wave(j.Q) / 2);
        while (d.nb > 0 && mj::decode_lds_bytes(j.Q, d.nb, d.ring_stride) > kLdsLimit) --d.nb;
        if (d.nb < 1) return MOJETTE_ENOTSUP;
        if (!gather && ((int64_t)d.nb * bw[c] * 8 >= ((int64_t)1 << 31) ||
                        (int64_t)d.nb * j.P * j.Q * 8 >= ((int64_t)1 << 31)))
            return MOJETTE_ENOTSUP;
        d.Q = j.Q;
        d.pool = j.projs;
        d.slots = j.slots;
        d.images = j.images;
        d.masks = j.erased;
        d.status = status;
        d.nblocks = j.nblocks;
        d.proj_stride = bw[c];
        d.img_stride = (int64_t)j.P * j.Q;
        d.mask_uniform = 0;
        int32_t off = 0;
        for (int i = 0; i < j.n; ++i) {
            d.off[i] = off;
            off += (int32_t)mojette_proj_size(j.dirs[i], j.P, j.Q);
        }
        const int nchunks = plan_chunks(pl, j.P);
        const int steps_j = scan_steps(pl, nchunks - 1, 1);   // the plan could scan
        d.chunk.ws = j.workspace;
        d.chunk.ws_alt = steps_j ? j.workspace + j.nblocks * (nchunks - 1) * (int64_t)j.Q *
                                                     pl->max_cols
                                 : nullptr;
        d.chunk.npow = pl->npow;
        d.chunk.lut = pl->lut;
        d.chunk.state_cols = pl->state_cols;
        d.chunk.tmat_off = pl->tmat_off;
        d.chunk.tmat = pl->tmat;
        d.chunk.tiles = pl->tiles;
        d.chunk.nchunks = nchunks;
        d.chunk.max_cols = pl->max_cols;
        tab.first_item[k] = items;
        items += (j.nblocks * (nchunks - 1) + d.nb - 1) / d.nb;
        tab.first_block[k] = blocks;
        blocks += j.nblocks;
        tab.first_pair[k] = pairs;
        pairs += j.nblocks * (nchunks - 1);
        if (nchunks > 2) {
            if (steps_j == 0) all_scan = false;
            max_steps = std::max(max_steps, steps_j);
            carry_waves += j.nblocks * mj::carry_waves(j.Q * pl->max_cols);
        }
        lds = std::max(lds, mj::decode_lds_bytes(j.Q, d.nb, d.ring_stride));
        state = std::max(state, j.Q * pl->max_cols);
        ++k;
    }
    tab.nclasses = k;
    tab.first_item[k] = items;
    tab.first_block[k] = blocks;
    tab.first_pair[k] = pairs;
    const int grid = (int)std::min<int64_t>(items, kDecodeGridCap);
    const int cgrid = (int)std::min<int64_t>(blocks, kDecodeGridCap);
    const bool regs = mj::carry_rows_in_registers(state);
    clear_stale_error();
    int st = status_of(mj::launch_decode_chunk_classes(mj::kLaunchChunkA, qmask, gather, tab, lds,
                                                       grid, mj::kWave, regs, stream));
    if (st != MOJETTE_OK) return st;
    // the parallel carry pays only while the sequential carries of all the
    // launch's blocks together would leave the chip mostly idle
    if (all_scan && max_steps > 0 && carry_waves <= kScanWaveBudget) {
        // parallel carry; classes with fewer chunks than the deepest copy
        // their entries through the extra steps, so every class ends in the
        // same buffer
        const size_t slds = ((size_t)state + 4 + (size_t)(state + 3) / 4 * 16) * sizeof(uint64_t);
        const int sgrid = (int)std::min<int64_t>(pairs, kDecodeGridCap);
        for (int s = 0; s < max_steps; ++s) {
            st = status_of(mj::launch_decode_chunk_classes(mj::kLaunchScan + s, qmask, gather, tab,
                                                           slds, sgrid,
                                                           mj::kWave * mj::carry_waves(state),
                                                           regs, stream));
            if (st != MOJETTE_OK) return st;
        }
        if (max_steps & 1)   // classes with a second buffer took part in every step
            for (int c = 0; c < k; ++c)
                if (tab.cls[c].chunk.ws_alt) tab.cls[c].chunk.ws = tab.cls[c].chunk.ws_alt;
    } else {
        st = status_of(mj::launch_decode_chunk_classes(mj::kLaunchCarry, qmask, gather, tab,
                                                       mj::carry_lds_bytes(state), cgrid,
                                                       mj::kWave * mj::carry_waves(state), regs,
                                                       stream));
        if (st != MOJETTE_OK) return st;
    }
    return status_of(mj::launch_decode_chunk_classes(mj::kLaunchChunkC, qmask, gather, tab, lds,
                                                     grid, mj::kWave, regs, stream));
}

int mojette_decode_jobs(const mojette_job *jobs, int32_t njobs, int32_t *status, void *stream) {
    std::vector<int64_t> bw;
    int rc = jobs_check(jobs, njobs, bw);
    if (rc != MOJETTE_OK) return rc;
    for (int c = 0; c < njobs; ++c)
        if (job_chunked(jobs[c]) && (!plan_matches(jobs[c].plan, jobs[c].dirs, jobs[c].n, jobs[c].Q) ||
                                     !jobs[c].workspace))
            return MOJETTE_EINVAL;
    std::vector<int> order;
    for (int c = 0; c < njobs; ++c)
        if (!job_chunked(jobs[c])) order.push_back(c);
    // longest rows (longest sweeps) first
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return jobs[x].P > jobs[y].P; });
    // chunked jobs first, longest rows first: merged launches of up to
    // kMaxChunkClasses jobs, else launches of their own
    std::vector<int> chunked;
    for (int c = 0; c < njobs; ++c)
        if (job_chunked(jobs[c])) chunked.push_back(c);
    std::stable_sort(chunked.begin(), chunked.end(),
                     [&](int x, int y) { return jobs[x].P > jobs[y].P; });
    for (size_t g = 0; g < chunked.size(); g += mj::kMaxChunkClasses) {
        std::vector<int> grp(chunked.begin() + g,
                             chunked.begin() + std::min(chunked.size(), g + mj::kMaxChunkClasses));
        rc = decode_jobs_chunked_merged(jobs, grp, bw, status, (hipStream_t)stream);
        if (rc == MOJETTE_ENOTSUP) {
            for (int c : grp) {
                rc = decode_job_chunked(jobs[c], bw[c], status, (hipStream_t)stream);
                if (rc != MOJETTE_OK) return rc;
            }
        } else if (rc != MOJETTE_OK) {
            return rc;
        }
    }
    unsigned qmask = 0;
    bool gather = false;
    for (int c : order)
        if (jobs[c].nblocks > 0) {
            qmask |= 1u << jobs[c].Q;
            gather = gather || jobs[c].slots != nullptr;
        }
    if (qmask == 0) return MOJETTE_OK;
    if (mj::decode_classes_supported(qmask, gather))
        return decode_jobs_launch(jobs, order, bw, gather, status, (hipStream_t)stream);
    // A mix of row counts without a compiled kernel: one launch per row count.
    for (int q = 1; q <= mj::kMaxRows; ++q) {
        if (!((qmask >> q) & 1u)) continue;
        if (!mj::decode_classes_supported(1u << q, gather)) return MOJETTE_ENOTSUP;
    }
    for (int q = 1; q <= mj::kMaxRows; ++q) {
        if (!((qmask >> q) & 1u)) continue;
        std::vector<int> sub;
        for (int oc : order)
            if (jobs[oc].Q == q) sub.push_back(oc);
        rc = decode_jobs_launch(jobs, sub, bw, gather, status, (hipStream_t)stream);
        if (rc != MOJETTE_OK) return rc;
    }
    return MOJETTE_OK;
}

// The pool layout of the class calls, expressed as jobs.
static int classes_to_jobs(const mojette_class *classes, int32_t nclasses, const uint64_t *images,
                           const uint64_t *projs, const uint16_t *erased,
                           std::vector<mojette_job> &jobs) {
    std::vector<int64_t> bw, io, po, mo;
    int64_t it = 0, pt = 0;
    const int rc = classes_check(classes, nclasses, bw, io, po, mo, it, pt);
    if (rc != MOJETTE_OK) return rc;
    if (it > 0 && (!images || !projs)) return MOJETTE_EINVAL;
    jobs.assign(nclasses, mojette_job{});
    for (int c = 0; c < nclasses; ++c) {
        mojette_job &j = jobs[c];
        j.P = classes[c].P;
        j.Q = classes[c].Q;
        j.n = classes[c].n;
        for (int i = 0; i < j.n; ++i) j.dirs[i] = classes[c].dirs[i];
        j.nblocks = classes[c].nblocks;
        j.images = const_cast<uint64_t *>(images) + io[c];
        j.projs = const_cast<uint64_t *>(projs) + po[c];
        j.slots = nullptr;
        j.erased = erased ? erased + mo[c] : nullptr;
    }
    return MOJETTE_OK;
}

int mojette_encode_classes(const mojette_class *classes, int32_t nclasses,
                           const uint64_t *images, uint64_t *projs, void *stream) {
    std::vector<mojette_job> jobs;
    const int rc = classes_to_jobs(classes, nclasses, images, projs, nullptr, jobs);
    if (rc != MOJETTE_OK) return rc;
    return mojette_encode_jobs(jobs.data(), nclasses, stream);
}

int mojette_decode_classes(const mojette_class *classes, int32_t nclasses,
                           const uint64_t *projs, const uint16_t *erased, uint64_t *images,
                           int32_t *status, void *stream) {
    std::vector<mojette_job> jobs;
    const int rc = classes_to_jobs(classes, nclasses, images, projs, erased, jobs);
    if (rc != MOJETTE_OK) return rc;
    return mojette_decode_jobs(jobs.data(), nclasses, status, stream);
}

// ---- plans over geometries and descriptor-driven calls -----------------------

struct mojette_plan {
    std::vector<mj::GeomDev> geoms;   // host copy of the code table
    mj::GeomDev *d_geoms;             // device
    unsigned qmask;                   // row counts of the codes
    int qmax;
    int dev;                          // device the table lives on
};

// Blocks per decode wavefront of a descriptor class: the library's choice
// for the ring (or the tuned count), within the share of LDS a workgroup of
// a mixed launch gets and the half-slot bodies the launch is compiled for.
static int desc_blocks(int Q, int ring_stride, int tuned) {
    int nb = tuned > 0 ? std::min(tuned, mj::decode_max_blocks_per_wave(Q))
                       : default_blocks(Q, ring_stride);
    while (nb > 1 && mj::decode_lds_bytes(Q, nb, ring_stride) > kMixedDecodeLds) --nb;
    return std::min(nb, std::max(1, mj::decode_max_blocks_per_wave(Q) / 2));
}


int mojette_plan_create(const mojette_geom *geoms, int32_t ngeoms, const mojette_tune *tune,
                        mojette_plan **plan) {
    if (!plan) return MOJETTE_EINVAL;
    *plan = nullptr;
    if (!geoms || ngeoms < 1 || ngeoms > 1024) return MOJETTE_EINVAL;
    std::vector<mj::GeomDev> tab(ngeoms);
    unsigned qmask = 0;
    int qmax = 0;
    for (int gi = 0; gi < ngeoms; ++gi) {
        const mojette_geom &gm = geoms[gi];
        const int Q = gm.Q, n = gm.n;
        if (!geometry_ok(gm.dirs, n, 1, Q) || n < Q) return MOJETTE_EINVAL;
        if (gm.flags != 0 && gm.flags != MOJETTE_GEOM_WIDE && gm.flags != MOJETTE_GEOM_TRIMMED)
            return MOJETTE_EINVAL;
        const mojette_tune *t = tune ? &tune[gi] : nullptr;
        mj::GeomDev &g = tab[gi];
        g = mj::GeomDev{};
        g.Q = Q;
        g.n = n;
        // 128-bit pixels: the word image of 2P columns, directions 2p
        g.pshift = gm.flags == MOJETTE_GEOM_WIDE ? 1 : 0;
        const int plim = 32767 >> g.pshift;
        int dirs[kMaxDirs];
        int maxabs = 0;
        for (int i = 0; i < n; ++i) {
            if (gm.dirs[i] < -plim || gm.dirs[i] > plim) return MOJETTE_EINVAL;
            dirs[i] = gm.dirs[i] * (1 << g.pshift);
            g.dirs[i] = dirs[i];
            g.sumabs += std::abs(dirs[i]);
            maxabs = std::max(maxabs, std::abs(dirs[i]));
        }
        // the bins each projection keeps (independent of P but for their
        // number, P + rows * |p|; the reading of kept_layout)
        for (int i = 0; i < kMaxDirs; ++i) g.keep_rows[i] = -1;
        if (gm.flags == MOJETTE_GEOM_TRIMMED) {
            if (t && t->decode_two_corner_min_P > 0) return MOJETTE_EINVAL;
            int32_t first[kMaxDirs], count[kMaxDirs];
            const int P1 = 1;
            if (!kept_layout(gm.dirs, n, P1, Q, first, count)) return MOJETTE_EINVAL;
            for (int i = 0; i < n; ++i) {
                g.keep_lo[i] = first[i];
                g.keep_rows[i] = gm.dirs[i] ? (count[i] - P1) / std::abs(gm.dirs[i]) : 0;
            }
        }
        std::vector<int> order(n);
        for (int i = 0; i < n; ++i) order[i] = i;
        std::sort(order.begin(), order.end(), [&](int x, int y) { return dirs[x] < dirs[y]; });
        std::vector<int> sp(n);
        for (int s = 0; s < n; ++s) {
            sp[s] = dirs[order[s]];
            g.p_sorted[s] = (int16_t)sp[s];
            g.id_sorted[s] = (int8_t)order[s];
        }
        // encode: tiles of at most enc_w columns beside the halo, within LDS
        g.H = (Q - 1) * maxabs;
        int pmin = 0, pmax = 0;
        for (int i = 0; i < n; ++i) {
            pmin = std::min(pmin, dirs[i]);
            pmax = std::max(pmax, dirs[i]);
        }
        g.plo = pmin;
        g.pspan = pmax - pmin;
        int w = t && t->encode_tile_cols > 0 ? t->encode_tile_cols : kEncodeTileCols;
        if (w % 64 != 0) return MOJETTE_EINVAL;
        while (w > 64 && (size_t)Q * (w + 2 * g.H) * 8 > kLdsLimit) w -= 64;
        if ((size_t)Q * (w + 2 * g.H) * 8 > kLdsLimit) return MOJETTE_ENOTSUP;
        g.enc_w = w;
        // decode: the full ring and, where a shorter ring serves most
        // survivor sets, a short-ring class for them
        int common = -1;
        double deep = 1;
        const int R = ring_length(sp, Q, &common, &deep);
        if (R < 0) return MOJETTE_EINVAL;
        const int tuned_nb = t ? t->decode_blocks_per_wave : 0;
        if (tuned_nb < 0) return MOJETTE_EINVAL;
        g.R = R;
        g.nb = desc_blocks(Q, mj::ring_stride_of(Q, R), tuned_nb);
        if (mj::decode_lds_bytes(Q, g.nb, mj::ring_stride_of(Q, R)) > kLdsLimit) return MOJETTE_ENOTSUP;
        const int split = t ? t->decode_ring_split : 0;
        if (split >= 0 && common > 0 && common < R) {
            g.R_short = common;
            g.depth_short = common - mj::kDecodeTile - 1;
            g.nb_short = desc_blocks(Q, mj::ring_stride_of(Q, common), tuned_nb);
        }
        // rows decoded from both ends: their ring covers the survivor sets
        // of the negated directions too; two slots per block
        // rows counted in words, as the descriptors' rows are classed
        g.two_min_P = t ? t->decode_two_corner_min_P : 0;
        if (g.two_min_P < 0 || g.two_min_P > (mj::kDescMaxP >> g.pshift)) return MOJETTE_EINVAL;
        g.two_min_P <<= g.pshift;
        if (g.two_min_P > 0) {
            std::vector<int> neg(n);
            for (int s = 0; s < n; ++s) neg[s] = -sp[n - 1 - s];
            const int Rn = ring_length(neg, Q);
            if (Rn < 0) return MOJETTE_EINVAL;
            g.R_two = std::max(R, Rn);
            g.nb_two = desc_blocks(Q, mj::ring_stride_of(Q, g.R_two), tuned_nb);
            if (mj::decode_lds_bytes(Q, g.nb_two, mj::ring_stride_of(Q, g.R_two)) > kLdsLimit)
                return MOJETTE_ENOTSUP;
        }
        qmask |= 1u << Q;
        qmax = std::max(qmax, Q);
    }
    auto *pl = new (std::nothrow) mojette_plan{};
    if (!pl) return MOJETTE_ENOMEM;
    pl->geoms = tab;
    pl->qmask = qmask;
    pl->qmax = qmax;
    hipError_t e = hipGetDevice(&pl->dev);
    if (e == hipSuccess) e = hipMalloc((void **)&pl->d_geoms, tab.size() * sizeof(mj::GeomDev));
    if (e == hipSuccess)
        e = hipMemcpy(pl->d_geoms, tab.data(), tab.size() * sizeof(mj::GeomDev),
                      hipMemcpyHostToDevice);
    if (e == hipSuccess && !fork_pool(pl->dev, true)) e = hipErrorOutOfMemory;
    if (e != hipSuccess) {
        mj::hip_status(e);
        if (pl->d_geoms) (void)hipFree(pl->d_geoms);
        delete pl;
        return MOJETTE_EHIP;
    }
    *plan = pl;
    return MOJETTE_OK;
}

int mojette_plan_destroy(mojette_plan *plan) {
    if (!plan) return MOJETTE_OK;
    if (plan->d_geoms) (void)hipFree(plan->d_geoms);
    delete plan;
    return MOJETTE_OK;
}

int64_t mojette_workspace_size(const mojette_plan *plan, int64_t nblocks) {
    if (!plan || nblocks < 0 || nblocks > INT32_MAX) return -1;
    return (int64_t)mj::DescWorkspace::bytes(nblocks);
}

// Checks a descriptor-driven call and fills what the bucket kernels need.
static int desc_call(const mojette_plan *plan, const mojette_block *blocks, int64_t nblocks,
                     uint64_t *pool, void *workspace, int32_t *status, bool decode,
                     mj::DescCall &c) {
    if (!plan || nblocks < 0 || nblocks > INT32_MAX) return MOJETTE_EINVAL;
    if (nblocks > 0 && (!blocks || !pool || !workspace)) return MOJETTE_EINVAL;
    if (((uintptr_t)workspace & 255) != 0) return MOJETTE_EINVAL;
    c = mj::DescCall{};
    c.desc = blocks;
    c.nblocks = nblocks;
    c.geoms = plan->d_geoms;
    c.ngeoms = (int32_t)plan->geoms.size();
    c.ws = static_cast<uint8_t *>(workspace);
    c.pool = pool;
    c.status = status;
    c.decode = decode ? 1 : 0;
    // one launch per row count: a combined kernel holds the registers of its
    // largest body (the (4,2)+(6,3)+(8,4)+(12,4) one ran at one wavefront
    // per SIMD), and launches of one row count size their LDS to it
    c.group_by_q = 1;
    return MOJETTE_OK;
}

int mojette_encode_batched(const mojette_plan *plan, const mojette_block *blocks,
                           int64_t nblocks, uint64_t *pool, void *workspace, int32_t *status,
                           void *stream) {
    mj::DescCall c;
    int rc = desc_call(plan, blocks, nblocks, pool, workspace, status, false, c);
    if (rc != MOJETTE_OK || nblocks == 0) return rc;
    const hipStream_t s = (hipStream_t)stream;
    clear_stale_error();
    if ((rc = status_of(mj::launch_desc_buckets(c, s))) != MOJETTE_OK) return rc;
    // one launch per row count: work items are (block, tile), each
    // wavefront takes a contiguous run of them; the LDS tile of a wavefront
    // fits the widest tile of the row count's codes, and workgroups hold
    // four wavefronts while their tiles take at most 48 KB
    for (int q = 1; q <= kMaxRows; ++q) {
        if (!((plan->qmask >> q) & 1u)) continue;
        // tiles of every row the same width (tile and both halos), or for 9
        // to 12 rows with register prefetch, row windows (the columns each
        // row's bins cross: 8 KB (12,4) tiles of 128 columns take 20 KB of
        // LDS instead of 29 KB, eight wavefronts per compute unit instead
        // of five)
        int tile_words = 0, max_row = 0, rw_words = 0, rw_row = 0;
        for (const mj::GeomDev &g : plan->geoms) {
            if (g.Q != q) continue;
            tile_words = std::max(tile_words, q * (g.enc_w + 2 * g.H));
            max_row = std::max(max_row, g.enc_w + 2 * g.H);
            rw_words = std::max(rw_words, mj::row_window_off(q, g.enc_w, g.pspan));
            rw_row = std::max(rw_row, g.enc_w + (q - 1) * g.pspan);
        }
        if (mj::encode_row_windows(q) && mj::encode_desc_prefetch(q, rw_row) > 0) {
            tile_words = rw_words;
            max_row = rw_row;
        }
        const int waves = (size_t)mj::kEncodeWaves * tile_words * 8 <= 48 * 1024 ? mj::kEncodeWaves : 1;
        const int64_t want_waves = std::max<int64_t>(1, std::min<int64_t>(nblocks * 8, 1 << 16));
        const int grid = (int)((want_waves + waves - 1) / waves);
        rc = status_of(mj::launch_encode_desc(q, c, q, waves, tile_words, max_row, grid, s));
        if (rc != MOJETTE_OK) return rc;
    }
    return MOJETTE_OK;
}

int mojette_decode_batched(const mojette_plan *plan, const mojette_block *blocks,
                           int64_t nblocks, uint64_t *pool, void *workspace, int32_t *status,
                           void *stream) {
    mj::DescCall c;
    int rc = desc_call(plan, blocks, nblocks, pool, workspace, status, true, c);
    if (rc != MOJETTE_OK || nblocks == 0) return rc;
    const hipStream_t s = (hipStream_t)stream;
    clear_stale_error();
    if ((rc = status_of(mj::launch_desc_buckets(c, s))) != MOJETTE_OK) return rc;
    // at most two batches per block: a grid of that many (capped) loops over them
    const int grid = (int)std::min<int64_t>(kDecodeGridCap, 2 * nblocks);
    ForkPool *fp = fork_pool(plan->dev, false);
    if (!fp) return MOJETTE_EHIP;
    std::lock_guard<std::mutex> fork_lock(fp->mu);
    // calls of fewer blocks keep their launches in order on the caller's
    // stream (serving iterations: p50/p99 at 1M requests/s 5.8/7.8 ms this
    // way against 6.2-6.3/8.6-8.9 ms forking every call)
    const bool fork = nblocks >= 16384;
    hipError_t fe = fork ? hipEventRecord(fp->fork, s) : hipSuccess;
    if (fe != hipSuccess) return mj::hip_status(fe);
    unsigned used = 0;   // fork streams that took a group
    int ngroup = 0;
    for (int two = 0; two < 2; ++two) {
        for (int q = 1; q <= kMaxRows; ++q) {
            if (!((plan->qmask >> q) & 1u)) continue;
            size_t lds = 0;
            for (const mj::GeomDev &g : plan->geoms) {
                if (g.Q != q) continue;
                if (two) {
                    if (g.two_min_P > 0)
                        lds = std::max(lds, mj::decode_lds_bytes(q, g.nb_two, mj::ring_stride_of(q, g.R_two)));
                    continue;
                }
                lds = std::max(lds, mj::decode_lds_bytes(q, g.nb, mj::ring_stride_of(q, g.R)));
                if (g.R_short > 0)
                    lds = std::max(lds, mj::decode_lds_bytes(q, g.nb_short, mj::ring_stride_of(q, g.R_short)));
            }
            if (lds == 0) continue;   // no code of this row count decodes from both ends
            const int grp = q + (two ? mj::kTwoGroup : 0);
            const int k = ngroup++ % kForkStreams;
            if (fork && !((used >> k) & 1u)) {
                fe = hipStreamWaitEvent(fp->st[k], fp->fork, 0);
                if (fe != hipSuccess) {
                    rc = mj::hip_status(fe);
                    break;
                }
                used |= 1u << k;
            }
            rc = status_of(mj::launch_decode_desc(q, two != 0, c, grp, lds, grid,
                                                  fork ? fp->st[k] : s));
            if (rc != MOJETTE_OK) break;
        }
        if (rc != MOJETTE_OK) break;
    }
    // the caller's stream continues once every group is done (also after a
    // failed launch: a captured fork must be joined)
    for (int k = 0; k < kForkStreams; ++k) {
        if (!((used >> k) & 1u)) continue;
        fe = hipEventRecord(fp->join[k], fp->st[k]);
        if (fe == hipSuccess) fe = hipStreamWaitEvent(s, fp->join[k], 0);
        if (fe != hipSuccess && rc == MOJETTE_OK) rc = mj::hip_status(fe);
    }
    return rc;
}

}  // extern "C"
