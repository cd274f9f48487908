// Host-side tables of the chunked decode: for one survivor set, the state
// width E and the GF(2) transfer matrix of one interior chunk.
//
// The sweep of decode_body.h reconstructs pixel (k, r) as the bin of row r's
// projection XOR the pixels (k + (l-r) p_r, l), l != r (Section 2.2), in a
// fixed order of half-steps.  Within a chunk that lies wholly inside the
// image, the pixels it produces are therefore a GF(2)-linear function of the
// bins it reads and of the pixels produced before it; the latter are read at
// most E columns behind each row's first column of the chunk.  The state of
// a chunk boundary is those E pixels of every row (Q*E words, word r*E + e =
// pixel of row r at column (chunk start of row r) - E + e); E also covers the
// pixels of the window a row has not yet stored when the chunk begins.  The
// transfer matrix maps a chunk's start state to its end state with every bin
// zero.  It is the same for every interior chunk: columns shift uniformly.
//
// The matrix is found by running the sweep of one chunk symbolically: every
// pixel is a bit set over the Q*E start-state words, each pixel the XOR of
// the sets of the pixels it reads.
#include <algorithm>
#include <vector>

#include "mj_internal.h"

namespace mj {

// Schedule of one survivor set: A_r, row parity, first column d_r of tile 0.
static void survivor_schedule(const int32_t *ps, int Q, std::vector<int> &d,
                              std::vector<bool> &isx, int &dmin) {
    std::vector<int> A(Q);
    d.assign(Q, 0);
    isx.assign(Q, false);
    int psum = 0;
    for (int r = 0; r < Q; ++r) {
        A[r] = 2 * psum + r;
        psum += ps[r];
    }
    const int Amax = *std::max_element(A.begin(), A.end());
    const int Amin = *std::min_element(A.begin(), A.end());
    for (int r = 0; r < Q; ++r) {
        isx[r] = (r & 1) == (Amax & 1);
        d[r] = isx[r] ? -((Amax - A[r]) >> 1) : -((Amax - A[r] - 1) >> 1);
    }
    dmin = -((Amax - Amin) >> 1);
}

// State width E: the deepest read back of the sweep and the unstored window.
static int state_width(const int32_t *ps, int Q, const std::vector<int> &d) {
    constexpr int TW = kDecodeTile;
    int E = 0;
    for (int r = 0; r < Q; ++r) {
        const int lag = (-d[r] + TW - 1) / TW;
        E = std::max(E, d[r] + lag * TW);             // the unstored window
        for (int l = 0; l < Q; ++l)
            if (l != r) E = std::max(E, d[l] - d[r] - (l - r) * ps[r]);   // deepest read back
    }
    return E;
}

bool chunk_state_cols(const int32_t *ps, int Q, int tiles, int &E) {
    std::vector<int> d;
    std::vector<bool> isx;
    int dmin = 0;
    survivor_schedule(ps, Q, d, isx, dmin);
    if (tiles * kDecodeTile < -dmin) return false;
    E = state_width(ps, Q, d);
    return true;
}

bool chunk_transfer(const int32_t *ps, int Q, int tiles, int &E, std::vector<uint64_t> &T) {
    constexpr int TW = kDecodeTile;
    std::vector<int> d;
    std::vector<bool> isx;
    int dmin = 0;
    survivor_schedule(ps, Q, d, isx, dmin);
    // An interior chunk must start at column >= 0 in every row.
    if (tiles * TW < -dmin) return false;
    E = state_width(ps, Q, d);
    const int dim = Q * E;
    const int RW = (dim + 63) / 64;
    const int W = E + tiles * TW;                     // columns per row in the run
    std::vector<uint64_t> M((size_t)Q * W * (RW > 0 ? RW : 1), 0);
    auto cell = [&](int r, int x) { return &M[((size_t)r * W + x) * RW]; };
    for (int r = 0; r < Q; ++r)
        for (int e = 0; e < E; ++e) {
            const int bit = r * E + e;
            cell(r, e)[bit / 64] |= 1ull << (bit % 64);
        }
    for (int tp = 0; tp < tiles; ++tp)
        for (int i = 0; i < TW; ++i)
            for (int phase = 1; phase >= 0; --phase)   // X rows first, then Y rows
                for (int r = 0; r < Q; ++r) {
                    if ((int)isx[r] != phase) continue;
                    const int x = E + tp * TW + i;
                    const int k = tp * TW + d[r] + i;
                    uint64_t *dst = cell(r, x);
                    for (int l = 0; l < Q; ++l) {
                        if (l == r) continue;
                        const int xl = k + (l - r) * ps[r] - (d[l] - E);
                        const int done = E + tp * TW + i + ((isx[l] && phase == 0) ? 1 : 0);
                        if (xl < 0 || xl >= done) return false;   // outside the state / not yet swept
                        const uint64_t *src = cell(l, xl);
                        for (int w = 0; w < RW; ++w) dst[w] ^= src[w];
                    }
                }
    T.assign((size_t)dim * RW, 0);
    for (int r = 0; r < Q; ++r)
        for (int e = 0; e < E; ++e) {
            const uint64_t *src = cell(r, tiles * TW + e);
            std::copy(src, src + RW, &T[(size_t)(r * E + e) * RW]);
        }
    return true;
}

void chunk_powers(const std::vector<uint64_t> &T, int dim, int npow, std::vector<uint64_t> &out) {
    const int RW = (dim + 63) / 64;
    const size_t msz = (size_t)dim * RW;
    out.assign(msz * npow, 0);
    if (dim == 0 || npow == 0) return;
    std::copy(T.begin(), T.begin() + msz, out.begin());
    for (int s = 1; s < npow; ++s) {
        const uint64_t *A = &out[msz * (s - 1)];
        uint64_t *C = &out[msz * s];
        // row i of A*A: XOR of the rows j of A that row i of A selects
        for (int i = 0; i < dim; ++i) {
            uint64_t *ci = C + (size_t)i * RW;
            const uint64_t *ai = A + (size_t)i * RW;
            for (int w = 0; w < RW; ++w) {
                uint64_t bits = ai[w];
                while (bits) {
                    const int j = 64 * w + __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const uint64_t *aj = A + (size_t)j * RW;
                    for (int v = 0; v < RW; ++v) ci[v] ^= aj[v];
                }
            }
        }
    }
}

}  // namespace mj
