/*
 * Mojette transform oracle -- plain, slow, obviously correct CPU code.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * library; the two meet only at their C-ABI inputs and outputs.
 *
 * Paper: Pertin, Feron, Van Kempen, Parrein, "Performance evaluation of the
 * Mojette erasure code for fault-tolerant distributed hot data storage"
 * (arXiv 1504.07038).
 *
 *   Section 2.1, Eq. 1   forward transform: bin b of projection (p,q) is the
 *                        group sum of every pixel f(k,l) with b = -k*q + l*p.
 *   Section 2.1, Eq. 2   projection size B = |p|(Q-1) + |q|(P-1) + 1.
 *   Section 2.2, Eq. 3   Katz criterion: unique reconstruction iff
 *                        P <= sum|p_i| or Q <= sum|q_i|.
 *   Section 2.2          inverse by peeling: find a bin that holds a single
 *                        unknown pixel, write that pixel, subtract it from
 *                        every projection, repeat.
 *   Section 2.1          "any addition works": the group is pluggable.  The
 *                        worked figure of Section 2.1 adds modulo 6; the
 *                        erasure code of Section 3 adds with XOR.
 *
 * Conventions (readings of the paper, all stated once here):
 *   - The image has Q rows ("lines", Section 2.3) of P pixels; pixel (k,l),
 *     column k in [0,P), row l in [0,Q), is stored at image[l*P + k].
 *   - Bin b of projection (p,q) is stored at index j = b - b_min, where b_min
 *     is the smallest value of -k*q + l*p over the image (attained at one of
 *     its four corners).  Bins are in ascending b.
 *   - Group kind 0: XOR on 64-bit words (identity 0, each element its own
 *     inverse).  Group kind 1: integers modulo N, values in [0,N).
 *
 * Parity status of each function is listed in the test suite: every function
 * here is pinned by at least one check that does not re-use this code
 * (closed forms, invariants, brute-force GF(2) elimination, textbook XOR
 * parity).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOTRECON (-2)
#define ORC_ENOMEM (-4)
#define ORC_EINCONSISTENT (-5)

/* ---- the group ------------------------------------------------------ */

static uint64_t grp_add(int kind, uint64_t mod, uint64_t a, uint64_t b) {
    if (kind == 0) return a ^ b;
    /* a, b < mod: compute (a + b) mod N without overflow */
    uint64_t s = a + b;
    if (s < a || s >= mod) s -= mod;
    return s;
}

static uint64_t grp_sub(int kind, uint64_t mod, uint64_t a, uint64_t b) {
    if (kind == 0) return a ^ b;
    return (a >= b) ? (a - b) : (mod - (b - a));
}

static int grp_ok(int kind, uint64_t mod) {
    return kind == 0 || (kind == 1 && mod >= 2);
}

/* ---- geometry ------------------------------------------------------- */

static int64_t iabs64(int64_t x) { return x < 0 ? -x : x; }

/* Eq. 2: number of bins of the projection along (p,q) of a P x Q image. */
int64_t orc_proj_size(int32_t p, int32_t q, int32_t P, int32_t Q) {
    return iabs64(p) * (int64_t)(Q - 1) + iabs64(q) * (int64_t)(P - 1) + 1;
}

/* Smallest bin position b = -k*q + l*p over the image: a linear function on
 * a rectangle takes its minimum at a corner, so look at the four corners. */
int64_t orc_bin_min(int32_t p, int32_t q, int32_t P, int32_t Q) {
    int64_t best = 0; /* corner (0,0) */
    int64_t c1 = -(int64_t)(P - 1) * q;
    int64_t c2 = (int64_t)(Q - 1) * p;
    int64_t c3 = -(int64_t)(P - 1) * q + (int64_t)(Q - 1) * p;
    if (c1 < best) best = c1;
    if (c2 < best) best = c2;
    if (c3 < best) best = c3;
    return best;
}

/* Eq. 3 (Katz): 1 if P <= sum|p_i| or Q <= sum|q_i|, else 0. */
int32_t orc_katz(int32_t P, int32_t Q, const int32_t *p, const int32_t *q, int32_t I) {
    int64_t sp = 0, sq = 0;
    for (int32_t i = 0; i < I; i++) {
        sp += iabs64(p[i]);
        sq += iabs64(q[i]);
    }
    return (P <= sp || Q <= sq) ? 1 : 0;
}

/* ---- forward transform (Eq. 1) -------------------------------------- */

/*
 * proj is one flat buffer; projection i starts at proj[proj_off[i]] and has
 * orc_proj_size(p[i], q[i], P, Q) bins.  Every bin is first set to the group
 * identity, then each pixel is added to the one bin of each projection whose
 * line passes through it (the Iverson bracket of Eq. 1 selects exactly that
 * bin).
 */
int32_t orc_forward_count(int32_t kind, uint64_t mod, const uint64_t *image, int32_t P,
                          int32_t Q, const int32_t *p, const int32_t *q, int32_t n,
                          uint64_t *proj, const int64_t *proj_off, int64_t *ops);

int32_t orc_forward(int32_t kind, uint64_t mod, const uint64_t *image, int32_t P, int32_t Q,
                    const int32_t *p, const int32_t *q, int32_t n, uint64_t *proj,
                    const int64_t *proj_off) {
    return orc_forward_count(kind, mod, image, P, Q, p, q, n, proj, proj_off, NULL);
}

/*
 * Eq. 1 as orc_forward, also counting in *ops (if not NULL) the group
 * additions that combine two pixels: a pixel added to a bin that already
 * holds one.  The first pixel of a bin is a copy, so a bin of c pixels costs
 * c - 1 additions (Section 3.1: at most k - 1 XORs per bin, none at the
 * edges).
 */
int32_t orc_forward_count(int32_t kind, uint64_t mod, const uint64_t *image, int32_t P,
                          int32_t Q, const int32_t *p, const int32_t *q, int32_t n,
                          uint64_t *proj, const int64_t *proj_off, int64_t *ops) {
    if (!grp_ok(kind, mod) || P <= 0 || Q <= 0 || n < 0) return ORC_EINVAL;
    int64_t total = 0;
    for (int32_t i = 0; i < n; i++) {
        int64_t B = orc_proj_size(p[i], q[i], P, Q);
        for (int64_t j = 0; j < B; j++) proj[proj_off[i] + j] = 0;
        total += B;
    }
    unsigned char *seen = NULL;
    if (ops) {
        *ops = 0;
        seen = (unsigned char *)calloc(total > 0 ? (size_t)total : 1, 1);
        if (!seen) return ORC_ENOMEM;
    }
    for (int32_t l = 0; l < Q; l++) {
        for (int32_t k = 0; k < P; k++) {
            uint64_t f = image[(int64_t)l * P + k];
            for (int32_t i = 0; i < n; i++) {
                int64_t b = -(int64_t)k * q[i] + (int64_t)l * p[i];
                int64_t j = b - orc_bin_min(p[i], q[i], P, Q);
                uint64_t *bin = &proj[proj_off[i] + j];
                *bin = grp_add(kind, mod, *bin, f);
                if (seen) {
                    if (seen[proj_off[i] + j]) ++*ops;
                    seen[proj_off[i] + j] = 1;
                }
            }
        }
    }
    free(seen);
    return ORC_OK;
}

/* ---- inverse transform by peeling (Section 2.2) ---------------------- */

/*
 * Rebuild the image from the m projections given (any number; with Katz
 * satisfied the answer is unique, so using all of them changes nothing).
 *
 *   1. For every bin, count how many pixels its line crosses.
 *   2. Residual bins start as copies of the input bins.  Every bin whose
 *      line crosses exactly one unknown pixel is "reconstructible".
 *   3. Take a reconstructible bin, find its single unknown pixel, and set
 *      the pixel to the bin's residual (the residual is the sum of the
 *      unknown pixels on the line, here just that one).
 *   4. Subtract the new pixel from the bin of every projection whose line
 *      passes through it and lower those bins' unknown counts; bins whose
 *      count drops to one become reconstructible.
 *   5. Stop when no reconstructible bin is left.  A pixel still unknown
 *      means the projections do not determine the image (ORC_ENOTRECON).
 *      With verify set, every bin whose count reached zero must have a zero
 *      residual, otherwise the projections are not the projections of any
 *      image (ORC_EINCONSISTENT).
 *
 * ops_out (may be NULL) receives the number of group subtractions made in
 * step 4, for the operation-count checks.
 */
static int32_t inverse_impl(int32_t kind, uint64_t mod, const uint64_t *proj,
                            const int64_t *proj_off, const int32_t *p, const int32_t *q, int32_t m,
                            int32_t P, int32_t Q, const int64_t *keep_lo, const int64_t *keep_n,
                            const unsigned char *known_in, uint64_t *image, int32_t verify,
                            int64_t *ops_out) {
    if (!grp_ok(kind, mod) || P <= 0 || Q <= 0 || m < 0) return ORC_EINVAL;
    int64_t npix = (int64_t)P * Q;
    int64_t total = 0;
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1));
    if (!start) return ORC_ENOMEM;
    for (int32_t i = 0; i < m; i++) {
        start[i] = total;
        total += orc_proj_size(p[i], q[i], P, Q);
    }
    start[m] = total;

    uint64_t *resid = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(total ? total : 1));
    int32_t *count = (int32_t *)calloc((size_t)(total ? total : 1), sizeof(int32_t));
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(total ? total : 1) * 2 + 16);
    unsigned char *known = (unsigned char *)calloc((size_t)npix, 1);
    if (!resid || !count || !queue || !known) {
        free(start); free(resid); free(count); free(queue); free(known);
        return ORC_ENOMEM;
    }

    /* step 1 and 2 (without keep_lo, every bin is given; with it, only bins
     * keep_lo[i] .. keep_lo[i]+keep_n[i]-1 of projection i are, stored from
     * proj[proj_off[i]], and a missing bin never becomes reconstructible) */
    for (int32_t i = 0; i < m; i++) {
        int64_t B = start[i + 1] - start[i];
        int64_t lo = keep_lo ? keep_lo[i] : 0, nk = keep_lo ? keep_n[i] : B;
        if (lo < 0 || nk < 0 || lo + nk > B) {
            free(start); free(resid); free(count); free(queue); free(known);
            return ORC_EINVAL;
        }
        for (int64_t j = 0; j < B; j++)
            resid[start[i] + j] = (j >= lo && j < lo + nk) ? proj[proj_off[i] + j - lo] : 0;
    }
    for (int32_t l = 0; l < Q; l++)
        for (int32_t k = 0; k < P; k++)
            for (int32_t i = 0; i < m; i++) {
                int64_t b = -(int64_t)k * q[i] + (int64_t)l * p[i];
                count[start[i] + b - orc_bin_min(p[i], q[i], P, Q)] += 1;
            }
    if (keep_lo) {
        for (int32_t i = 0; i < m; i++)
            for (int64_t j = 0; j < start[i + 1] - start[i]; j++)
                if (j < keep_lo[i] || j >= keep_lo[i] + keep_n[i]) count[start[i] + j] = -(P + Q) - 1;
    }
    /* Pixels known in advance (known_in[x] set, value in image[x]) are
     * removed from every projection first, as step 4 removes a pixel it has
     * just found. */
    if (known_in) {
        for (int32_t l = 0; l < Q; l++)
            for (int32_t k = 0; k < P; k++) {
                int64_t x = (int64_t)l * P + k;
                if (!known_in[x]) continue;
                known[x] = 1;
                for (int32_t i = 0; i < m; i++) {
                    int64_t b = -(int64_t)k * q[i] + (int64_t)l * p[i];
                    int64_t t = start[i] + b - orc_bin_min(p[i], q[i], P, Q);
                    resid[t] = grp_sub(kind, mod, resid[t], image[x]);
                    count[t] -= 1;
                }
            }
    }
    /* A bin can be queued at most twice: once at start, once when its count
     * falls to one; the queue is sized for that. */
    int64_t qhead = 0, qtail = 0;
    for (int64_t t = 0; t < total; t++)
        if (count[t] == 1) queue[qtail++] = t;

    int64_t ops = 0;
    while (qhead < qtail) {
        int64_t t = queue[qhead++];
        if (count[t] != 1) continue;
        int32_t i = 0;
        while (t >= start[i + 1]) i++;
        int64_t b = (t - start[i]) + orc_bin_min(p[i], q[i], P, Q);
        /* step 3: find the single unknown pixel on line b = -k*q + l*p */
        int32_t fk = -1, fl = -1;
        for (int32_t l = 0; l < Q && fk < 0; l++) {
            int64_t num = (int64_t)l * p[i] - b; /* = k*q */
            int64_t k;
            if (q[i] == 0) {
                if (num != 0) continue;
                /* a (1,0)-type line: every column of this row */
                for (k = 0; k < P; k++)
                    if (!known[(int64_t)l * P + k]) { fk = (int32_t)k; fl = l; break; }
                continue;
            }
            if (num % q[i] != 0) continue;
            k = num / q[i];
            if (k < 0 || k >= P) continue;
            if (!known[(int64_t)l * P + k]) { fk = (int32_t)k; fl = l; }
        }
        if (fk < 0) continue; /* cannot happen while count == 1 */
        uint64_t v = resid[t];
        image[(int64_t)fl * P + fk] = v;
        known[(int64_t)fl * P + fk] = 1;
        /* step 4: back-project, i.e. remove the pixel from every projection */
        for (int32_t i2 = 0; i2 < m; i2++) {
            int64_t b2 = -(int64_t)fk * q[i2] + (int64_t)fl * p[i2];
            int64_t t2 = start[i2] + b2 - orc_bin_min(p[i2], q[i2], P, Q);
            resid[t2] = grp_sub(kind, mod, resid[t2], v);
            ops += 1;
            count[t2] -= 1;
            if (count[t2] == 1) queue[qtail++] = t2;
        }
    }

    int32_t rc = ORC_OK;
    for (int64_t x = 0; x < npix; x++)
        if (!known[x]) { rc = ORC_ENOTRECON; break; }
    if (rc == ORC_OK && verify) {
        for (int64_t t = 0; t < total; t++)
            if (count[t] == 0 && resid[t] != 0) { rc = ORC_EINCONSISTENT; break; }
    }
    if (ops_out) *ops_out = ops;
    free(start); free(resid); free(count); free(queue); free(known);
    return rc;
}

int32_t orc_inverse(int32_t kind, uint64_t mod, const uint64_t *proj, const int64_t *proj_off,
                    const int32_t *p, const int32_t *q, int32_t m, int32_t P, int32_t Q,
                    uint64_t *image, int32_t verify, int64_t *ops_out) {
    return inverse_impl(kind, mod, proj, proj_off, p, q, m, P, Q, NULL, NULL, NULL, image, verify,
                        ops_out);
}

/*
 * The same peeling when only some bins of each projection are stored: the
 * never-used bins of Section 2.3 left out.  Projection i holds bins
 * keep_lo[i] .. keep_lo[i]+keep_n[i]-1 (indices as in orc_inverse) at
 * proj[proj_off[i]]; the other bins are unknown and never used.
 */
int32_t orc_inverse_kept(int32_t kind, uint64_t mod, const uint64_t *proj, const int64_t *proj_off,
                         const int32_t *p, const int32_t *q, int32_t m, int32_t P, int32_t Q,
                         const int64_t *keep_lo, const int64_t *keep_n, uint64_t *image,
                         int32_t verify, int64_t *ops_out) {
    if (!keep_lo || !keep_n) return ORC_EINVAL;
    return inverse_impl(kind, mod, proj, proj_off, p, q, m, P, Q, keep_lo, keep_n, NULL, image,
                        verify, ops_out);
}

/*
 * The same peeling when some pixels are known in advance: known_in[x] set
 * means image[x] already holds pixel x.  The systematic code (Section 2.3
 * mentions a systematic version; data lines are stored as they are) decodes
 * lost lines this way from the surviving lines and parity projections.
 */
int32_t orc_inverse_known(int32_t kind, uint64_t mod, const uint64_t *proj,
                          const int64_t *proj_off, const int32_t *p, const int32_t *q, int32_t m,
                          int32_t P, int32_t Q, const unsigned char *known_in, uint64_t *image,
                          int32_t verify, int64_t *ops_out) {
    if (!known_in) return ORC_EINVAL;
    return inverse_impl(kind, mod, proj, proj_off, p, q, m, P, Q, NULL, NULL, known_in, image,
                        verify, ops_out);
}

/* ---- erasure-code convenience: many independent blocks --------------- */

/*
 * The code of Section 2.3 and Section 3: XOR group, q = 1 for every
 * direction, k = Q data lines per block.  These loops only call the two
 * functions above block after block; they exist so that timing the oracle
 * over many blocks does not time the Python call overhead.
 *
 *   images: nblocks x Q x P words; projs: nblocks x (sum of B_i) words,
 *   projection i of a block at offset sum_{i' < i} B_i'.
 */
int32_t orc_encode_blocks(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                          const int32_t *p, int32_t n, uint64_t *projs) {
    int32_t q[64];
    int64_t off[65];
    if (n < 0 || n > 64) return ORC_EINVAL;
    off[0] = 0;
    for (int32_t i = 0; i < n; i++) {
        q[i] = 1;
        off[i + 1] = off[i] + orc_proj_size(p[i], 1, P, Q);
    }
    for (int64_t b = 0; b < nblocks; b++) {
        int32_t rc = orc_forward(0, 0, images + b * (int64_t)P * Q, P, Q, p, q, n,
                                 projs + b * off[n], off);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}

/*
 * Decode each block from the projections whose bit is clear in erased[b]
 * (bit i set = projection i lost).  All surviving projections are used.
 */
int32_t orc_decode_blocks(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                          int32_t P, int32_t Q, const int32_t *p, int32_t n, uint64_t *images) {
    int32_t q[64], ps[64];
    int64_t off[65], offs[64];
    if (n < 0 || n > 16) return ORC_EINVAL;
    off[0] = 0;
    for (int32_t i = 0; i < n; i++) off[i + 1] = off[i] + orc_proj_size(p[i], 1, P, Q);
    for (int64_t b = 0; b < nblocks; b++) {
        int32_t m = 0;
        for (int32_t i = 0; i < n; i++) {
            if ((erased[b] >> i) & 1u) continue;
            ps[m] = p[i];
            q[m] = 1;
            offs[m] = off[i];
            m++;
        }
        int32_t rc = orc_inverse(0, 0, projs + b * off[n], offs, ps, q, m, P, Q,
                                 images + b * (int64_t)P * Q, 0, NULL);
        if (rc != ORC_OK) return rc;
    }
    return ORC_OK;
}
