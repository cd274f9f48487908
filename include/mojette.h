/*
 * mojette.h -- C ABI of the MI355X (gfx950) Mojette erasure-code library.
 *
 * The Mojette erasure code of Pertin, Feron, Van Kempen and Parrein
 * (arXiv 1504.07038): the k data packets of a block are the Q = k rows of a
 * P x Q image of 64-bit pixels (Section 2.3); encoding is the forward Mojette
 * transform along n directions (p_i, q_i = 1) (Section 2.1, Eq. 1, with XOR as
 * the addition, Section 3.1); decoding rebuilds the image from any Q surviving
 * projections (Katz criterion, Section 2.2, Eq. 3) by peeling pixels along a
 * reconstruction path fixed before the sweep (Section 2.2).
 *
 * Conventions shared by every call:
 *   - Pixel (k, l), column k in [0, P), row l in [0, Q), of a block is word
 *     l*P + k of the block's image (row l = data packet l).
 *   - Directions are given by their p values only (q = 1 for all, as the code
 *     of Section 2.3 fixes); they must be distinct.  n <= 16, 1 <= Q <= 16.
 *   - Projection i has B_i = |p_i|(Q-1) + P bins (Eq. 2 with q = 1); bin b
 *     (the line b = -k + l*p_i of Eq. 1) is stored at index b - b_min(p_i),
 *     b_min(p) = -(P-1) + min(0, (Q-1)p), in ascending b.
 *   - In a batch pool, the n projections of a block are contiguous, projection
 *     i at word offset sum_{i' < i} B_i' of the block's slice; the slice is
 *     mojette_block_words() long and block b's slice starts at b times that.
 *   - Pixel and bin buffers are DEVICE pointers owned by the caller; small
 *     host arrays (dirs, pointer tables, ids) are read before the call
 *     returns.  No call allocates or frees device memory except the plan
 *     calls of the chunked decode.  Images must not overlap projections.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the default stream)
 *     and the call returns without waiting.  Argument errors are reported
 *     before anything is enqueued; a failed launch returns MOJETTE_EHIP.
 *   - The batch calls allocate nothing and never synchronise, so they may be
 *     recorded into a HIP graph.
 *   - Calls on distinct streams may run concurrently.
 */
#ifndef MOJETTE_H
#define MOJETTE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MOJETTE_OK 0
#define MOJETTE_EINVAL (-1)        /* bad argument */
#define MOJETTE_ENOTRECON (-2)     /* fewer than Q projections survive (Eq. 3) */
#define MOJETTE_EHIP (-3)          /* a HIP runtime call failed */
#define MOJETTE_ENOMEM (-4)        /* host-side bookkeeping could not allocate */
#define MOJETTE_EINCONSISTENT (-5) /* projections that no image has (mojette_verify_batch) */
#define MOJETTE_ENOTSUP (-6)       /* geometry beyond the kernels' LDS limits */
#define MOJETTE_ESCRATCH (-7)      /* beyond the fixed scratch memory (..._noalloc call) */

#define MOJETTE_MAX_DIRS 16
#define MOJETTE_MAX_ROWS 16

/* Human-readable name of a status code. */
const char *mojette_strerror(int status);

/* Name of the HIP error behind the calling thread's most recent
 * MOJETTE_EHIP ("no HIP error" if there was none).  A call clears any error
 * an earlier HIP call of the thread left pending before it launches, so
 * MOJETTE_EHIP always reports the library's own launch.  The string is
 * static; the call never fails. */
const char *mojette_last_hip_error(void);

/* Eq. 2 with q = 1: number of bins of the projection along (p, 1) of a
 * P x Q image, |p|(Q-1) + P.  Returns -1 if P < 1 or Q < 1. */
int64_t mojette_proj_size(int32_t p, int32_t P, int32_t Q);

/* Smallest line position b = -k + l*p over a P x Q image (Eq. 1): bin b is
 * stored at index b - mojette_bin_offset(p, P, Q). */
int64_t mojette_bin_offset(int32_t p, int32_t P, int32_t Q);

/* Words of projection data per block: sum over the n directions of B_i.
 * Returns -1 on bad arguments. */
int64_t mojette_block_words(const int32_t *dirs, int32_t n, int32_t P, int32_t Q);

/*
 * Forward transform of ONE block (Section 2.1, Eq. 1; encoding, Section 2.3).
 *   image     device, Q*P words, row-major.
 *   dirs      host, n distinct p values.
 *   proj_out  host array of n device pointers; proj_out[i] receives the B_i
 *             bins of direction dirs[i].
 * Returns MOJETTE_OK, MOJETTE_EINVAL, MOJETTE_ENOTSUP or MOJETTE_EHIP.
 */
int mojette_encode(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                   uint64_t *const *proj_out, void *stream);

/*
 * Inverse transform of ONE block (Section 2.2).
 *   proj      host array of m device pointers; proj[t] holds the full B bins
 *             of direction dirs[proj_ids[t]].
 *   proj_ids  host, m distinct indices into dirs.
 *   dirs, n   the code's directions, as given to mojette_encode.
 *   image_out device, Q*P words.
 *   flags     0 or MOJETTE_VERIFY.  With MOJETTE_VERIFY the call checks
 *             consistency (Section 2.2: projections that are not the
 *             projections of any image leave bins with a nonzero residue):
 *             every given projection, all of its Eq. 2 bins, is recomputed
 *             from the decoded image and compared; the call then waits for
 *             the result (it is synchronous, not for graph capture) and
 *             returns MOJETTE_EINCONSISTENT on any difference.  Verified
 *             decodes on one device take turns on a device word of the
 *             library's.
 * m >= Q is required (Katz with q_i = 1: any Q of the n projections
 * reconstruct, Section 2.3); with m > Q the Q survivors of smallest p are
 * used.  Returns MOJETTE_OK, MOJETTE_EINVAL, MOJETTE_ENOTRECON,
 * MOJETTE_ENOTSUP, MOJETTE_EHIP or (verified) MOJETTE_EINCONSISTENT.
 */
#define MOJETTE_VERIFY 1u
int mojette_decode(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                   const int32_t *dirs, int32_t n, int32_t P, int32_t Q, uint64_t *image_out,
                   uint32_t flags, void *stream);

/*
 * Forward transform of nblocks blocks of one geometry in one launch.
 *   images  device, nblocks x Q x P words (block b at b*Q*P).
 *   projs   device, nblocks x mojette_block_words() words (layout above).
 * nblocks == 0 is a no-op.  Returns as mojette_encode.
 */
int mojette_encode_batch(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                         const int32_t *dirs, int32_t n, uint64_t *projs, void *stream);

/*
 * Inverse transform of nblocks blocks of one geometry in one launch (two
 * for large batches whose survivor sets need rings of two lengths: the
 * deep sets then decode on a stream of the library's, forked from `stream`
 * and joined back to it, so ordering on `stream` is as for one launch; under
 * graph capture that stream must have been made by an earlier call or plan
 * on the device, else the two launches run in order on `stream`).
 *   projs    device, pool laid out as for mojette_encode_batch.  Bins of
 *            erased projections are never read.
 *   erased   device, nblocks uint16 masks; bit i set = projection i of that
 *            block is lost.  NULL means no erasures.
 *   images   device, nblocks x Q x P words, written for every decodable
 *            block.
 *   status   device int32 or NULL.  A block with fewer than Q survivors is
 *            left unwritten and MOJETTE_ENOTRECON is stored to *status; the
 *            call never clears *status, so the caller sets it to 0 first.
 * Returns as mojette_decode (argument errors only; per-block survivor
 * shortfalls are reported through status).
 */
int mojette_decode_batch(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                         int32_t P, int32_t Q, const int32_t *dirs, int32_t n, uint64_t *images,
                         int32_t *status, void *stream);

/*
 * Consistency check of decoded blocks (the peeling of Section 2.2 detects
 * projections that are not the projections of any image: a bin left with a
 * nonzero residue once every pixel on its line is known).  For every block,
 * every projection whose bit is clear in erased[b] is recomputed from the
 * block's image (Eq. 1) and compared bin by bin, all of Eq. 2's bins, with
 * the stored one; any difference stores MOJETTE_EINCONSISTENT to *status
 * (device int32, required; the call never clears it).  With the image from
 * mojette_decode_batch on the same masks, a clean *status means every
 * surviving projection is exactly the projection of the decoded image.  A
 * single corrupted bin is always caught once two projections survive: the
 * bins of each projection XOR to the XOR of all pixels.  Arguments as for
 * mojette_decode_batch; nothing is written but *status.
 */
int mojette_verify_batch(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                         int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                         const uint64_t *images, int32_t *status, void *stream);

/*
 * 128-bit pixels and bins (Section 3.1 sets pixel and bin to 128 bits for
 * the XOR code): the same two calls for blocks of P x Q pixels of 16 bytes.
 *   images  device, nblocks x Q x P pixels, each pixel two 64-bit words
 *           (block b at word 2*b*Q*P, pixel (k,l) at words 2*(l*P+k) and
 *           2*(l*P+k)+1).
 *   projs   device, nblocks x 2*mojette_block_words(dirs, n, P, Q) words:
 *           projection i of a block holds mojette_proj_size(dirs[i], P, Q)
 *           bins of two words each, bin j's words in the order of a
 *           pixel's (bin j is the XOR of its line's pixels, word by word).
 *   erased, status  as for mojette_decode_batch.
 * P may be up to 2^23 and |p| up to 2^15.  Returns as the 64-bit calls.
 */
int mojette_encode_batch_wide(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                              const int32_t *dirs, int32_t n, uint64_t *projs, void *stream);
int mojette_decode_batch_wide(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                              int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                              uint64_t *images, int32_t *status, void *stream);

/*
 * ONE block of 128-bit pixels (Section 3.1): mojette_encode and
 * mojette_decode for a P x Q image of 16-byte pixels.
 *   image, image_out  device, Q*P pixels of two words (pixel (k,l) at words
 *                     2*(l*P+k) and 2*(l*P+k)+1).
 *   proj_out[i], proj[t]  device, 2*mojette_proj_size(p, P, Q) words: the
 *                     bins of that direction, two words each, bin j's words
 *                     in the order of a pixel's.
 * Other arguments, flags (MOJETTE_VERIFY) and return codes as for the 64-bit
 * one-block calls; P may be up to 2^23 and |p| up to 2^15.
 */
int mojette_encode_wide(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs,
                        int32_t n, uint64_t *const *proj_out, void *stream);
int mojette_decode_wide(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                        const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                        uint64_t *image_out, uint32_t flags, void *stream);

/*
 * Never-used bins left out (Section 2.3 notes that some bins are used by no
 * reconstruction, whatever the projections at hand).  For this library's
 * reconstruction path (of the survivors the Q with the smallest p are used,
 * the r-th rebuilding image row r from its bins r*p - k, k = 0..P-1) the
 * projection whose p has rank i among the sorted directions keeps the bins
 * it can be read from, r = max(0, i - (n - Q)) .. min(i, Q - 1): P +
 * (r_hi - r_lo)*|p| consecutive bins instead of Eq. 2's |p|(Q-1) + P.
 *
 * mojette_trimmed_layout: words per block of the trimmed layout (the kept
 *   bins of projection 0, then of projection 1, ...), or -1 on bad
 *   arguments (including n < Q).  first[i] (may be NULL) receives the index
 *   (b - b_min, as in the full projection) of projection i's first kept
 *   bin, count[i] (may be NULL) their number; both host arrays of n.
 * mojette_encode_batch_trimmed / mojette_decode_batch_trimmed: as the
 *   batched calls, projections in the trimmed layout (block b's slice at
 *   word b * mojette_trimmed_layout()).
 * mojette_encode_trimmed / mojette_decode_trimmed: as the one-block calls
 *   mojette_encode / mojette_decode (flags: MOJETTE_VERIFY, which then
 *   compares the kept bins), each projection buffer holding count[i] words:
 *   its kept bins, from index first[i] on.
 *
 * The layout is tied to the reconstruction path above: another decoder
 * (another assignment of projections to rows) may need bins it leaves out.
 * mojette_trimmed_path returns MOJETTE_TRIMMED_PATH, the number of that path
 * in this library; a store keeps it beside a trimmed pool and reads the pool
 * back only with a library that returns the same number.
 */
#define MOJETTE_TRIMMED_PATH 1
int32_t mojette_trimmed_path(void);
int64_t mojette_trimmed_layout(const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                               int64_t *first, int64_t *count);
int mojette_encode_batch_trimmed(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                                 const int32_t *dirs, int32_t n, uint64_t *projs, void *stream);
int mojette_decode_batch_trimmed(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                                 int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                                 uint64_t *images, int32_t *status, void *stream);
int mojette_encode_trimmed(const uint64_t *image, int32_t P, int32_t Q, const int32_t *dirs,
                           int32_t n, uint64_t *const *proj_out, void *stream);
int mojette_decode_trimmed(const uint64_t *const *proj, const int32_t *proj_ids, int32_t m,
                           const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                           uint64_t *image_out, uint32_t flags, void *stream);

/*
 * Systematic code (Section 2.3 mentions a systematic version of the code as
 * under development and gives no construction; this is the one used here).
 * A block's Q data lines are stored as they are (the image, Q x P words),
 * and m parity projections along (p, 1), p = pdirs[0..m-1], beside them
 * (the layout of mojette_encode_batch with n = m).  Packet i < Q is data
 * line i, packet Q + j parity projection j; Q + m <= 16, 1 <= m <= 8.
 *
 * mojette_encode_batch_sys: computes the parity pool from the images (the
 *   data lines need no encoding).  Returns as mojette_encode_batch.
 * mojette_decode_batch_sys: rebuilds, in place in `images`, every lost line
 *   of every block; surviving lines are read and never written, and a block
 *   that lost no line is not touched (its read is the lines themselves).
 *   Lost lines are rebuilt from the surviving parity projections and the
 *   surviving lines, peeled in the order of Section 2.2 (the r-th lost line
 *   from the r-th surviving projection in ascending p; the surviving lines'
 *   pixels on a bin's line are read from `images` as the sweep goes).
 *     images     device, nblocks x Q x P words, in/out.
 *     parity     device, the parity pool, read only.
 *     erased     device, nblocks uint16 masks (bit i = packet i lost); NULL
 *                means nothing lost (no-op).
 *     workspace  unused (the decode needs none; may be NULL).
 *     status     as for mojette_decode_batch: a block that lost more lines
 *                than it has surviving parity projections is left as it is
 *                and MOJETTE_ENOTRECON is stored.
 * mojette_sys_workspace: words of workspace for nblocks blocks (0), -1 on
 *   bad arguments.
 */
int mojette_encode_batch_sys(const uint64_t *images, int64_t nblocks, int32_t P, int32_t Q,
                             const int32_t *pdirs, int32_t m, uint64_t *parity, void *stream);
int64_t mojette_sys_workspace(const int32_t *pdirs, int32_t m, int32_t P, int32_t Q,
                              int64_t nblocks);
int mojette_decode_batch_sys(uint64_t *images, const uint64_t *parity, const uint16_t *erased,
                             int64_t nblocks, int32_t P, int32_t Q, const int32_t *pdirs,
                             int32_t m, uint64_t *workspace, int32_t *status, void *stream);

/*
 * mojette_decode_batch with the decode schedule's blocks per wavefront set by
 * the caller (an autotuner): blocks_per_wave >= 1 asks for that many (capped
 * by what fits in LDS), 0 keeps the library's choice.  Fewer blocks per
 * wavefront spread a small batch over more compute units and leave LDS for
 * more wavefronts per unit; more give each wavefront more independent work.
 */
int mojette_decode_batch_tuned(const uint64_t *projs, const uint16_t *erased, int64_t nblocks,
                               int32_t P, int32_t Q, const int32_t *dirs, int32_t n,
                               uint64_t *images, int32_t *status, int32_t blocks_per_wave,
                               void *stream);

/*
 * mojette_decode_batch with a shallower reconstruction path (Section 2.2:
 * the path is fixed in advance and may propagate from the corners of the
 * image toward its center).  Every block is swept from both ends at once:
 * from column 0 as in mojette_decode_batch, and from column P-1 as the same
 * sweep of the column-mirrored block (whose projections are those along
 * (-p, 1), bins in reverse order; its rows take the survivors in ascending
 * -p).  Each sweep stops once every row has reached the middle column, so
 * a block's dependency chain is about half as deep (about P half-steps
 * instead of 2P); the work is the same, plus the columns both sweeps reach.
 * Results are bit-identical to mojette_decode_batch.  blocks_per_wave as for
 * mojette_decode_batch_tuned (two slots per block).  Arguments, layouts and
 * errors as for mojette_decode_batch.
 */
int mojette_decode_batch_two_corner(const uint64_t *projs, const uint16_t *erased,
                                    int64_t nblocks, int32_t P, int32_t Q, const int32_t *dirs,
                                    int32_t n, uint64_t *images, int32_t *status,
                                    int32_t blocks_per_wave, void *stream);

/* Blocks per decode wavefront for this geometry: the most that fit in LDS,
 * and the library's own choice for mojette_decode_batch (all the lanes
 * allow when their rings take at most 34 KB of LDS, else at most half of
 * them within 26 KB; for 4-row codes with 32-word rings at most half, the
 * body that loads whole lines).  Both use the ring of the launch that sweeps most
 * blocks: the shorter ring when a large batch is decoded in two ring
 * classes.  -1 on bad arguments. */
int32_t mojette_decode_max_blocks_per_wave(const int32_t *dirs, int32_t n, int32_t P, int32_t Q);
int32_t mojette_decode_default_blocks_per_wave(const int32_t *dirs, int32_t n, int32_t P,
                                               int32_t Q);

/* The launches mojette_decode_batch_tuned makes for nblocks blocks of this
 * geometry (blocks_per_wave as there; 0 is mojette_decode_batch's own
 * choice), computed on the host without launching anything.  Returns their
 * number (1, or 2 when a large batch is split into ring classes) or a
 * negative status (MOJETTE_EINVAL; MOJETTE_ENOTSUP when a wavefront's slice
 * of the pools is beyond 32-bit byte offsets).  For launch t < cap, ring[t]
 * receives its ring length in words, blocks[t] its blocks per wavefront and
 * mode[t] what it sweeps: 0 every block, 1 the blocks whose survivor set
 * fits the short ring, 2 the others (gathered from ranges of 256 blocks,
 * which the split needs to address with 32-bit offsets; otherwise the batch
 * is decoded in one launch).  Host arrays of cap entries, each may be NULL. */
int32_t mojette_decode_batch_launches(const int32_t *dirs, int32_t n, int32_t P, int32_t Q,
                                      int64_t nblocks, int32_t blocks_per_wave, int32_t *ring,
                                      int32_t *blocks, int32_t *mode, int32_t cap);

/*
 * Mixed batches: blocks of up to MOJETTE_MAX_CLASSES geometry classes (each
 * class: nblocks blocks of one P, Q and direction set) encoded or decoded in
 * ONE launch.  Classes are laid out one after another in each pool, in the
 * order given: class c's images start at word sum_{c'<c} nblocks*P*Q of the
 * image pool, its projection slices (layout as for mojette_encode_batch) at
 * word sum_{c'<c} nblocks*block_words of the projection pool, and its erasure
 * masks at entry sum_{c'<c} nblocks of the mask array.  The launch walks the
 * classes' work heaviest first (largest rows first) so that long items start
 * early.  Directions must satisfy |p| <= 32767.  Same ownership, error and
 * stream rules as the batch calls; safe to record into a HIP graph.
 */
#define MOJETTE_MAX_CLASSES 16

typedef struct mojette_class {
    int32_t P;                        /* pixels per row */
    int32_t Q;                        /* rows = data packets, 1..16 */
    int32_t n;                        /* projections, Q..16 */
    int32_t dirs[MOJETTE_MAX_DIRS];   /* p of each projection (q = 1), distinct */
    int64_t nblocks;                  /* blocks of this class, >= 0 */
} mojette_class;

/* Pool sizes of a mixed batch: *image_words and *proj_words receive the total
 * words of the image and projection pools.  Returns MOJETTE_OK or
 * MOJETTE_EINVAL. */
int mojette_classes_layout(const mojette_class *classes, int32_t nclasses, int64_t *image_words,
                           int64_t *proj_words);

/* Forward transform (Section 2.1, Eq. 1) of every block of every class. */
int mojette_encode_classes(const mojette_class *classes, int32_t nclasses,
                           const uint64_t *images, uint64_t *projs, void *stream);

/* Inverse transform (Section 2.2) of every block of every class; erased,
 * images and status as for mojette_decode_batch (erased may be NULL). */
int mojette_decode_classes(const mojette_class *classes, int32_t nclasses,
                           const uint64_t *projs, const uint16_t *erased, uint64_t *images,
                           int32_t *status, void *stream);

/*
 * Jobs: the general form of a mixed batch, for callers that keep projections
 * at scattered slots (an object store).  A job is one geometry class with its
 * own device buffers:
 *   images   nblocks images back to back (encode reads them, decode writes).
 *   projs    a region of projection slices, each mojette_block_words() long.
 *   slots    device int64 array or NULL: block b's slice is slice slots[b] of
 *            projs (NULL: slice b).  Encode scatters to the slots, decode
 *            gathers from them.
 *   erased   decode: device uint16 masks, one per block, or NULL.
 * Up to MOJETTE_MAX_CLASSES jobs run in one launch.  Decode launches with any
 * `slots` support row counts 2, 4, ..., 16 alone and the {4, 8} mix
 * (MOJETTE_ENOTSUP otherwise); chunked jobs take any row count.  Same ownership, error and stream rules as the
 * batch calls; safe to record into a HIP graph.
 */
typedef struct mojette_chunk_plan mojette_chunk_plan;   /* chunked decode, see below */

typedef struct mojette_job {
    int32_t P, Q, n;
    int32_t dirs[MOJETTE_MAX_DIRS];
    int64_t nblocks;
    uint64_t *images;
    uint64_t *projs;
    const int64_t *slots;
    const uint16_t *erased;
    /* decode only, optional: with a plan for this code (same dirs and Q) and
     * rows long enough to cut, the job's blocks are decoded in chunks (see
     * mojette_decode_batch_chunked) in launches of their own on the same
     * stream, using `workspace` (mojette_decode_chunked_workspace() words). */
    const mojette_chunk_plan *plan;
    uint64_t *workspace;
} mojette_job;

/* Forward transform (Section 2.1, Eq. 1) of every block of every job. */
int mojette_encode_jobs(const mojette_job *jobs, int32_t njobs, void *stream);

/* Inverse transform (Section 2.2) of every block of every job; status as for
 * mojette_decode_batch. */
int mojette_decode_jobs(const mojette_job *jobs, int32_t njobs, int32_t *status, void *stream);

/*
 * Descriptor-driven batched calls: any number of blocks, each with its own
 * code and row length, in one call.  A plan holds the codes (geometries:
 * Q = k data lines, n projections along (p_i, 1), Section 2.3) and, per
 * code, the schedule of its launches.  Each block is described by a device
 * descriptor (mojette_block) that names its code (geom_id), its row length
 * P, its erasure mask and where its image and its projections sit in one
 * device word pool: the image is Q x P words from image_off (row-major, row l
 * = data packet l), the n projections are back to back from proj_off
 * (projection i, mojette_proj_size(dirs[i], P, Q) bins, at proj_off +
 * sum_{i' < i} B_i').  Blocks may come in any order and interleave codes and
 * row lengths.
 *
 * A call first groups the blocks by (code, P) on the device, in the caller's
 * workspace (mojette_workspace_size bytes), then runs the transform of every
 * block in one persistent launch per row count Q among the plan's codes,
 * longest rows first.  Calls allocate nothing,
 * never synchronise and are safe to record into a HIP graph.  At most 2,048
 * distinct (geom_id, P) pairs per call; the blocks of pairs beyond that are
 * not transformed and MOJETTE_ENOTSUP is stored to *status.
 */
/* Layout options of a code (mojette_geom.flags), one at most:
 * MOJETTE_GEOM_WIDE     128-bit pixels and bins (Section 3.1), as the _wide
 *                       batch calls lay them out: a block's P counts 16-byte
 *                       pixels, its image is Q x 2P words (pixel k of a row
 *                       at words 2k, 2k+1, low word first), projection i
 *                       holds mojette_proj_size(dirs[i], P, Q) 16-byte bins
 *                       (twice as many words); image_off and proj_off still
 *                       count words.  2P <= 2^24, |p| <= 16383.
 * MOJETTE_GEOM_TRIMMED  never-used bins left out (Section 2.3), as the
 *                       _trimmed batch calls lay them out: projection i
 *                       holds only its kept bins (mojette_trimmed_layout),
 *                       the projections back to back.  Tied to this
 *                       library's reconstruction path (MOJETTE_TRIMMED_PATH);
 *                       not with decode_two_corner_min_P. */
#define MOJETTE_GEOM_WIDE 1u
#define MOJETTE_GEOM_TRIMMED 2u

typedef struct mojette_geom {
    int32_t Q;                        /* rows = data packets, 1..16 */
    int32_t n;                        /* projections, Q..16 */
    int32_t dirs[MOJETTE_MAX_DIRS];   /* p of each projection (q = 1), distinct, |p| <= 32767 */
    uint32_t flags;                   /* 0 or one MOJETTE_GEOM_* layout option */
} mojette_geom;

/* Schedule of one code (zero fields: the library's choice).  An autotuner
 * fills these from measurements. */
typedef struct mojette_tune {
    int32_t decode_blocks_per_wave;   /* blocks swept by one decode wavefront (>= 1) */
    int32_t decode_ring_split;        /* 1: survivor sets that read shallowly get a short ring and
                                         more blocks per wavefront (their own classes); -1: never;
                                         0: the library's choice (split where 90% of sets fit) */
    int32_t encode_tile_cols;         /* encode tile width cap, a multiple of 64 */
    int32_t decode_two_corner_min_P;  /* blocks of at least this row length are decoded from
                                         both ends (mojette_decode_batch_two_corner); 0: none */
} mojette_tune;

/* A block of a descriptor-driven call (device memory, 24 bytes). */
typedef struct mojette_block {
    uint64_t image_off;               /* word offset of the block's image in the pool */
    uint64_t proj_off;                /* word offset of its first projection in the pool */
    uint32_t P;                       /* pixels per row, 1..2^24 with P*Q <= 2^30 */
    uint16_t geom_id;                 /* index into the plan's codes */
    uint16_t erasure_mask;            /* decode: bit i set = projection i lost */
} mojette_block;

typedef struct mojette_plan mojette_plan;

/* Creates a plan over ngeoms codes (1..1024).  tune: NULL or ngeoms entries.
 * Checks every code (EINVAL: bad Q, n, duplicate or out-of-range
 * directions, unknown or combined flags, a trimmed code asked to decode
 * from both ends; ENOTSUP: beyond the kernels' LDS limits), computes each
 * code's decode rings on the host and copies the code table to the current
 * device: it allocates device memory and synchronises, so it is not for
 * use under graph capture.  The plan is used on that device only. */
int mojette_plan_create(const mojette_geom *geoms, int32_t ngeoms, const mojette_tune *tune,
                        mojette_plan **plan);
/* Frees the plan (NULL is a no-op). */
int mojette_plan_destroy(mojette_plan *plan);

/* Workspace bytes a call on up to nblocks blocks needs (non-decreasing in
 * nblocks), or -1 on bad arguments.  About 1.7 MB plus 12 bytes per block. */
int64_t mojette_workspace_size(const mojette_plan *plan, int64_t nblocks);

/* Forward transform (Section 2.1, Eq. 1) of every described block: reads
 * each block's image, writes its n projections.  blocks: device, nblocks
 * descriptors; pool: device words holding every image and projection;
 * workspace: device, mojette_workspace_size(plan, nblocks) bytes, 256-byte
 * aligned, overwritten.  status: device int32 or NULL, receives
 * MOJETTE_EINVAL for a descriptor with a bad geom_id or P (that block is
 * skipped) and MOJETTE_ENOTSUP as above; never cleared by the call.
 * Returns MOJETTE_OK, MOJETTE_EINVAL (bad arguments) or MOJETTE_EHIP. */
int mojette_encode_batched(const mojette_plan *plan, const mojette_block *blocks,
                           int64_t nblocks, uint64_t *pool, void *workspace, int32_t *status,
                           void *stream);

/* Inverse transform (Section 2.2) of every described block from the
 * projections its erasure mask leaves (bins of erased projections are never
 * read), writing its image.  A block with fewer than Q survivors is left
 * unwritten and MOJETTE_ENOTRECON is stored to *status.  Other arguments as
 * for mojette_encode_batched.  In calls of 16,384 blocks or more the
 * launches of different row counts run on streams of the library's (created
 * with the first plan on a device),
 * forked from `stream` after its earlier work and joined back to it before
 * its later work: ordering on `stream` is as for one launch, and the call
 * stays safe to record into a HIP graph. */
int mojette_decode_batched(const mojette_plan *plan, const mojette_block *blocks,
                           int64_t nblocks, uint64_t *pool, void *workspace, int32_t *status,
                           void *stream);

/*
 * Chunked decode of long rows (the inverse of Section 2.2, cut into chunks).
 * A block's decode is a left-to-right sweep whose length grows with P; for
 * long rows (large blocks) the sweep of one block is cut into chunks of about
 * chunk_cols columns that run in parallel: every chunk is swept from a zero
 * start, a carry pass applies the GF(2) transfer matrix of the block's
 * survivor set to turn the chunks' end states into exact start states
 * (XOR is linear), and every chunk is swept again from its exact start.
 * Results are bit-identical to mojette_decode_batch.
 *
 * A plan holds the transfer matrices of every Q-subset of the directions for
 * one chunk length.  mojette_chunk_plan_create computes them on the host and
 * copies them to the current device: it allocates device memory and
 * synchronises, so it is not for use under graph capture.  It returns
 * MOJETTE_ENOTSUP if chunks of that length are shorter than the decode's
 * own lead-in.  mojette_chunk_plan_destroy frees the plan (NULL is a no-op).
 */
int mojette_chunk_plan_create(const int32_t *dirs, int32_t n, int32_t Q, int32_t chunk_cols,
                              mojette_chunk_plan **plan);
/* A plan for blocks of 128-bit pixels (Section 3.1; layouts as for
 * mojette_decode_batch_wide): mojette_decode_batch_chunked and
 * mojette_decode_chunked_workspace on such a plan take P in 16-byte pixels
 * and the 128-bit layouts; chunk_cols counts 16-byte pixels.  |p| up to 2^14.
 * Not for jobs (mojette_decode_jobs) or mojette_decode_batch_chunked_trimmed,
 * which return MOJETTE_EINVAL on it. */
int mojette_chunk_plan_create_wide(const int32_t *dirs, int32_t n, int32_t Q,
                                   int32_t chunk_cols, mojette_chunk_plan **plan);
int mojette_chunk_plan_destroy(mojette_chunk_plan *plan);

/* Host only: the state width E (*state_cols) and transfer matrix of one
 * survivor set, directions p_sorted[0..Q) strictly ascending.  Row i of the
 * matrix (ceil(Q*E/64) words, bit j of word w = start-state word 64w + j)
 * lists the start-state words whose XOR is end-state word i when every bin
 * is zero; state word r*E + e is the pixel of row r at e columns from the
 * start of the state window.  Writes the rows when cap_words is large
 * enough and returns the words they take, -1 on bad arguments, -2 if chunks
 * of chunk_cols columns are too short. */
int64_t mojette_chunk_matrix(const int32_t *p_sorted, int32_t Q, int32_t chunk_cols,
                             int32_t *state_cols, uint64_t *rows, int64_t cap_words);

/* Device workspace (words) a chunked decode of nblocks blocks of row length
 * P needs; 0 when P is too short to cut (the call then decodes whole
 * blocks).  It is non-decreasing in nblocks: a workspace sized for nblocks
 * serves every call on at most nblocks blocks.  -1 on bad arguments. */
int64_t mojette_decode_chunked_workspace(const mojette_chunk_plan *plan, int32_t P,
                                         int64_t nblocks);

/*
 * mojette_decode_batch with the plan's directions and row count, the sweep
 * of every block cut into chunks.  Arguments as for mojette_decode_batch;
 * workspace: device, mojette_decode_chunked_workspace() words, owned by the
 * caller, overwritten.  Three launches on `stream` (two when a block has
 * only two chunks); allocates nothing; safe to record into a HIP graph.
 */
int mojette_decode_batch_chunked(const mojette_chunk_plan *plan, const uint64_t *projs,
                                 const uint16_t *erased, int64_t nblocks, int32_t P,
                                 uint64_t *images, int32_t *status, uint64_t *workspace,
                                 void *stream);

/*
 * mojette_decode_batch_chunked for projections in the layout without
 * never-used bins (block b's slice at word b * mojette_trimmed_layout(),
 * see mojette_decode_batch_trimmed): the chunks read only bins that layout
 * keeps.  Arguments, workspace and errors as mojette_decode_batch_chunked.
 */
int mojette_decode_batch_chunked_trimmed(const mojette_chunk_plan *plan, const uint64_t *projs,
                                         const uint16_t *erased, int64_t nblocks, int32_t P,
                                         uint64_t *images, int32_t *status,
                                         uint64_t *workspace, void *stream);

/*
 * mojette_decode_batch_chunked for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  The workspace is a fixed array of
 * MOJETTE_SCRATCH_WORDS 64-bit words (64 MiB) in the library's device
 * memory, which each GPU the library runs on holds until the process ends.
 * The call allocates nothing; its first call on a device looks up that
 * device's array (no allocation, no synchronisation).  Arguments and results
 * as for mojette_decode_batch_chunked.  A call whose
 * mojette_decode_chunked_workspace(plan, P, nblocks) exceeds
 * MOJETTE_SCRATCH_WORDS returns MOJETTE_ESCRATCH before anything is enqueued
 * (decode fewer blocks per call).  Every call on a GPU shares that GPU's
 * array and leaves its contents behind: calls that may overlap on one GPU
 * (on concurrent streams or threads) race and must be serialised by the
 * caller.
 */
#define MOJETTE_SCRATCH_WORDS ((int64_t)1 << 23)
int mojette_decode_batch_chunked_noalloc(const mojette_chunk_plan *plan, const uint64_t *projs,
                                         const uint16_t *erased, int64_t nblocks, int32_t P,
                                         uint64_t *images, int32_t *status, void *stream);

/*
 * Cost model of the schedule autotuner (not part of the paper's method: it
 * predicts how long a decode schedule takes and never touches pixel or bin
 * bits).  A two-hidden-layer fp32 perceptron with ReLU units and one linear
 * output, d_in inputs (1..16) and `hidden` units per layer (16 or 32):
 *   y = w3 . relu(W2 relu(W1 x + b1) + b2) + b3,
 * parameters packed as W1 (hidden x d_in, row-major), b1, W2 (hidden x
 * hidden), b2, w3, b3.  All buffers are device fp32; x is n x d_in row-major.
 */
int32_t mojette_mlp_params(int32_t d_in, int32_t hidden);   /* parameter count, -1 if unsupported */
int mojette_mlp_forward(const float *params, int32_t d_in, int32_t hidden, const float *x,
                        int64_t n, float *y, void *stream);
/* Gradient of the mean squared error L = (1/n) sum (y - t)^2 by
 * backpropagation: grad receives the parameter count + 1 floats, the last
 * one L.  workspace: mojette_mlp_grad_workspace() floats.  Deterministic (no
 * atomics). */
int64_t mojette_mlp_grad_workspace(int32_t d_in, int32_t hidden, int64_t n);
int mojette_mlp_grad(const float *params, int32_t d_in, int32_t hidden, const float *x,
                     const float *t, int64_t n, float *grad, float *workspace, void *stream);
/* One Adam step (Kingma and Ba, with bias correction; step counts from 1)
 * on params in place; m and v are the moment buffers. */
int mojette_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t nparams,
                     float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/* Ring length (words per row) the decoder needs for this geometry: the
 * longest distance, over every choice of Q survivors, between a pixel a row
 * needs and the newest pixel of that row, rounded up to a power of two and
 * at least the tile width.  -1 on bad arguments. */
int32_t mojette_decode_ring(const int32_t *dirs, int32_t n, int32_t P, int32_t Q);

#ifdef __cplusplus
}
#endif

#endif /* MOJETTE_H */
