/*
 * mojette_synth.h -- input generation and measurement helpers of the HIP
 * library.  None of these is part of the Mojette method: they fill device
 * pools with the seeded synthetic data the tests and the benchmark use, and
 * provide a plain streaming copy whose bandwidth serves as the practical
 * ceiling the kernels are compared with.
 */
#ifndef MOJETTE_SYNTH_H
#define MOJETTE_SYNTH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dst[i] = output (start + i) of SplitMix64 seeded with `seed` (Steele, Lea
 * and Flood, OOPSLA 2014): mix(seed + (start + i + 1) * 0x9E3779B97F4A7C15),
 * mix = xor-shift 30, * 0xBF58476D1CE4E5B9, xor-shift 27,
 * * 0x94D049BB133111EB, xor-shift 31.  dst is a device pointer to nwords
 * words.  Asynchronous on stream.  Returns 0 or a negative mojette status. */
int mojette_fill_splitmix64(uint64_t *dst, int64_t nwords, uint64_t seed, uint64_t start,
                            void *stream);

/* Streaming device copy of nwords 64-bit words (16-byte accesses where the
 * pointers allow).  dst and src are device pointers and must not overlap. */
int mojette_copy_words(uint64_t *dst, const uint64_t *src, int64_t nwords, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MOJETTE_SYNTH_H */
