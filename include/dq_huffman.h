/*
 * dq_huffman.h - entropy stage of libdq: canonical Huffman over the uint16
 * quantisation codes (SZ's coding of the codes, Section II-B; the paper
 * keeps it out of the optimised prediction step).
 *
 * Format (the same as the oracle's):
 *  - code lengths by the two-queue Huffman construction over the present
 *    symbols sorted by (frequency, symbol), a leaf taken before an internal
 *    node of equal weight; a single present symbol has length 1; lengths
 *    above 32 are avoided by halving every present frequency (kept >= 1) and
 *    building again;
 *  - canonical codewords: symbols in (length, symbol) order;
 *  - the bitstream: chunks of DQ_HUFF_CHUNK codes, each starting on a 32-bit
 *    word, codewords most significant bit first; chunk_off[c] is the first
 *    word of chunk c and chunk_off[n_chunks] the total (uint64);
 *    sub_off[3 c + k] (uint16) is the bit offset, from the start of chunk c,
 *    of its code (k + 1) * DQ_HUFF_SUB (the chunk's bit count when the chunk
 *    is shorter): a chunk is decoded from four places at once.
 *
 * Memory: all arrays are DEVICE pointers owned by the caller; calls enqueue
 * kernels on hip_stream and return; status (device int32) receives DQ_OK or
 * the first error of the call: DQ_EINVAL (a code >= n_symbols, or a code
 * without a codeword), DQ_ENOTSUP (more than DQ_HUFF_MAX_PRESENT distinct
 * codes), DQ_ECAPACITY (words_cap too small), DQ_ECORRUPT (decode: a
 * bitstream that does not parse). Host-side errors return before anything
 * is enqueued.
 */
#ifndef DQ_HUFFMAN_H
#define DQ_HUFFMAN_H

#include <stdint.h>

#include "dq.h"

#ifdef __cplusplus
extern "C" {
#endif

#define DQ_HUFF_CHUNK 1024
#define DQ_HUFF_SUB 256
#define DQ_HUFF_MAX_SYMBOLS 65536 /* alphabet size limit (codes are uint16) */
#define DQ_HUFF_MAX_PRESENT 2048  /* distinct codes the GPU codebook builder takes */

/* Device workspace (bytes) of the calls below for n codes. */
dq_status dq_huff_workspace(uint64_t n, uint64_t *bytes);

/* Words a bitstream of n codes can need at most (32-bit codewords plus the
 * padding of every chunk). */
dq_status dq_huff_max_words(uint64_t n, uint64_t *words);

/* Histogram hist[n_symbols] of the n codes, code lengths lengths[n_symbols]
 * (uint8, 0 for absent codes) and canonical codewords codewords[n_symbols]. */
dq_status dq_huff_codebook(const uint16_t *codes, uint64_t n, uint32_t n_symbols, uint32_t *hist,
                           uint8_t *lengths, uint32_t *codewords, int32_t *status, void *ws,
                           uint64_t ws_bytes, void *hip_stream);

/* Bitstream of the n codes: chunk_off[n_chunks + 1], sub_off[3 n_chunks],
 * words[words_cap]. */
dq_status dq_huff_encode(const uint16_t *codes, uint64_t n, uint32_t n_symbols, const uint8_t *lengths,
                         const uint32_t *codewords, uint64_t *chunk_off, uint16_t *sub_off, uint32_t *words,
                         uint64_t words_cap, int32_t *status, void *ws, uint64_t ws_bytes, void *hip_stream);

/* The n codes back from the bitstream words[n_words] (four threads per
 * chunk; canonical decoding with an 11-bit lookup table). Reads stay inside
 * words whatever chunk_off and sub_off hold. */
dq_status dq_huff_decode(const uint32_t *words, uint64_t n_words, const uint64_t *chunk_off,
                         const uint16_t *sub_off, uint64_t n, uint32_t n_symbols, const uint8_t *lengths,
                         uint16_t *codes, int32_t *status, void *ws, uint64_t ws_bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
