/*
 * dqref.h - CPU oracle for SZ dual-quantisation (TEST INFRASTRUCTURE ONLY).
 *
 * A plain, slow, obviously correct implementation of the dual-quantisation
 * prediction/quantisation step of "SIMD Lossy Compression for Scientific Data"
 * (Dube et al., arXiv 2201.04614), Section III-A, with the block padding
 * values of Section IV (IV-A value choice, IV-B granularity). It exists to
 * check the GPU library against; only tests, the smoke check and the
 * benchmark's CPU-baseline leg may call it. It shares no code, header or
 * constant with the GPU library.
 *
 * What it computes (each step cites the passage it follows):
 *   eb        absolute bound, or value-range relative bound rel*(max-min)
 *             (Section II-B, error-bound modes)
 *   q         prequantised integer q = round(x / (2 eb)) (Section III-A, the
 *             pre-quantisation stage; bound |x - 2 eb q| <= eb), the exact
 *             rational quotient rounded to nearest, halves to even
 *   pads      per-block padding value: zero, global mean, block mean or
 *             edge mean (Section IV-A value, IV-B granularity)
 *   delta     first-order Lorenzo residual of q inside each block, with the
 *             padding forming the halo in front of the block (Section III-A
 *             post-quantisation stage; predictor as in the Lorenzo papers
 *             the paper cites)
 *   codes     uint16 code delta+R when -R < delta < R, else 0 and an outlier
 *             entry (global index, delta) in block-major order (Section III-A,
 *             values that do not quantise are stored separately)
 *   decode    sequential Lorenzo reconstruction from already reconstructed
 *             neighbours (Section III-A: decompression reverses the
 *             prediction point by point), then x_hat = (float)(q * 2 eb).
 *
 * All integer arithmetic on q and delta wraps modulo 2^32. Floating point is
 * IEEE fp64, round to nearest even, no contraction.
 *
 * Status codes (returned as int):
 *    0 OK, -1 EINVAL (bad parameters), -2 ERANGE (non-finite input or
 *    |q| beyond 2^31-1), -3 ECAPACITY (more outliers than out_cap;
 *    *n_out still holds the true count), -6 ECORRUPT (decode input
 *    inconsistent: a zero code without its outlier, an outlier on a non-zero
 *    code, an index out of range, or outliers not in strict block-major order).
 */
#ifndef DQREF_H
#define DQREF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DQREF_OK 0
#define DQREF_EINVAL (-1)
#define DQREF_ERANGE (-2)
#define DQREF_ECAPACITY (-3)
#define DQREF_ECORRUPT (-6)

#define DQREF_EB_ABS 0
#define DQREF_EB_REL 1

#define DQREF_PAD_ZERO 0
#define DQREF_PAD_BLOCK_MEAN 1
#define DQREF_PAD_EDGE_MEAN 2
#define DQREF_PAD_GLOBAL_MEAN 3
/* Section IV-A also takes the minimum or the maximum of the data as the
 * statistic, at block or global granularity (Section IV-B) */
#define DQREF_PAD_BLOCK_MIN 4
#define DQREF_PAD_BLOCK_MAX 5
#define DQREF_PAD_GLOBAL_MIN 6
#define DQREF_PAD_GLOBAL_MAX 7
/* one value per block chosen by the caller (a per-block padding selector):
 * pads is an input of compress, and the halo of block b is pads[b] */
#define DQREF_PAD_GIVEN 8

/* Field description. shape[0] is the slowest axis (C order); only the first
 * ndim entries are used. eb is the absolute bound (eb_mode ABS) or the
 * relative factor (eb_mode REL). block is the cubic block edge B (>= 1).
 * radius R in [1, 32768]. */
typedef struct {
    int32_t ndim;
    int32_t eb_mode;
    int64_t shape[3];
    double eb;
    int32_t block;
    int32_t pad_mode;
    int32_t radius;
    int32_t reserved;
} dqref_params;

int dqref_validate(const dqref_params *p);
/* number of int32 pad values: 0 (zero), 1 (global mean / min / max),
 * nBlocks (block mean / min / max, given), nBlocks*ndim (edge); -1 on
 * invalid parameters */
int64_t dqref_pad_count(const dqref_params *p);
int64_t dqref_num_blocks(const dqref_params *p);

/* nearest integer to S/n, halves toward +infinity (n > 0) */
int64_t dqref_round_mean(int64_t S, int64_t n);

/* absolute error bound from the parameters and the field */
int dqref_resolve_eb(const dqref_params *p, const float *x, double *eb_abs);
/* q[i] = nearest integer to the exact x[i] / (2 eb_abs), halves to even */
int dqref_prequantize(const dqref_params *p, const float *x, double eb_abs, int32_t *q);
/* pad values from q (length dqref_pad_count); GIVEN leaves pads as they are */
int dqref_pad_values(const dqref_params *p, const int32_t *q, int32_t *pads);
/* Lorenzo residual of every element, natural (C-order) layout */
int dqref_residuals(const dqref_params *p, const int32_t *q, const int32_t *pads,
                    int32_t *delta, int nthreads);
/* sequential inverse of dqref_residuals */
int dqref_reconstruct(const dqref_params *p, const int32_t *delta, const int32_t *pads,
                      int32_t *q, int nthreads);

/* Whole compression: codes[N] (natural layout), outliers in block-major
 * order, pads, and the absolute bound actually used. */
int dqref_compress(const dqref_params *p, const float *x, uint16_t *codes,
                   uint32_t *out_idx, int32_t *out_val, uint64_t out_cap,
                   uint64_t *n_out, int32_t *pads, double *eb_abs, int nthreads);

/* Whole decompression. */
int dqref_decompress(const dqref_params *p, double eb_abs, const uint16_t *codes,
                     const uint32_t *out_idx, const int32_t *out_val, uint64_t n_out,
                     const int32_t *pads, float *x_hat, int nthreads);

#ifdef __cplusplus
}
#endif
#endif
