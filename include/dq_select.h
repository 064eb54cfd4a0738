/*
 * dq_select.h - C ABI of the per-block padding / block-size selector of libdq.
 *
 * The padding of a block only enters the residual of its origin cell, where
 * the residual is q_o - P_eff (the halo is constant on every face, so it
 * cancels in every other Lorenzo difference; Section III-A with the block
 * padding of Section IV). Choosing a padding value per block among
 * statistics of the data (Section IV-A: mean, minimum, maximum; Section
 * IV-B: per field, per block, per block and axis) is therefore decided by
 * the origin alone, and the choice is stored as the per-block values of
 * DQ_PAD_GIVEN, which every decoder reads back exactly. The block size is
 * searched per 16^d super-block over {4, 8, 16} (the paper tunes the block
 * size by trying the configurations on the data, Section III-E).
 *
 * Entry points, in the order a search or a learned selection uses them:
 *   dq_block_stats    per-block integer statistics of q = round(x / 2eb)
 *   dq_block_select   candidates, origin outlier flags, exhaustive label and
 *                     24 features per block
 *   dq_super_cost     side cost of a per-block choice, per super-block
 *   dq_gather_pads    the chosen candidates as DQ_PAD_GIVEN values
 *   dq_mlp_*          the 24-64-64-8 network: gradient (fp32), Adam update,
 *                     bf16 packing and bf16 inference with fp32 accumulation
 *
 * Memory: all array arguments are DEVICE pointers owned by the caller; the
 * calls enqueue kernels on hip_stream (a hipStream_t, NULL = null stream)
 * and return without waiting. Host-side errors are returned before anything
 * is enqueued. Block order is the row-major order of the block grid.
 */
#ifndef DQ_SELECT_H
#define DQ_SELECT_H

#include <stdint.h>

#include "dq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Integer statistics of the pre-quantised values q of one block (80 bytes).
 * Axis a counts from the slowest axis (C order); entries a >= ndim are 0.
 *   qo        q at the block origin
 *   mn, mx    minimum and maximum of q
 *   nonorig   zero codes (outliers) at the block's other cells, from the
 *             codes of a compression of the same field and block (0 when
 *             no codes are given)
 *   sum       sum of q; mad = sum |q - qo|
 *   fsum[a]   sum of q over the cells with local coordinate 0 along a
 *   rough[a]  sum |q(u) - q(u - e_a)| over the in-block neighbour pairs */
typedef struct {
    int32_t qo, mn, mx;
    uint32_t nonorig;
    int64_t sum, mad;
    int64_t fsum[3];
    int64_t rough[3];
} dq_block_stat;

#define DQ_SEL_FEATURES 24
#define DQ_SEL_CANDIDATES 5 /* zero, global mean, block mean, edge-mean effective value, block midrange */
#define DQ_SEL_HIDDEN 64
#define DQ_SEL_OUTPUTS 8    /* 5 padding logits, then 3 block-size logits (edge 4, 8, 16) */
#define DQ_SEL_SUPER 16     /* super-block edge of the block-size choice */

/* Number of fp32 network parameters: W1[64][24], b1[64], W2[64][64], b2[64],
 * W3[8][64], b3[8], packed in that order, row-major. */
#define DQ_MLP_PARAMS (64 * 24 + 64 + 64 * 64 + 64 + 8 * 64 + 8)

/* Statistics of every block of the field x (N fp32) for the bound eb_abs
 * (p->eb and p->eb_mode are ignored) and block p->block, which must satisfy
 * block^ndim <= 4096. codes: the codes of a compression of x with the same
 * block (any padding), or NULL. status (device int32, may be NULL) receives
 * DQ_ERANGE if some |q| exceeds 2^31 - 1 or x is not finite (it is not
 * written otherwise). */
dq_status dq_block_stats(const dq_params *p, double eb_abs, const float *x, const uint16_t *codes,
                         dq_block_stat *stats, int32_t *status, void *hip_stream);

/* From the statistics: per block the five candidate padding values
 * cand[b * 5 + c] (zero, global mean, block mean, edge-mean effective value,
 * block midrange; means rounded to nearest, halves up), the bit set flags[b]
 * of candidates that leave the origin an outlier (|q_o - P| >= radius,
 * modulo 2^32), the exhaustive label[b] (first candidate that keeps the
 * origin predictable, 0 if none) and 24 fp32 features feat[b * 24 + k], each
 * an fp64 expression of exact integers rounded once. Any output but cand
 * may be NULL. ws: device scratch of at least 8 bytes, 8-byte aligned. */
dq_status dq_block_select(const dq_params *p, const dq_block_stat *stats, int32_t *cand, uint8_t *flags,
                          int32_t *label, float *feat, void *ws, void *hip_stream);

/* Adds to cost[s] (one uint64 per 16^d super-block, row-major over the
 * super-block grid) the side cost 8 * outliers + 4 of every block of the
 * super-block, where a block's outliers are its nonorig count plus the
 * flag of its chosen candidate choice[b]. */
dq_status dq_super_cost(const dq_params *p, const dq_block_stat *stats, const uint8_t *flags,
                        const int32_t *choice, uint64_t *cost, void *hip_stream);

/* Number of 16^d super-blocks of the field. */
dq_status dq_num_super(const dq_params *p, uint64_t *n_super);

/* pads[b] = cand[b * 5 + choice[b]]: the values of DQ_PAD_GIVEN. choice
 * entries outside 0..4 select candidate 0. */
dq_status dq_gather_pads(const int32_t *cand, const int32_t *choice, uint64_t n_blocks, int32_t *pads,
                         void *hip_stream);

/* Device workspace (bytes) of dq_mlp_grad for n samples. */
dq_status dq_mlp_workspace(uint64_t n, uint64_t *bytes);

/* Gradient of the mean over the n samples (n >= 1) of the two heads' softmax
 * cross-entropies, labels y_pad in 0..4 and y_bsz in 0..2 (rows of X are the
 * 24 features), with respect to the packed parameters theta (fp32
 * arithmetic). grad receives DQ_MLP_PARAMS floats, loss one float (may be
 * NULL). The reduction over samples is in a fixed order, so the result
 * does not depend on timing. */
dq_status dq_mlp_grad(const float *theta, const float *X, const int32_t *y_pad, const int32_t *y_bsz,
                      uint64_t n, float *grad, float *loss, void *ws, uint64_t ws_bytes, void *hip_stream);

/* One Adam step (Kingma and Ba: beta1 0.9, beta2 0.999, eps 1e-8) of
 * theta with moments m, v (all DQ_MLP_PARAMS floats) at step t >= 1. */
dq_status dq_mlp_adam(float *theta, float *m, float *v, const float *grad, int32_t t, float lr,
                      void *hip_stream);

/* theta rounded to bfloat16 (nearest, ties to even): DQ_MLP_PARAMS uint16. */
dq_status dq_mlp_to_bf16(const float *theta, uint16_t *theta_bf16, void *hip_stream);

/* Inference of n samples with bf16 weights, the inputs and hidden
 * activations rounded to bf16, products accumulated in fp32. logits (n x 8,
 * may be NULL); pad_choice / bsz_choice (may be NULL) receive the argmax of
 * each head (lowest index on ties). */
dq_status dq_mlp_infer_bf16(const uint16_t *theta_bf16, const float *X, uint64_t n, float *logits,
                            int32_t *pad_choice, int32_t *bsz_choice, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
