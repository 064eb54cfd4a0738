/*
 * dq_mixed.h - streams whose block edge changes from one 16^d super-block to
 * the next (libdq).
 *
 * The paper tunes the block size by trying the configurations on the data
 * (Section III-E) and finds that the best padding and block size depend on
 * the data (Section IV, Section V-I). Here the field is cut into super-blocks
 * of 16 cells along every axis (aligned at the origin, truncated at the high
 * end), and each super-block s carries its own block edge edges[s] in
 * {4, 8, 16}: its cells are split into cubic blocks of that edge, aligned at
 * the super-block origin and truncated at the field's end. Every block is
 * coded exactly as a block of dq_compress with DQ_PAD_GIVEN (its halo value
 * pads[b], Section IV): q = round(x / 2eb), first-order Lorenzo residual
 * inside the block, code = delta + R within the radius, else code 0 and an
 * outlier (Section III-A). Orders:
 *   super-blocks   row-major over the super-block grid;
 *   blocks         super-block by super-block, row-major inside each;
 *   pads           one int32 per block, in that block order;
 *   outliers       block by block in that order, cells in local row-major
 *                  order; C-order linear indices into the field (uint32);
 *   codes          uint16 in C order of the field, as dq_compress.
 * With every edge 16 the stream is exactly that of dq_compress with block 16
 * and DQ_PAD_GIVEN. The edges and the pads are part of the stream: the
 * decoder needs them (and eb_abs, n_out) to invert it exactly.
 *
 * Parameters: p->ndim, p->shape and p->radius as in dq.h, p->eb the
 * ABSOLUTE bound (p->eb_mode must be DQ_EB_ABS); p->block, p->pad_mode and
 * p->vec are ignored.
 *
 * Memory: every array is a DEVICE pointer owned by the caller; calls enqueue
 * kernels on hip_stream and return without waiting; host-side errors return
 * before anything is enqueued. An edge value other than 4, 8 or 16 is coded
 * as 16 and makes the call's device status DQ_EINVAL.
 */
#ifndef DQ_MIXED_H
#define DQ_MIXED_H

#include <stdint.h>

#include "dq.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Number of 16^d super-blocks of the field (host only). */
dq_status dq_mixed_num_super(const dq_params *p, uint64_t *n_super);

/* pad_off[s] = number of blocks of the super-blocks before s (n_super + 1
 * entries; pad_off[n_super] = number of pads of the stream), from the edges
 * (n_super uint8). status (device int32, may be NULL) receives DQ_EINVAL for
 * an invalid edge (it is not written otherwise). */
dq_status dq_mixed_pad_offsets(const dq_params *p, const uint8_t *edges, uint32_t *pad_off, int32_t *status,
                               void *hip_stream);

/* Device workspace (bytes) of dq_mixed_compress / dq_mixed_decompress. */
dq_status dq_mixed_workspace(const dq_params *p, uint64_t *bytes);

/* Compress x (N fp32) with the per-super-block edges and the per-block pads
 * (pad_off from dq_mixed_pad_offsets for the same edges). res as dq_compress
 * (status, exact n_out, eb_abs); more outliers than out_cap give
 * DQ_ECAPACITY with complete codes and the exact count. */
dq_status dq_mixed_compress(const dq_params *p, const float *x, const uint8_t *edges, const uint32_t *pad_off,
                            const int32_t *pads, uint16_t *codes, uint32_t *out_idx, int32_t *out_val,
                            uint64_t out_cap, dq_result *res, void *ws, uint64_t ws_bytes, void *hip_stream);

/* Decompress into x_hat (N fp32). res->status becomes DQ_ECORRUPT when the
 * outliers are not exactly the zero codes in stream order (x_hat is then
 * unspecified); res->n_out and res->eb_abs echo the arguments. */
dq_status dq_mixed_decompress(const dq_params *p, double eb_abs, const uint8_t *edges, const uint32_t *pad_off,
                              const int32_t *pads, const uint16_t *codes, const uint32_t *out_idx,
                              const int32_t *out_val, uint64_t n_out, float *x_hat, dq_result *res, void *ws,
                              uint64_t ws_bytes, void *hip_stream);

/* The edge of every super-block from the side costs of the three edges
 * (cost: 3 x n_super uint64, edge 4 first, as dq_super_cost writes them per
 * edge): the lowest cost, ties to the larger edge. edges receives 4, 8 or 16,
 * label 0, 1 or 2; either may be NULL. */
dq_status dq_super_label(const dq_params *p, const uint64_t *cost, uint8_t *edges, int32_t *label,
                         void *hip_stream);

/* The network's edge of every super-block: logits (8 floats per block of
 * the field at edge `base`, in row-major block order, as
 * dq_mlp_infer_bf16 writes them) summed over the super-block's blocks in
 * outputs 5, 6, 7 (edge 4, 8, 16), the largest sum, ties to the larger edge.
 * edges / label as dq_super_label. */
dq_status dq_super_vote(const dq_params *p, int32_t base, const float *logits, uint8_t *edges, int32_t *label,
                        void *hip_stream);

/* The pads of a mixed stream (pad_off[n_super] int32, stream order) from
 * per-edge pads in each edge's row-major block order of the whole field
 * (pads4 / pads8 / pads16: one int32 per block at that edge). */
dq_status dq_mixed_gather_pads(const dq_params *p, const uint8_t *edges, const uint32_t *pad_off,
                               const int32_t *pads4, const int32_t *pads8, const int32_t *pads16, int32_t *pads,
                               void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
