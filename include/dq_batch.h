/*
 * dq_batch.h - many fields, one HIP graph launch (libdq).
 *
 * A batch of fields of different shapes, bounds, blocks and paddings is
 * compressed and decompressed by one graph: every field's dq_compress and
 * dq_decompress_dev (which takes the outlier count and bound from the
 * compress result on the device) are captured once, spread over parallel
 * branches (largest fields first, each to the least loaded branch), and the
 * instantiated graph is launched as often as wanted. The fields' buffers are
 * bound at creation: a launch reads the current contents of every x and
 * rewrites every output. Blocks are compressed independently (Section III-A),
 * so the fields need no ordering among themselves.
 *
 * Callers: batch pipelines and serving loops that launch the same set of
 * buffers repeatedly. Memory: every pointer in dq_batch_field is a DEVICE
 * pointer owned by the caller, sized as for dq_compress / dq_decompress; the
 * graph handle is host memory owned by the library until
 * dq_batch_graph_destroy. The parameters are copied at creation.
 */
#ifndef DQ_BATCH_H
#define DQ_BATCH_H

#include <stdint.h>

#include "dq.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    dq_params p;
    const float *x;     /* field */
    uint16_t *codes;
    uint32_t *out_idx;
    int32_t *out_val;
    uint64_t out_cap;
    int32_t *pads;      /* read instead of written for DQ_PAD_GIVEN */
    dq_result *cres;    /* compress result */
    void *cws;
    uint64_t cws_bytes;
    float *x_hat;       /* NULL: compress only */
    dq_result *dres;    /* decompress result */
    void *dws;
    uint64_t dws_bytes;
} dq_batch_field;

typedef struct dq_batch_graph dq_batch_graph;

/* Capture the batch (n >= 1 fields) over `branches` parallel branches
 * (1..16) into a graph. Host-side errors of any field (as dq_compress /
 * dq_decompress_dev would return them) abort the creation and are returned;
 * DQ_EDEVICE if a HIP call fails. */
dq_status dq_batch_graph_create(const dq_batch_field *fields, uint64_t n, int branches,
                                dq_batch_graph **graph);

/* The persistent form of the batch (Section III-F: blocks are independent
 * work items, here taken from every field at once). The graph holds a fixed
 * number of kernels whatever the number of fields: one value-range pass
 * over all fields (which also resolves every field's bound), one persistent
 * encode per (dimensionality, block, cells per lane) class of the batch
 * whose waves drain a flattened queue of (field, run of tiles) units with an
 * atomic ticket, one outlier placement pass over all fields, and one
 * persistent decode per class. Every field is compressed and decompressed
 * exactly as dq_compress and dq_decompress_dev would (same streams, same
 * results in cres / dres).
 * Needs, beyond dq_batch_graph_create: x_hat != NULL, out_cap >= the field's
 * cell count, a padding other than DQ_PAD_GLOBAL_MEAN, cws of
 * dq_compress_workspace(p, out_cap) bytes (256-byte aligned) - else
 * DQ_ENOTSUP / DQ_EINVAL; dws and dws_bytes are not used. The decode takes
 * each block's outlier run from the compress call's workspace, so the
 * graph must be launched as a whole.
 * ws: device workspace (256-byte aligned) of at least
 * dq_batch_persistent_workspace bytes, holding the queues and the fields'
 * arguments; written once here (synchronously), read by every launch, owned
 * by the caller and kept until dq_batch_graph_destroy. Launches of the same
 * graph must not overlap (they share the tickets in ws).
 * class_out / vec_out (host arrays of n, either may be NULL): each field's
 * class (0 = the class with the most cells, the one dq_batch_persistent_run
 * times) and cells per lane. */
dq_status dq_batch_persistent_workspace(const dq_batch_field *fields, uint64_t n, uint64_t *bytes);
dq_status dq_batch_persistent_create(const dq_batch_field *fields, uint64_t n, void *ws, uint64_t ws_bytes,
                                     int32_t *class_out, int32_t *vec_out, dq_batch_graph **graph);

/* The kernels of a persistent batch enqueued directly on hip_stream, one
 * after another (no graph, no branches; same results as a graph launch),
 * with optional timing events recorded right before and after the encode
 * (enc_hooks) and decode (dec_hooks) kernel of the class with the most
 * cells. DQ_EINVAL for a graph not made by dq_batch_persistent_create. */
dq_status dq_batch_persistent_run(dq_batch_graph *graph, void *hip_stream, const dq_hooks *enc_hooks,
                                  const dq_hooks *dec_hooks);

/* Enqueue one execution of the graph on hip_stream. Per-field outcomes land
 * in each field's cres / dres. */
dq_status dq_batch_graph_launch(dq_batch_graph *graph, void *hip_stream);

dq_status dq_batch_graph_destroy(dq_batch_graph *graph);

#ifdef __cplusplus
}
#endif
#endif
