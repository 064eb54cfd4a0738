/*
 * dq.h - C ABI of libdq, the MI355X (gfx950) dual-quantisation library.
 *
 * Dual-quantisation is the prediction/quantisation step of SZ as re-designed
 * by cuSZ and studied in "SIMD Lossy Compression for Scientific Data" (Dube
 * et al., arXiv 2201.04614), Section III-A:
 *
 *   compress    q = round(x / (2 eb))                   pre-quantisation
 *               delta = q - Lorenzo prediction of q      inside fixed-size
 *                       from its lower neighbours         blocks, the block
 *                       in the same block                 padding forming the
 *                                                         halo (Section IV)
 *               code = delta + R   if -R < delta < R     post-quantisation
 *               else code = 0 and (index, delta) is an outlier
 *   decompress  the inverse: outlier scatter, a blockwise n-D prefix sum of
 *               delta plus the block's effective padding, and
 *               x_hat = (float)((double)q * 2 eb).
 *
 * Every result is exact integer or IEEE arithmetic and is defined uniquely:
 *  - q is the nearest integer to the exact rational x / (2 eb), exact halves
 *    to even, so |x - 2 eb q| <= eb for every element; |q| <= 2^31 - 1;
 *  - arithmetic on q and delta wraps modulo 2^32 (the inverse is exact);
 *  - padding values are a statistic of q (Section IV-A): its integer mean,
 *    rounded to nearest with halves toward +infinity, or its minimum or
 *    maximum; taken per field, per block, or per block and axis (Section
 *    IV-B). The EDGE value of axis a is the mean of the block's own cells
 *    whose local coordinate along a is 0; a halo cell in front of the block
 *    along several axes takes the rounded mean of those axes' values;
 *  - blocks are cubic (edge B along every axis of the field), aligned at the
 *    origin, truncated at the high end of each axis;
 *  - outliers are listed block by block (blocks in row-major order of the
 *    block grid), cells in local row-major order; indices are C-order linear
 *    indices into the field (uint32).
 *
 * Memory: every buffer is owned by the caller. Pointers named x, codes,
 * out_idx, out_val, pads, x_hat, res and ws are DEVICE pointers (hipMalloc
 * or torch CUDA tensors); params and res_host are host pointers. The library
 * allocates nothing. Its mutable global state is a process-wide counter that
 * tags each decompress call's result (atomic, so calls from several host
 * threads are safe), the fixed scratch array of dq_compress_noalloc (one per
 * device) and a table of that array's device addresses (guarded by a lock).
 * Calls on different streams with different buffers may run concurrently,
 * except dq_compress_noalloc calls on the same device, which share its
 * scratch array.
 *
 * Streams: dq_compress and dq_decompress validate on the host, then enqueue
 * their kernels on hip_stream (a hipStream_t; NULL = the null stream) and
 * return without waiting. Device-side outcomes (status, outlier count, the
 * absolute error bound used) are written to the device-resident dq_result;
 * dq_result_sync copies it to the host and waits for the stream.
 *
 * Errors are returned, never thrown. A host-side error means nothing was
 * enqueued.
 */
#ifndef DQ_H
#define DQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DQ_OK = 0,
    DQ_EINVAL = -1,     /* invalid parameter, null pointer, workspace too small,
                           or (device) a relative bound over a zero value range */
    DQ_ERANGE = -2,     /* (device) non-finite input, or |q| > 2^31 - 1 */
    DQ_ECAPACITY = -3,  /* (device) more outliers than out_cap; n_out is exact */
    DQ_ENOTSUP = -4,    /* valid but not supported by the GPU kernels (block
                           not a power of two, beyond the supported edge, or
                           a 2-D block of 128 / 256 over rows whose length
                           is not a multiple of block / 64) */
    DQ_EDEVICE = -5,    /* a HIP runtime call failed */
    DQ_ECORRUPT = -6,   /* (device, decompress) codes and outliers disagree */
    DQ_ENOSCRATCH = -7  /* dq_compress_noalloc: the call needs more workspace
                           than the fixed scratch array holds */
} dq_status;

typedef enum { DQ_EB_ABS = 0, DQ_EB_REL = 1 } dq_eb_mode;

typedef enum {
    DQ_PAD_ZERO = 0,        /* no side data */
    DQ_PAD_BLOCK_MEAN = 1,  /* one int32 per block */
    DQ_PAD_EDGE_MEAN = 2,   /* ndim int32 per block, axis-major inside a block */
    DQ_PAD_GLOBAL_MEAN = 3, /* one int32 */
    DQ_PAD_BLOCK_MIN = 4,   /* one int32 per block: min of the block's q */
    DQ_PAD_BLOCK_MAX = 5,   /* one int32 per block: max of the block's q */
    DQ_PAD_GLOBAL_MIN = 6,  /* one int32: min of q over the field (also takes
                               the value-range pass with an absolute bound) */
    DQ_PAD_GLOBAL_MAX = 7,  /* one int32: max of q over the field (idem) */
    DQ_PAD_GIVEN = 8        /* one int32 per block chosen by the caller (a
                               per-block padding selector): an INPUT of
                               dq_compress, the halo value of its block */
} dq_pad_mode;

/* Field and codec parameters.
 *  ndim      1, 2 or 3
 *  shape     extents, shape[0] slowest (C order); entries >= ndim ignored;
 *            product < 2^32
 *  eb        absolute bound (DQ_EB_ABS) or factor of the value range
 *            max(x) - min(x) (DQ_EB_REL), finite and > 0
 *  block     block edge B >= 1 (GPU: a power of two, B <= 4096 in 1-D,
 *            B <= 256 in 2-D, B <= 64 in 3-D)
 *  pad_mode  dq_pad_mode
 *  radius    R in [1, 32768]: codes are uint16, 0 marks an outlier
 *  vec       kernel tuning hint, no effect on results: consecutive cells per
 *            lane (vector length of the loads), 1, 2 or 4; 0 = automatic.
 *            A hint the field or the buffer alignment does not allow is
 *            replaced by the automatic choice. */
typedef struct {
    int32_t ndim;
    int32_t eb_mode;
    int64_t shape[3];
    double eb;
    int32_t block;
    int32_t pad_mode;
    int32_t radius;
    int32_t vec;
} dq_params;

/* Device-resident outcome of one call, 8-byte aligned. status and reserved
 * form one 64-bit word that the kernels update atomically; reserved holds a
 * per-call tag of the library (its value has no meaning to the caller). */
typedef struct {
    int32_t status;   /* dq_status */
    uint32_t reserved;
    uint64_t n_out;   /* exact number of outliers (compress) */
    double eb_abs;    /* absolute error bound used (compress) */
} dq_result;

/* Optional timing hooks: hipEvent_t handles recorded on hip_stream right
 * before and right after the call's main kernel (encode or decode).
 * Either may be NULL. */
typedef struct {
    void *ev_before;
    void *ev_after;
} dq_hooks;

/* Host-only parameter check (no GPU needed): DQ_OK, DQ_EINVAL or DQ_ENOTSUP. */
dq_status dq_validate(const dq_params *p);

/* Number of blocks of the field. */
dq_status dq_num_blocks(const dq_params *p, uint64_t *n_blocks);

/* Number of int32 padding values: 0 (ZERO), 1 (GLOBAL_MEAN / MIN / MAX),
 * n_blocks (BLOCK_MEAN / MIN / MAX, GIVEN), n_blocks * ndim (EDGE_MEAN). */
dq_status dq_pad_count(const dq_params *p, uint64_t *n_pads);

/* Device workspace (bytes, 256-byte aligned start) needed by dq_compress
 * with room for out_cap outliers, and by dq_decompress. */
dq_status dq_compress_workspace(const dq_params *p, uint64_t out_cap, uint64_t *bytes);
dq_status dq_decompress_workspace(const dq_params *p, uint64_t *bytes);

/* Compress x (N fp32, C order) into codes (N uint16, C order), the outlier
 * list out_idx/out_val (room for out_cap entries, block-major order) and pads
 * (dq_pad_count int32; read instead of written for DQ_PAD_GIVEN). out_idx/
 * out_val may be NULL when out_cap == 0; pads may be NULL when dq_pad_count
 * is 0. res receives status, n_out, eb_abs.
 * If n_out > out_cap the status is DQ_ECAPACITY, the codes are complete, the
 * outlier list is not, and n_out is exact: retry with out_cap >= n_out.
 * x, codes and ws must not overlap any other buffer. */
dq_status dq_compress(const dq_params *p, const float *x, uint16_t *codes,
                      uint32_t *out_idx, int32_t *out_val, uint64_t out_cap,
                      int32_t *pads, dq_result *res, void *ws, uint64_t ws_bytes,
                      void *hip_stream, const dq_hooks *hooks);

/* Decompress into x_hat (N fp32). eb_abs is the absolute bound reported by
 * compress; p->eb and p->eb_mode are ignored. n_out entries of out_idx/out_val
 * are read. res->status becomes DQ_ECORRUPT if an outlier index is out of
 * range or out of block-major order, a zero code has no outlier, or an
 * outlier sits on a non-zero code; x_hat is then unspecified. */
dq_status dq_decompress(const dq_params *p, double eb_abs, const uint16_t *codes,
                        const uint32_t *out_idx, const int32_t *out_val, uint64_t n_out,
                        const int32_t *pads, float *x_hat, dq_result *res,
                        void *ws, uint64_t ws_bytes, void *hip_stream,
                        const dq_hooks *hooks);

/* Decompress the stream written by a dq_compress call enqueued earlier on the
 * same stream (or ordered before this one), taking the outlier count and the
 * absolute bound from that call's device-resident result cres instead of the
 * host: no synchronisation between the two calls, and both can be captured
 * in one HIP graph. out_cap is the capacity given to that compress call (the
 * outlier buffers hold that many entries). If cres->status is not DQ_OK,
 * res->status receives it and x_hat is not written. Otherwise as
 * dq_decompress; ws is needed whenever out_cap > 0. Enqueues one more
 * (one-thread) kernel that clears res's status word first, so that a replayed
 * graph reports each replay's own outcome. */
dq_status dq_decompress_dev(const dq_params *p, const dq_result *cres, uint64_t out_cap,
                            const uint16_t *codes, const uint32_t *out_idx, const int32_t *out_val,
                            const int32_t *pads, float *x_hat, dq_result *res, void *ws,
                            uint64_t ws_bytes, void *hip_stream, const dq_hooks *hooks);

/* Bytes of the fixed device scratch array that dq_compress_noalloc uses as
 * its workspace (one array per device, held until the process ends). */
#define DQ_SCRATCH_BYTES (64ull << 20)

/* dq_compress without a workspace argument and without any allocation: for
 * callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc). The workspace is a fixed
 * array of DQ_SCRATCH_BYTES in the library's code object, one per device;
 * the first call on a device (the current device, which must be the device
 * of hip_stream) looks up that device's copy once. Arguments, outputs and
 * errors as dq_compress, plus DQ_ENOSCRATCH (returned before anything is
 * enqueued) when dq_compress_workspace(p, out_cap) exceeds DQ_SCRATCH_BYTES:
 * about 32 bytes per outlier of capacity, 4 per block and 8 per tile, e.g. a
 * 256^3 field with 8^3 blocks fits with out_cap up to ~2 million. No hooks.
 * Every call on a device shares its array and leaves its contents behind
 * (the kernels initialise what they read, so nothing needs clearing): calls
 * that overlap in time on one device - on different streams or from
 * different host threads - race and corrupt each other's results. Calls
 * ordered on one stream are safe. */
dq_status dq_compress_noalloc(const dq_params *p, const float *x, uint16_t *codes,
                              uint32_t *out_idx, int32_t *out_val, uint64_t out_cap,
                              int32_t *pads, dq_result *res, void *hip_stream);

/* Copy a device dq_result to the host after waiting for hip_stream. */
dq_status dq_result_sync(const dq_result *res_dev, dq_result *res_host, void *hip_stream);

/* hipEvent helpers for dq_hooks (timing events, no allocation on the device). */
dq_status dq_event_create(void **ev);
dq_status dq_event_destroy(void *ev);
dq_status dq_event_elapsed_ms(void *ev_before, void *ev_after, float *ms);

/* Static description of a status code. */
const char *dq_strerror(int status);

#ifdef __cplusplus
}
#endif
#endif
